// Batches of instances, the multigrid hierarchy, the Krylov solvers and the
// backward-Euler time step (Section 2: P^{n+1} from Eq. 3, then T^{n+1}
// from Eq. 4 with the Darcy flux of P^{n+1}).
#include <cctype>
#include <cstdio>
#include <algorithm>
#include <chrono>
#include <cstring>
#include <functional>
#include <random>

#include "internal.h"
#include "krylov.h"
#include "solve.h"

#include <atomic>
#include <mutex>
#include <thread>

namespace hts {

hts_status guard_call(const std::function<void()> &f);

// ------------------------------------------------------------ helpers
template <typename T> struct Pick;
template <> struct Pick<double> {
    template <typename A, typename B> static double *get(A &a, B &) { return a.p; }
};
template <> struct Pick<float> {
    template <typename A, typename B> static float *get(A &, B &b) { return b.p; }
};
#define PK(T, a, b) Pick<T>::get((a), (b))

static void sync(hipStream_t s) { HTS_HIP(hipStreamSynchronize(s)); }

static double env_or(const char *name, double def)
{
    const char *v = getenv(name);
    return v ? atof(v) : def;
}

static void build_chunks(const std::vector<int64_t> &off, const std::vector<int64_t> &cnt, int len,
                         std::vector<Chunk> &ch, std::vector<int32_t> &segp)
{
    ch.clear(); segp.assign(1, 0);
    for (size_t i = 0; i < off.size(); i++) {
        for (int64_t b = 0; b < cnt[i]; b += len) {
            Chunk c{};
            c.inst = (int32_t)i;
            c.beg = off[i] + b;
            c.end = off[i] + std::min<int64_t>(cnt[i], b + len);
            ch.push_back(c);
        }
        segp.push_back((int32_t)ch.size());
    }
}

// ----------------------------------------------------------- batch build
Batch::~Batch()
{
    drop_graphs();
    if (cap) (void)hipStreamDestroy(cap);
    if (hS) (void)hipHostFree(hS);
    if (hact) (void)hipHostFree(hact);
    if (hexpS) (void)hipHostFree(hexpS);
    if (hseq) (void)hipHostFree(hseq);
}

void Batch::drop_graphs()
{
    for (auto &kv : graphs) {
        if (kv.second.e) (void)hipGraphExecDestroy(kv.second.e);
        if (kv.second.g) (void)hipGraphDestroy(kv.second.g);
    }
    graphs.clear();
}

// Run body's launches as one graph: captured on first use on a private
// stream (the caller's stream may be the legacy default stream, which
// cannot be captured), then replayed on the batch stream.
void Batch::replay(const std::string &key, const std::function<void()> &body)
{
    if (!cap) {
        HTS_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    }
    auto it = graphs.find(key);
    if (it == graphs.end()) {
        Graph G;
        hipStream_t saved = s;
        s = cap;
        HTS_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        try {
            body();
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(cap, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            s = saved;
            throw;
        }
        s = saved;
        HTS_HIP(hipStreamEndCapture(cap, &G.g));
        HTS_HIP(hipGraphInstantiate(&G.e, G.g, nullptr, nullptr, 0));
        it = graphs.emplace(key, G).first;
        static const bool verbose = env_or("HTS_VERBOSE", 0.0) > 2.0;
        if (verbose) std::fprintf(stderr, "[hts] captured graph %zu: %s\n", graphs.size(), key.c_str());
    }
    // replayed on the batch stream itself: ordered with the surrounding work
    // without a cross-stream event pair
    HTS_HIP(hipGraphLaunch(it->second.e, s));
}

// ----------------------------------------------------------- tuning cache
// z-chunk depth per (degree, field, node dims), filled by hts_autotune and
// optionally kept in the JSON file named by HTS_TUNE_CACHE.
namespace {
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

std::string tune_key(int degree, int field, int prec, int NX, int NY, int NZ)
{
    char b[96];
    snprintf(b, sizeof(b), "q%d_f%d_%s_%dx%dx%d", degree, field, prec ? "fp32" : "fp64", NX, NY, NZ);
    return b;
}

void tune_load()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = getenv("HTS_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char key[96];
    int v;
    // {"q1_f0_129x129x65": 8, ...}: skip the opening brace first
    int c0 = fgetc(f);
    while (c0 != EOF && isspace(c0)) c0 = fgetc(f);
    if (c0 != '{' && c0 != EOF) ungetc(c0, f);
    while (fscanf(f, " \"%95[^\"]\" : %d", key, &v) == 2) {
        g_tune[key] = v;
        int c = fgetc(f);
        while (c != EOF && c != ',' && c != '}') c = fgetc(f);
        if (c == '}' || c == EOF) break;
    }
    fclose(f);
}

void tune_save()
{
    const char *path = getenv("HTS_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "w");
    if (!f) return;
    fprintf(f, "{");
    bool first = true;
    for (auto &kv : g_tune) {
        fprintf(f, "%s\n  \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
        first = false;
    }
    fprintf(f, "\n}\n");
    fclose(f);
}
}  // namespace

void set_tuned_zc(int degree, int field, int prec, int NX, int NY, int NZ, int zc)
{
    tune_load();
    g_tune[tune_key(degree, field, prec, NX, NY, NZ)] = zc;
}

void save_tuning() { tune_save(); }

int tuned_zc(int degree, int field, int prec, int NX, int NY, int NZ)
{
    tune_load();
    auto it = g_tune.find(tune_key(degree, field, prec, NX, NY, NZ));
    return it == g_tune.end() ? 0 : it->second;
}

// Q1: wide tiles for the pressure operator, narrow ones for the heat operator
// (degree: the kernel family; general hexahedra use the narrow tiles)
int tile_own_x(int degree, int field) { return degree == 2 ? 30 : (field == 0 && degree == 1 ? 31 : 15); }
int tile_own_y(int degree, int field) { return degree == 2 ? 30 : 15; }

// work-list / tuning index of an operand type: 0 FP64, 1 FP32
template <typename T>
constexpr int prec_of() { return std::is_same<T, double>::value ? 0 : 1; }

int zc_for(const hts_mesh *M, int field, int prec, int64_t tiles, int force)
{
    const int NZ = M->N[2];
    // Q2 work items start on even node planes (cell-layer boundaries)
    auto fit = [&](int z) { return M->p == 2 ? std::max(2, (std::min(z, NZ) + 1) / 2 * 2) : std::min(z, NZ); };
    if (force > 0) return fit(force);
    const int t = tuned_zc(kernel_degree(M), field, prec, M->N[0], M->N[1], NZ);
    if (t > 0) return fit(t);
    // enough blocks to fill 256 CUs several times over
    int64_t z = std::max<int64_t>(4, (tiles * NZ) / 2048);
    z = std::min<int64_t>(z, 32);
    return fit((int)z);
}

int Batch::pick_zc(int field, int prec, const hts_mesh *M, int64_t tiles) const
{
    return zc_for(M, field, prec, tiles, zc_force[field][prec]);
}

void Batch::build_work()
{
    drop_graphs();
    for (int f = 0; f < 2; f++)
    for (int pr = 0; pr < 2; pr++) {
        std::vector<WorkItem> nat;
        for (int i = 0; i < n; i++) {
            hts_mesh *M = m[i];
            // owned node columns per tile along x and y
            const int ox = tile_own_x(kernel_degree(M), f), oy = tile_own_y(kernel_degree(M), f);
            const int tx = (M->N[0] + ox - 1) / ox, ty = (M->N[1] + oy - 1) / oy;
            const int zc = pick_zc(f, pr, M, (int64_t)tx * ty);
            for (int z0 = 0; z0 < M->N[2]; z0 += zc)
                for (int y = 0; y < ty; y++)
                    for (int x = 0; x < tx; x++) {
                        WorkItem w{};
                        w.inst = i; w.tx = x; w.ty = y; w.z0 = z0; w.z1 = std::min(M->N[2], z0 + zc);
                        w.slot = (int32_t)nat.size();
                        nat.push_back(w);
                    }
        }
        // XCD-aware order: block b is dispatched to XCD b % 8; give each XCD a
        // contiguous run of neighbouring tiles so halos stay in its L2.
        const int64_t T = (int64_t)nat.size(), per = (T + 7) / 8;
        hwork[f][pr].clear();
        for (int64_t b = 0; b < 8 * per; b++) {
            int64_t idx = (b % 8) * per + b / 8;
            if (idx < T) hwork[f][pr].push_back(nat[idx]);
        }
        nwork[f][pr] = (int)hwork[f][pr].size();
        work[f][pr].upload(al, hwork[f][pr], s);
        // a block writes its partial sum at the tile's natural index, so the
        // partials of an instance are contiguous and reduced in natural tile
        // order: a batched instance sums exactly like the same instance alone
        std::vector<int32_t> sp(n + 1, 0);
        for (const WorkItem &w : nat) sp[w.inst + 1]++;
        for (int i = 0; i < n; i++) sp[i + 1] += sp[i];
        wkp[f][pr].upload(al, sp, s);
        rwk[f][pr] = RedCtx{wkp[f][pr].p, n, n == 1 ? sp[1] : -1};
    }
    int64_t mw = nch;
    for (int f = 0; f < 2; f++)
        for (int pr = 0; pr < 2; pr++) mw = std::max<int64_t>(mw, nwork[f][pr]);
    partial.alloc(al, (size_t)mw * 64 + 64);
}

std::shared_ptr<Batch> build_batch(const std::vector<hts_mesh *> &ms)
{
    auto B = std::make_shared<Batch>();
    B->m = ms;
    B->n = (int)ms.size();
    B->p = ms[0]->p;
    B->s = ms[0]->stream;
    B->al = &ms[0]->alloc;
    B->device = ms[0]->desc.device;
    for (hts_mesh *M : ms) {
        if (M->p != B->p) throw Error(HTS_ERR_ARG, "all meshes of a batch must have the same degree");
        if (M->general != ms[0]->general)
            throw Error(HTS_ERR_ARG, "general hexahedral and box meshes cannot share a batch");
        if (M->desc.device != B->device) throw Error(HTS_ERR_ARG, "all meshes of a batch must share a device");
        prepare_mesh(M);
    }
    Alloc *al = B->al;
    hipStream_t s = B->s;
    const int n = B->n;
    std::vector<int64_t> cnt(n);
    B->off.resize(n);
    int64_t tot = 0;
    for (int i = 0; i < n; i++) {
        B->off[i] = tot;
        cnt[i] = ms[i]->nnode;
        tot += cnt[i];
    }
    B->ntot = tot;
    B->ctot = 0;
    for (int i = 0; i < n; i++) B->ctot += ms[i]->ncell;
    B->graded = false;
    for (int i = 0; i < n; i++) B->graded = B->graded || ms[i]->graded;
    B->general = ms[0]->general;
    std::vector<int32_t> sp;
    build_chunks(B->off, cnt, CHUNK_LEN, B->hch, sp);
    B->nch = (int)B->hch.size();
    B->ch.upload(al, B->hch, s);
    B->chp.upload(al, sp, s);
    B->rch = RedCtx{B->chp.p, n, n == 1 ? sp[1] : -1};
    B->build_work();

    B->S.alloc(al, (size_t)n * NSLOT);
    B->S.zero(s);
    B->active.alloc(al, n);
    B->nn_use.alloc(al, n);
    B->nn_mg.alloc(al, n);
    B->act_save.alloc(al, n);
    HTS_HIP(hipHostMalloc((void **)&B->hS, sizeof(double) * n * NSLOT, hipHostMallocDefault));
    HTS_HIP(hipHostMalloc((void **)&B->hact, sizeof(int32_t) * n, hipHostMallocCoherent));
    HTS_HIP(hipHostMalloc((void **)&B->hexpS, sizeof(double) * n * NSLOT, hipHostMallocCoherent));
    HTS_HIP(hipHostMalloc((void **)&B->hseq, sizeof(uint32_t) * 64, hipHostMallocCoherent));
    *B->hseq = 0;
    std::memset(B->hS, 0, sizeof(double) * n * NSLOT);
    B->redout.alloc(al, (size_t)n * 64);
    B->redout2.alloc(al, (size_t)n * 64);
    B->redout3.alloc(al, (size_t)n * 64);

    B->alias_state = n == 1;
    if (B->alias_state) {
        // views of the mesh's buffers (no allocator: not released here)
        hts_mesh *M = ms[0];
        DBuf<double> *views[6] = {&B->Pn, &B->Tn, &B->Pp, &B->Tp, &B->Ppp, &B->Tpp};
        double *bufs[6] = {M->P.p, M->T.p, M->Pprev.p, M->Tprev.p, M->Pprev2.p, M->Tprev2.p};
        for (int k = 0; k < 6; k++) {
            views[k]->p = bufs[k];
            views[k]->n = (size_t)tot;
            views[k]->al = nullptr;
        }
    } else {
        for (DBuf<double> *v : {&B->Pn, &B->Tn, &B->Pp, &B->Tp, &B->Ppp, &B->Tpp}) {
            v->alloc(al, tot);
            v->zero(s);
        }
    }
    for (DBuf<double> *v : {&B->P1, &B->T1, &B->g, &B->b, &B->x, &B->r, &B->z,
                            &B->pp, &B->q, &B->rold, &B->y, &B->ld0, &B->ld1, &B->inner_b, &B->inner_x}) {
        v->alloc(al, tot);
        v->zero(s);
    }
    for (DBuf<float> *v : {&B->P32, &B->b32, &B->x32, &B->r32, &B->z32, &B->p32, &B->q32, &B->rold32, &B->y32}) {
        v->alloc(al, tot);
        v->zero(s);
    }
    // boundary tables, sources, line coefficients, static loads
    for (int f = 0; f < 2; f++) {
        std::vector<BcDev> bc(n);
        std::vector<int64_t> rows;
        std::vector<int32_t> rowptr(1, 0);
        std::vector<SrcEnt> ents;
        std::vector<SrcDev> srcs;
        for (int i = 0; i < n; i++) {
            hts_mesh *M = ms[i];
            BcDev &b = bc[i];
            std::memset(&b, 0, sizeof(b));
            for (const FaceSpec &fs : M->bcs[f])
                if (fs.kind == HTS_BC_DIRICHLET && b.nface < 6) {
                    b.faces[b.nface] = fs.face;
                    b.ftf[b.nface] = to_dev(fs.tf);
                    b.nface++;
                }
            b.x0 = M->x0[0]; b.y0 = M->x0[1]; b.z0 = M->x0[2];
            b.dx = M->L[0] / (M->p * M->n[0]);
            b.dy = M->L[1] / (M->p * M->n[1]);
            b.dz = M->L[2] / (M->p * M->n[2]);
            b.xyz = M->general ? M->xyz.p : nullptr;
            b.xn = M->graded ? M->dnode[0].p : nullptr;
            b.yn = M->graded ? M->dnode[1].p : nullptr;
            b.zn = M->graded ? M->dnode[2].p : nullptr;
            b.colspec = M->colspec[f].p;
            b.coltf = M->coltf[f].p;
            const SrcRows &R = M->src[f];
            const int sbase = (int)srcs.size();
            for (SrcDev sd : R.srcs) {
                sd.inst = i;
                srcs.push_back(sd);
            }
            for (size_t r = 0; r < R.rows.size(); r++) {
                rows.push_back(B->off[i] + R.rows[r]);
                for (int e = R.rowptr[r]; e < R.rowptr[r + 1]; e++) {
                    SrcEnt se = R.ents[e];
                    se.src += sbase;
                    ents.push_back(se);
                }
                rowptr.push_back((int32_t)ents.size());
            }
        }
        B->bc[f].upload(al, bc, s);
        B->nsrows[f] = (int64_t)rows.size();
        B->srows[f].upload(al, rows, s);
        B->srowptr[f].upload(al, rowptr, s);
        B->sents[f].upload(al, ents, s);
        B->ssrc[f].upload(al, srcs, s);
    }
    {
        std::vector<SrcDev> ls;
        B->lbase.assign(n, 0);
        for (int i = 0; i < n; i++) {
            B->lbase[i] = (int)ls.size();
            for (SrcDev sd : ms[i]->line_srcs) {
                sd.inst = i;
                ls.push_back(sd);
            }
        }
        B->nlsrc = (int)ls.size();
        B->lsrc.upload(al, ls, s);
        B->lcoef.alloc(al, std::max(1, B->nlsrc));
        B->lcoef.zero(s);
    }
    for (int i = 0; i < n; i++) {
        HTS_HIP(hipMemcpyAsync(B->ld0.p + B->off[i], ms[i]->load[0].p, cnt[i] * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
        HTS_HIP(hipMemcpyAsync(B->ld1.p + B->off[i], ms[i]->load[1].p, cnt[i] * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
    }
    B->make_tables(B->massP, 0, 1.0, false, true);
    B->make_tables(B->massH, 1, 1.0, false, true);
    sync(s);
    return B;
}

void Batch::make_tables(Tables &t, int field, double dt, bool steady, bool mass_only)
{
    t.h64.resize(n);
    t.h32.resize(n);
    for (int i = 0; i < n; i++) {
        for (int prec = 0; prec < 2; prec++) {
            OpDev o = make_op(m[i], field, prec == 1, dt, steady, mass_only);
            o.off = off[i];
            if (field == 1) {
                o.P = prec ? (const void *)(P32.p + off[i]) : (const void *)(P1.p + off[i]);
                o.lcoef = lcoef.p + lbase[i];
                if (prec) o.rho_g = 0.0;   // P32 holds the piezometric pressure
            }
            (prec ? t.h32 : t.h64)[i] = o;
        }
    }
    t.d64.upload(al, t.h64, s);
    t.d32.upload(al, t.h32, s);
    t.field = field;
}

void Batch::upload_S() { HTS_HIP(hipMemcpyAsync(S.p, hS, sizeof(double) * n * NSLOT, hipMemcpyHostToDevice, s)); }
// Host reads of the scalar slots and flags: one small kernel writes both into
// coherent pinned memory (no copy engine round trip), then the stream is
// synchronised; the slots are copied into hS, which the host may edit.
void Batch::export_state()
{
    const uint32_t want = ++exp_seq;
    vexport(S.p, n * NSLOT, active.p, n, hexpS, hact, hseq, want, s);
    // Spin on the sequence number the kernel writes last (a stream wait
    // costs a much longer wake-up); every so often ask the runtime whether
    // the stream has finished or failed, so a launch error cannot hang here.
    const volatile uint32_t *seq = hseq;
    for (uint64_t k = 1;; k++) {
        if (*seq == want) break;
        if ((k & 255) == 0) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                if (*seq == want) break;
                throw Error(HTS_ERR_HIP, "state export finished without its sequence number");
            }
            if (e != hipErrorNotReady) HTS_HIP(e);
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
}
void Batch::download_S()
{
    export_state();
    slots_from_export();
}
void Batch::slots_from_export() { std::memcpy(hS, hexpS, sizeof(double) * n * NSLOT); }
void Batch::set_active(const std::vector<int32_t> &a) { vset_flags(a.data(), n, active.p, s); }
std::vector<int32_t> Batch::get_active()
{
    export_state();
    return std::vector<int32_t>(hact, hact + n);
}
bool Batch::any_active()
{
    auto a = get_active();
    for (int v : a)
        if (v) return true;
    return false;
}
VecCtx Batch::vctx(bool use_active) const { return VecCtx{ch.p, nch, use_active ? active.p : nullptr, S.p, s}; }

// --------------------------------------------------------- level operators
// ------------------------------------------------------ kernel timing
namespace {
struct TimingRec {
    hipEvent_t a, b;
    int field, prec;
    double bytes, flops;
};
struct TimingState {
    bool on = false;
    std::vector<TimingRec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        HTS_HIP(hipEventCreate(&e));
        return e;
    }
};
TimingState g_timing;
}  // namespace

// Algorithmic traffic of one fine-level launch: each node vector the
// epilogue touches once, the per-cell coefficients, and (heat) the pressure.
static double apply_bytes(int field, int epi, int64_t nodes, int64_t cells, int ts)
{
    int nvec = 2;   // x read, y written
    if (epi == EPI_RESID || epi == EPI_RESID_NORM) nvec = 3;
    if (epi == EPI_CHEB) nvec = 6;   // x, b, d (read + write), D^-1, x_out
    if (epi == EPI_CHEB0) nvec = 4;  // b, D^-1, d and x_out written
    const int ncoef = field == 0 ? 1 : 3;
    const int extra = field == 0 ? 0 : 1;
    return (double)ts * ((double)nodes * (nvec + extra) + (double)cells * ncoef);
}
static double apply_flops(int field, int p, int64_t cells)
{
    // per cell: Kronecker mass + stiffness about 150 flop (Q1), the
    // convection term about 270 more; Q2 about 8x the Q1 count
    const double q1 = field == 0 ? 150.0 : 420.0;
    return (p == 1 ? q1 : 8.0 * q1) * (double)cells;
}

template <typename T>
void Batch::fine_apply(int field, const OpDev *ops, int epi, bool masked, const T *x, T *y, const EpiArgs<T> &ep)
{
    constexpr int pr = std::is_same<T, double>::value ? 0 : 1;
    if (!g_timing.on) {
        launch_apply<T>(general ? DEGREE_HEX : p, field, epi, masked, graded, ops, work[field][pr].p,
                        nwork[field][pr], x, y, ep, s);
        return;
    }
    TimingRec r{};
    r.a = g_timing.get();
    r.b = g_timing.get();
    r.field = field;
    r.prec = std::is_same<T, double>::value ? 0 : 1;
    r.bytes = apply_bytes(field, epi, ntot, ctot, sizeof(T));
    r.flops = apply_flops(field, p, ctot);
    HTS_HIP(hipEventRecord(r.a, s));
    launch_apply<T>(general ? DEGREE_HEX : p, field, epi, masked, graded, ops, work[field][pr].p, nwork[field][pr], x,
                    y, ep, s);
    HTS_HIP(hipEventRecord(r.b, s));
    g_timing.recs.push_back(r);
}

template <typename T>
void Batch::apply_lvl(Hier &H, int l, int epi, bool masked, const T *x, T *y, EpiArgs<T> ep)
{
    if (!ep.active) ep.active = active.p;
    if (l == 0) {
        const OpDev *ops = std::is_same<T, double>::value ? H.ops.d64.p : H.ops.d32.p;
        fine_apply<T>(H.field, ops, epi, masked, x, y, ep);
    } else {
        Level &L = H.lev[l];
        const LevelDev *g = std::is_same<T, double>::value ? L.g64.p : L.g32.p;
        launch_stencil<T>(epi, g, L.ch_ext, L.nch, ep.active, x, y, ep, s);
    }
}

template <typename T>
void Batch::apply_op(const Tables &t, int epi, bool masked, const T *x, T *y, EpiArgs<T> ep)
{
    if (!ep.active) ep.active = active.p;
    const OpDev *ops = std::is_same<T, double>::value ? t.d64.p : t.d32.p;
    fine_apply<T>(t.field, ops, epi, masked, x, y, ep);
}

// ---------------------------------------------------------- hierarchy
static void invert_dense(std::vector<double> &A, int n)
{
    // Gauss-Jordan with partial pivoting, in place
    std::vector<int> piv(n);
    for (int i = 0; i < n; i++) piv[i] = i;
    std::vector<double> I((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++) I[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; c++) {
        int pr = c;
        double best = std::fabs(A[(size_t)c * n + c]);
        for (int r = c + 1; r < n; r++)
            if (std::fabs(A[(size_t)r * n + c]) > best) { best = std::fabs(A[(size_t)r * n + c]); pr = r; }
        if (best == 0.0) throw Error(HTS_ERR_BREAKDOWN, "singular coarse-grid operator");
        if (pr != c)
            for (int k = 0; k < n; k++) {
                std::swap(A[(size_t)c * n + k], A[(size_t)pr * n + k]);
                std::swap(I[(size_t)c * n + k], I[(size_t)pr * n + k]);
            }
        const double inv = 1.0 / A[(size_t)c * n + c];
        for (int k = 0; k < n; k++) {
            A[(size_t)c * n + k] *= inv;
            I[(size_t)c * n + k] *= inv;
        }
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            const double f = A[(size_t)r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; k++) {
                A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
                I[(size_t)r * n + k] -= f * I[(size_t)c * n + k];
            }
        }
    }
    A.swap(I);
}

// Inverse of a symmetric positive definite 27-point operator in lexicographic
// order (bandwidth bw = NX NY + NX + 1) from its banded Cholesky factor:
// A = L L^T costs n bw^2 / 2, then column j of A^-1 is L^-T L^-1 e_j, the
// columns split over host threads.  Returns false (A untouched) when a pivot
// is not positive, i.e. the operator is not SPD.
static bool invert_spd_banded(std::vector<double> &A, int n, int bw)
{
    bw = std::min(bw, n - 1);
    const size_t W = (size_t)bw + 1;
    std::vector<double> L((size_t)n * W, 0.0);   // L[i][j] at L[i*W + (i - j)], i - bw <= j <= i
    auto l = [&](int i, int j) -> double & { return L[(size_t)i * W + (size_t)(i - j)]; };
    for (int i = 0; i < n; i++) {
        const int j0 = std::max(0, i - bw);
        for (int j = j0; j <= i; j++) {
            double s = A[(size_t)i * n + j];
            for (int k = std::max(j0, j - bw); k < j; k++) s -= l(i, k) * l(j, k);
            if (j == i) {
                if (!(s > 0.0)) return false;
                l(i, i) = std::sqrt(s);
            } else {
                l(i, j) = s / l(j, j);
            }
        }
    }
    const int nt = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
    std::atomic<int> next(0);
    auto work = [&]() {
        std::vector<double> y(n);
        for (int j; (j = next.fetch_add(1)) < n;) {
            for (int i = 0; i < j; i++) y[i] = 0.0;
            for (int i = j; i < n; i++) {
                double s = i == j ? 1.0 : 0.0;
                for (int k = std::max(j, i - bw); k < i; k++) s -= l(i, k) * y[k];
                y[i] = s / l(i, i);
            }
            for (int i = n - 1; i >= 0; i--) {
                double s = y[i];
                const int k1 = std::min(n - 1, i + bw);
                for (int k = i + 1; k <= k1; k++) s -= l(k, i) * y[k];
                y[i] = s / l(i, i);
            }
            // A^-1 is symmetric: column j is row j
            std::copy(y.begin(), y.end(), A.begin() + (size_t)j * n);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; t++) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
    return true;
}

// Chebyshev iteration for a spectrum of D^-1 A inside the ellipse with
// centre theta on the real axis, real semi-axis delta and imaginary
// semi-axis beta (beta = 0: the interval [lmin, lmax]).  Its foci are
// theta +- c with c^2 = delta^2 - beta^2, real or imaginary; with
// mu_k = rho_k / c the recurrence needs c^2 only and stays real:
//   d_0 = D^-1 r_0 / theta,  mu_0 = 1 / theta,
//   mu_k = 1 / (2 theta - c^2 mu_{k-1}),
//   d_k = c^2 mu_k mu_{k-1} d_{k-1} + 2 mu_k D^-1 r_k,  x_{k+1} = x_k + d_k.
// out[2k], out[2k+1] are the two factors of step k (out[0] = 0).
static void cheb_coeffs(double lmax_est, double ratio, int steps, double beta_est, double *out /* 2*steps */)
{
    static const double safety = env_or("HTS_LMAX_SAFETY", 1.1);
    const double lmax = safety * lmax_est, lmin = lmax / ratio;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), beta = safety * beta_est;
    const double c2 = delta * delta - beta * beta;
    double mu_prev = 1.0 / theta;
    out[0] = 0.0;
    out[1] = mu_prev;
    for (int k = 1; k < steps; k++) {
        const double mu = 1.0 / (2.0 * theta - c2 * mu_prev);
        out[2 * k] = c2 * mu * mu_prev;
        out[2 * k + 1] = 2.0 * mu;
        mu_prev = mu;
    }
}

void Batch::estimate_lmax(Hier &H, int l, std::vector<double> &lmax)
{
    Level &L = H.lev[l];
    lmax.assign(n, 1.0);
    if (L.nch == 0) return;
    // probe vector: the same per instance whatever batch it sits in
    std::vector<double> hv(std::max<int64_t>(L.ntot, 1), 0.0);
    for (int i = 0; i < n; i++) {
        if (!L.cont[i]) continue;
        std::mt19937_64 rng(12345 + l);
        std::uniform_real_distribution<double> U(-1.0, 1.0);
        const int64_t b0 = L.h64[i].off, cnt = L.h64[i].n;
        for (int64_t e = 0; e < cnt; e++) hv[b0 + e] = U(rng);
    }
    HTS_HIP(hipMemcpyAsync(L.x64.p, hv.data(), L.ntot * sizeof(double), hipMemcpyHostToDevice, s));
    std::vector<int32_t> act(n, 0);
    for (int i = 0; i < n; i++) act[i] = L.cont[i] ? 1 : 0;
    set_active(act);
    VecCtx v{L.ch_ext, L.nch, active.p, S.p, s};
    RedCtx rc = L.red;
    if (l == 0) vmask<double>(v, H.ops.d64.p, L.x64.p, 0.0);
    EpiArgs<double> ep{};
    const int iters = (int)env_or("HTS_LMAX_ITERS", 12.0);
    for (int it = 0; it < iters; it++) {
        apply_lvl<double>(H, l, EPI_STORE, true, L.x64.p, L.t64.p, ep);
        vjacobi<double>(v, 1.0, -1, L.invd64.p, L.t64.p, L.xb64.p);
        vdot<double>(v, L.xb64.p, L.xb64.p, nullptr, partial.p);
        vreduce(rc, partial.p, 2, RED_INVSQRT, S_TMP0, S.p, active.p, 0, 0.0, nullptr, s);
        vaxpby<double>(v, 1.0, S_TMP1, L.xb64.p, 0.0, -1, L.x64.p);
    }
    download_S();
    for (int i = 0; i < n; i++)
        if (L.cont[i]) lmax[i] = std::sqrt(std::max(hS[(size_t)i * NSLOT + S_TMP0], 1e-300));
}

static void level_alloc(Level &L, Alloc *al, hipStream_t s, int64_t ntot)
{
    L.ntot = ntot;
    const int64_t m = std::max<int64_t>(ntot, 1);
    for (DBuf<double> *v : {&L.x64, &L.xb64, &L.b64, &L.d64, &L.t64, &L.invd64}) { v->alloc(al, m); v->zero(s); }
    for (DBuf<float> *v : {&L.x32, &L.xb32, &L.b32, &L.d32, &L.t32, &L.invd32}) { v->alloc(al, m); v->zero(s); }
}

void Batch::build_smoother(Hier &H, int l, int steps, double ratio, const std::vector<double> *given,
                           const std::vector<double> *beta, const std::vector<int> *steps_i)
{
    Level &L = H.lev[l];
    std::vector<double> lm;
    if (given) lm = *given;
    else estimate_lmax(H, l, lm);
    std::vector<double> c((size_t)n * NSLOT, 0.0);
    static const bool verbose = env_or("HTS_VERBOSE", 0.0) > 0.0;
    for (int i = 0; i < n; i++) {
        double *ci = &c[(size_t)i * NSLOT + S_CHEB];
        cheb_coeffs(lm[i], ratio, steps, beta ? (*beta)[i] : 0.0, ci);
        // an instance of lower degree: its later steps add nothing (d_k = 0)
        if (steps_i)
            for (int k = std::max(1, (*steps_i)[i]); k < steps; k++) ci[2 * k] = ci[2 * k + 1] = 0.0;
        if (L.cont[i]) H.lmax.push_back(lm[i]);
        if (verbose && L.cont[i])
            std::fprintf(stderr, "[hts] field %d level %d instance %d lmax(D^-1 A) %.6g ratio %g steps %d\n", H.field, l,
                         i, lm[i], ratio, steps);
    }
    L.cheb.upload(al, c, s);
}

Hier &Batch::pressure_hier(bool steady, double dt, const hts_solver_opts &o)
{
    const int deg = std::max(1, std::min(o.cheb_degree, 8));
    auto key = std::make_tuple(steady ? 1 : 0, steady ? 0.0 : dt, deg, o.mg_coarse_max);
    auto it = hier.find(key);
    if (it != hier.end()) {
        hier_used[key] = ++hier_clock;
        return *it->second;
    }
    // keep at most two (typically the steady one of the initial state and
    // the transient one of the time step): a new time-step size replaces
    // the least recently used, with the graphs captured on it
    if (hier.size() >= 2) {
        auto lru = hier_used.begin();
        for (auto u = hier_used.begin(); u != hier_used.end(); ++u)
            if (u->second < lru->second) lru = u;
        drop_graphs();
        hier.erase(lru->first);
        hier_used.erase(lru);
    }
    auto H = std::make_unique<Hier>();
    H->field = 0;
    H->deg = deg;
    H->ratio = env_or("HTS_P_RATIO", 15.0);
    H->ratio_coarse = env_or("HTS_P_RATIO", 15.0);
    make_tables(H->ops, 0, dt, steady, false);
    build_hierarchy(*H, o);
    Hier &ref = *H;
    hier[key] = std::move(H);
    hier_used[key] = ++hier_clock;
    return ref;
}

// Separable heat preconditioner tables (Q1): nodal S = cbar_T^-1/2 and the
// Thomas factors of each axis's 1D matrix B = M + alpha K, per cell
// h [1/3 1/6; 1/6 1/3] + (alpha / h) [1 -1; -1 1], alpha = dt median(lambda /
// c_T) of the instance, with identity end rows where that face is Dirichlet.
void Batch::build_tmass(Hier &H, double dt)
{
    H.tensor = true;
    std::vector<double> sv((size_t)ntot);
    std::vector<TMassInst> h64(n), h32(n);
    std::vector<int64_t> lb[3];
    for (int a = 0; a < 3; a++) lb[a].assign(n + 1, 0);
    H.tfac.clear();
    H.tfac.reserve(3 * n);
    for (int i = 0; i < n; i++) {
        hts_mesh *M = m[i];
        const int NX = M->N[0], NY = M->N[1], NZ = M->N[2];
        for (int k = 0; k < NZ; k++)
            for (int j = 0; j < NY; j++)
                for (int x = 0; x < NX; x++) {
                    double acc = 0.0;
                    int cnt = 0;
                    for (int dz = -1; dz <= 0; dz++)
                        for (int dy = -1; dy <= 0; dy++)
                            for (int dx = -1; dx <= 0; dx++) {
                                const int cx = x + dx, cy = j + dy, cz = k + dz;
                                if (cx < 0 || cx >= M->n[0] || cy < 0 || cy >= M->n[1] || cz < 0 || cz >= M->n[2])
                                    continue;
                                acc += M->hcT[(size_t)cx + (size_t)M->n[0] * (cy + (size_t)M->n[1] * cz)];
                                cnt++;
                            }
                    sv[(size_t)off[i] + x + (size_t)NX * (j + (size_t)NY * k)] = 1.0 / std::sqrt(acc / cnt);
                }
        TMassInst t{};
        t.N[0] = NX; t.N[1] = NY; t.N[2] = NZ;
        t.off = off[i];
        const int dm = M->dmask[1];
        std::vector<double> ratio(M->hcT.size());
        for (size_t c = 0; c < ratio.size(); c++) ratio[c] = M->hlam[c] / M->hcT[c];
        std::nth_element(ratio.begin(), ratio.begin() + ratio.size() / 2, ratio.end());
        const double alpha = dt * ratio[ratio.size() / 2];
        for (int a = 0; a < 3; a++) {
            const int nn = M->N[a];
            const bool dlo = (dm >> (2 * a)) & 1, dhi = (dm >> (2 * a + 1)) & 1;
            std::vector<double> A(nn, 0.0), B(nn, 0.0), Cc(nn, 0.0);
            for (int e = 0; e + 1 < nn; e++) {   // cell [e, e+1]
                const double h = M->cell_h(a, e);
                B[e] += h / 3.0 + alpha / h;
                B[e + 1] += h / 3.0 + alpha / h;
                Cc[e] += h / 6.0 - alpha / h;
                A[e + 1] += h / 6.0 - alpha / h;
            }
            auto ident = [&](int e) {
                A[e] = 0.0; B[e] = 1.0; Cc[e] = 0.0;
                if (e > 0) Cc[e - 1] = 0.0;
                if (e < nn - 1) A[e + 1] = 0.0;
            };
            if (dlo) ident(0);
            if (dhi) ident(nn - 1);
            std::vector<double> f(3 * (size_t)nn);
            double cprev = 0.0;
            for (int e = 0; e < nn; e++) {
                const double piv = B[e] - A[e] * cprev;
                const double inv = 1.0 / piv;
                const double cp = Cc[e] * inv;
                f[e] = A[e];
                f[nn + e] = inv;
                f[2 * nn + e] = cp;
                cprev = cp;
            }
            H.tfac.emplace_back();
            H.tfac.back().upload(al, f, s);
            t.fac[a] = H.tfac.back().p;
        }
        h64[i] = t;
        h32[i] = t;
    }
    // lines per wavefront (staged in at most 64 KB of LDS in FP64) and the
    // first block of every instance along each axis
    for (int a = 0; a < 3; a++) {
        int nmax = 1;
        for (int i = 0; i < n; i++) nmax = std::max(nmax, m[i]->N[a]);
        const int ld = nmax | 1;
        H.tlb[a] = std::max(1, std::min(64, 65536 / (ld * 8)));
        H.tlds64[a] = H.tlb[a] * ld * 8;
        H.tlds32[a] = H.tlb[a] * ld * 4;
        for (int i = 0; i < n; i++) {
            const int NX = m[i]->N[0], NY = m[i]->N[1], NZ = m[i]->N[2];
            const int64_t lines = a == 0 ? (int64_t)NY * NZ : (a == 1 ? (int64_t)NX * NZ : (int64_t)NX * NY);
            lb[a][i + 1] = lb[a][i] + (lines + H.tlb[a] - 1) / H.tlb[a];
        }
    }
    H.ts64.upload(al, sv, s);
    std::vector<float> sf(sv.begin(), sv.end());
    H.ts32.upload(al, sf, s);
    for (int i = 0; i < n; i++) {
        h64[i].s = H.ts64.p;
        h32[i].s = H.ts32.p;
    }
    H.tm64.upload(al, h64, s);
    H.tm32.upload(al, h32, s);
    for (int a = 0; a < 3; a++) {
        H.tl[a].upload(al, lb[a], s);
        H.tn[a] = lb[a][n];
    }
}

template <typename T>
void Batch::tmass_prec(Hier &H, const T *b, T *x)
{
    const int64_t *lb[3] = {H.tl[0].p, H.tl[1].p, H.tl[2].p};
    const bool d = std::is_same<T, double>::value;
    const OpDev *ops = d ? H.ops.d64.p : H.ops.d32.p;
    launch_tmass<T>(d ? H.tm64.p : H.tm32.p, n, lb, H.tn, H.tlb, d ? H.tlds64 : H.tlds32, active.p, ops, b, x, s);
}

Hier &Batch::heat_prec(double dt, const hts_solver_opts &o)
{
    const bool mg = o.heat_precond == 0;
    const bool tensor = o.heat_precond == 2 && p == 1;
    // degree 0: automatic, 4 on degree-1 cells, 2 on degree-2 cells (a Q2
    // apply costs about eight times the flops of a Q1 apply per node, so
    // fewer products per Krylov iteration pay there)
    const int dreq = o.heat_cheb_degree > 0 ? o.heat_cheb_degree : (p == 2 ? 2 : 4);
    const int deg = mg ? std::max(1, std::min(dreq, 8)) : std::max(1, std::min(dreq, 16));
    if (heat && heat->dt == dt && heat->deg_req == deg && heat->multigrid == mg && heat->tensor == tensor)
        return *heat;
    drop_graphs();
    heat = std::make_unique<Hier>();
    Hier &H = *heat;
    H.field = 1;
    H.dt = dt;
    H.deg = deg;
    H.deg_req = deg;
    H.multigrid = mg;
    if (tensor) {
        make_tables(H.ops, 1, dt, false, false);
        build_tmass(H, dt);
        return H;
    }
    // Chebyshev-Jacobi on [lmax/15, 1.1 lmax], alone or as a multigrid
    // smoother (alone, degree 2, on the 128x128x64 layered aquifer: ratio 8:
    // 10.9 FGMRES iterations, 15: 10.6, 20: 12.0, 30: 12.4, 60: 15.8)
    H.ratio = env_or("HTS_HEAT_RATIO", 15.0);
    H.ratio_coarse = env_or("HTS_HEAT_RATIO_COARSE", 15.0);
    make_tables(H.ops, 1, dt, false, false);
    // The Chebyshev intervals are estimated on the symmetric part (mass,
    // conduction, injection line) wherever convection does not widen the
    // spectrum much: they then depend on the mesh, the coefficients and dt
    // only, not on the Darcy flux of the step in which the preconditioner
    // happens to be built, so a run resumed from a saved state applies the
    // same preconditioner as the uninterrupted one (convection-dominated
    // instances take the full operator's estimate, below).
    auto advection = [&](bool on) {
        for (int i = 0; i < n; i++) {
            H.ops.h64[i].cadv = on ? cadv_save[i] : 0.0;
            H.ops.h32[i].cadv = on ? cadv_save[i] : 0.0;
        }
        H.ops.d64.upload(al, H.ops.h64, s);
        H.ops.d32.upload(al, H.ops.h32, s);
    };
    cadv_save.resize(n);
    for (int i = 0; i < n; i++) cadv_save[i] = H.ops.h64[i].cadv;
    if (mg) {
        // Galerkin levels of the static symmetric part; the fine level
        // smooths with the full operator (current Darcy flux in P1)
        advection(false);
        build_hierarchy(H, o);
        advection(true);
        return H;
    }
    H.lev.resize(1);
    Level &L = H.lev[0];
    level_alloc(L, al, s, ntot);
    L.nch = L.nch_all = nch;
    L.red = rch;
    L.ch_ext = L.ch_all_ext = ch.p;
    L.present.assign(n, 1);
    L.cont.assign(n, 1);
    L.h64.resize(n);
    for (int i = 0; i < n; i++) {
        L.h64[i].NX = m[i]->N[0]; L.h64[i].NY = m[i]->N[1]; L.h64[i].NZ = m[i]->N[2];
        L.h64[i].off = off[i]; L.h64[i].n = m[i]->nnode; L.h64[i].S = nullptr;
    }
    for (int i = 0; i < n; i++) launch_inv_diag(H.ops.h64[i], L.invd64.p + off[i], s);
    convert_plain(ntot, L.invd64.p, L.invd32.p, s);
    // Where the Darcy flux does not move the largest eigenvalue of D^-1 A by
    // more than 25 % (conduction-dominated transport), the interval comes
    // from the symmetric part alone, so that it does not depend on the step
    // in which the preconditioner is built.  Where it does (convection-
    // dominated, e.g. next to an injection well), the convection term's
    // imaginary spectrum makes the symmetric interval far too narrow and
    // the preconditioned iteration stagnates: the full operator's estimate
    // (with the flux of the build step) is used instead.
    std::vector<double> lsym(n, 1.0), lfull(n, 1.0), lm(n);
    bool cached = true;
    for (int i = 0; i < n; i++) cached = cached && m[i]->heat_spec[0] == dt;
    if (!cached) {
        advection(false);
        estimate_lmax(H, 0, lsym);
        advection(true);
        estimate_lmax(H, 0, lfull);
    }
    static const bool verbose = env_or("HTS_VERBOSE", 0.0) > 0.0;
    // Imaginary extent of the spectrum: the convection part C = A - A_0 (A_0
    // the operator without the Darcy flux term) is close to skew, so D^-1 C
    // has nearly imaginary eigenvalues +-i beta.  beta^2 comes from power
    // iteration on (D^-1 C)^2 with the interval estimates' probe; the
    // Chebyshev polynomial is then the one of the ellipse over the real
    // interval with that imaginary semi-axis (a real-interval polynomial of
    // degree 3 or more grows on the imaginary part and can stall FGMRES).
    std::vector<double> beta(n, 0.0);
    if (!cached) {
        Tables T0;
        make_tables(T0, 1, dt, false, false);
        for (int i = 0; i < n; i++) T0.h64[i].cadv = T0.h32[i].cadv = 0.0;
        T0.d64.upload(al, T0.h64, s);
        T0.d32.upload(al, T0.h32, s);
        std::vector<double> hv(std::max<int64_t>(L.ntot, 1), 0.0);
        for (int i = 0; i < n; i++) {
            std::mt19937_64 rng(12345);
            std::uniform_real_distribution<double> U(-1.0, 1.0);
            const int64_t b0 = L.h64[i].off, cnt = L.h64[i].n;
            for (int64_t e = 0; e < cnt; e++) hv[b0 + e] = U(rng);
        }
        HTS_HIP(hipMemcpyAsync(L.x64.p, hv.data(), L.ntot * sizeof(double), hipMemcpyHostToDevice, s));
        std::vector<int32_t> all(n, 1);
        set_active(all);
        VecCtx v{L.ch_ext, L.nch, active.p, S.p, s};
        vmask<double>(v, H.ops.d64.p, L.x64.p, 0.0);
        EpiArgs<double> ep{};
        // w = D^-1 C x into dst (t, u: scratch)
        auto dinv_c = [&](const double *x, double *dst) {
            apply_op<double>(H.ops, EPI_STORE, true, x, L.t64.p, ep);
            apply_op<double>(T0, EPI_STORE, true, x, L.b64.p, ep);
            vaxpby<double>(v, -1.0, -1, L.b64.p, 1.0, -1, L.t64.p);
            vjacobi<double>(v, 1.0, -1, L.invd64.p, L.t64.p, dst);
        };
        const int iters = (int)env_or("HTS_LMAX_ITERS", 12.0);
        for (int it = 0; it < iters; it++) {
            dinv_c(L.x64.p, L.xb64.p);
            dinv_c(L.xb64.p, L.d64.p);
            vdot<double>(v, L.d64.p, L.d64.p, nullptr, partial.p);
            vreduce(rch, partial.p, 2, RED_INVSQRT, S_TMP0, S.p, active.p, 0, 0.0, nullptr, s);
            vaxpby<double>(v, 1.0, S_TMP1, L.d64.p, 0.0, -1, L.x64.p);
        }
        download_S();
        for (int i = 0; i < n; i++) beta[i] = std::pow(std::max(hS[(size_t)i * NSLOT + S_TMP0], 0.0), 0.25);
    }
    // a mesh that already holds estimates for this dt keeps them (a run
    // resumed with them builds the same preconditioner as the run that made
    // them); the others record the new ones
    for (int i = 0; i < n; i++) {
        double *hs = m[i]->heat_spec;
        if (hs[0] == dt) {
            lsym[i] = hs[1];
            lfull[i] = hs[2];
            beta[i] = hs[3];
        } else {
            hs[0] = dt;
            hs[1] = lsym[i];
            hs[2] = lfull[i];
            hs[3] = beta[i];
        }
    }
    // Where the imaginary extent reaches the real half-width of the interval
    // (convection-dominated), the ellipse reaches nearly to the origin
    // relative to its size and higher polynomial degrees no longer pay (the
    // injection column stalls at degree 4): such instances keep degree 2,
    // their later steps add nothing.
    static const double safety = env_or("HTS_LMAX_SAFETY", 1.1);
    std::vector<int> degi(n, deg);
    int dmax = 1;
    for (int i = 0; i < n; i++) {
        lm[i] = lfull[i] > 1.25 * lsym[i] ? lfull[i] : lsym[i];
        const double lmax = safety * lm[i], half = 0.5 * (lmax - lmax / H.ratio);
        if (safety * beta[i] >= half) degi[i] = std::min(deg, 2);
        dmax = std::max(dmax, degi[i]);
        if (verbose)
            std::fprintf(stderr, "[hts] heat Chebyshev instance %d: lmax symmetric %.6g, with convection %.6g, "
                         "imaginary extent %.6g, degree %d\n", i, lsym[i], lfull[i], beta[i], degi[i]);
    }
    H.deg = dmax;
    build_smoother(H, 0, H.deg, H.ratio, &lm, &beta, &degi);
    return H;
}

// Per-instance depth: every instance coarsens (2:1 per axis, odd counts
// included) until its own level has at most coarse_max nodes, whatever batch
// it sits in.  On each level the batch keeps the instances present there and,
// among them, the ones that continue to a coarser level; an instance ends
// with a dense FP64 solve on its last level.
void Batch::build_hierarchy(Hier &H, const hts_solver_opts &o)
{
    const int coarse_max = std::max(8, o.mg_coarse_max);
    H.lev.clear();
    H.lev.emplace_back();
    {
        Level &L = H.lev[0];
        level_alloc(L, al, s, ntot);
        L.nch = nch;
        L.red = rch;
        L.ch_ext = ch.p;
        L.nch_all = nch;
        L.ch_all_ext = ch.p;
        L.present.assign(n, 1);
        L.cont.assign(n, 1);        // the matrix-free level always has a coarser level
        std::vector<LevelDev> g(n);
        for (int i = 0; i < n; i++) {
            g[i].NX = m[i]->N[0]; g[i].NY = m[i]->N[1]; g[i].NZ = m[i]->N[2];
            g[i].off = off[i]; g[i].n = m[i]->nnode; g[i].S = nullptr;
        }
        L.h64 = g;
        L.g64.upload(al, g, s);
        L.g32.upload(al, g, s);
        for (int i = 0; i < n; i++) launch_inv_diag(H.ops.h64[i], L.invd64.p + off[i], s);
        convert_plain(ntot, L.invd64.p, L.invd32.p, s);
        L.dims.resize(3 * n);
        L.off.assign(off.begin(), off.end());
        for (int i = 0; i < n; i++)
            for (int d = 0; d < 3; d++) L.dims[3 * i + d] = m[i]->N[d];
    }
    for (int lev = 1; lev < 24; lev++) {
        {
            bool any = false;
            for (int i = 0; i < n; i++) any |= H.lev[lev - 1].cont[i] != 0;
            if (!any) break;
        }
        H.lev.emplace_back();
        Level &C = H.lev.back();
        const Level &Fl = H.lev[lev - 1];
        C.dims.assign(3 * n, 0);
        C.present.assign(n, 0);
        C.cont.assign(n, 0);
        std::vector<int64_t> coff(n, 0), ccnt(n, 0);
        int64_t ctot = 0;
        for (int i = 0; i < n; i++) {
            coff[i] = ctot;
            if (!Fl.cont[i]) continue;
            C.present[i] = 1;
            int64_t nn = 1;
            bool shrink = false;
            for (int d = 0; d < 3; d++) {
                const int cells_c = (Fl.dims[3 * i + d] - 1 + 1) / 2;
                C.dims[3 * i + d] = cells_c + 1;
                nn *= cells_c + 1;
                shrink |= C.dims[3 * i + d] > 2;
            }
            ccnt[i] = nn;
            ctot += nn;
            C.cont[i] = (nn > coarse_max && shrink) ? 1 : 0;
        }
        level_alloc(C, al, s, ctot);
        C.off = coff;
        // chunk lists: all present instances (restriction target) and the
        // continuing ones (smoothing, residual, prolongation)
        {
            std::vector<int32_t> sp;
            build_chunks(coff, ccnt, CHUNK_LEN_COARSE, C.hch_all, sp);
            C.nch_all = (int)C.hch_all.size();
            C.ch_all.upload(al, C.hch_all, s);
            C.ch_all_ext = C.ch_all.p;
            std::vector<int64_t> kcnt(n, 0);
            for (int i = 0; i < n; i++) kcnt[i] = C.cont[i] ? ccnt[i] : 0;
            build_chunks(coff, kcnt, CHUNK_LEN_COARSE, C.hch, sp);
            C.nch = (int)C.hch.size();
            C.ch.upload(al, C.hch, s);
            C.segp.upload(al, sp, s);
            C.red = RedCtx{C.segp.p, n, n == 1 ? sp[1] : -1};
            C.ch_ext = C.ch.p;
        }
        C.S64.alloc(al, (size_t)27 * std::max<int64_t>(ctot, 1));
        C.S32.alloc(al, (size_t)27 * std::max<int64_t>(ctot, 1));
        C.soff = coff;
        for (int i = 0; i < n; i++) {
            if (!C.present[i]) continue;
            const int fN[3] = {Fl.dims[3 * i], Fl.dims[3 * i + 1], Fl.dims[3 * i + 2]};
            const int cN[3] = {C.dims[3 * i], C.dims[3 * i + 1], C.dims[3 * i + 2]};
            double *Sc = C.S64.p + 27 * coff[i];
            if (lev == 1) {
                if (p == 1) {
                    DBuf<double> Sf;
                    Sf.alloc(al, (size_t)27 * m[i]->nnode);
                    launch_fine_stencil(H.ops.h64[i], Sf.p, s);
                    launch_rap(fN[0], fN[1], fN[2], Sf.p, cN[0], cN[1], cN[2], Sc, s);
                    sync(s);
                } else {
                    // p-coarsening: the Q1 operator on the same cells
                    // p-coarsening: the Q1 operator on the same cells, its
                    // vertices constrained where the Q2 node at the vertex is
                    OpDev q1 = H.ops.h64[i];
                    q1.p = 1;
                    q1.NX = cN[0]; q1.NY = cN[1]; q1.NZ = cN[2];
                    q1.nnode = ccnt[i];
                    q1.lcol = nullptr;
                    q1.lfcol = nullptr;
                    q1.dcol = nullptr;
                    const std::vector<int32_t> &fd = m[i]->h_dcol[H.field];
                    if (!fd.empty()) {
                        std::vector<int32_t> cd((size_t)cN[0] * cN[1], DCOL_NONE);
                        for (int J = 0; J < cN[1]; J++)
                            for (int I = 0; I < cN[0]; I++) {
                                const int packed = fd[(size_t)(2 * I) + (size_t)fN[0] * (2 * J)];
                                const int lo = packed & 0xFFFF, hi = (packed >> 16) & 0xFFFF;
                                if (packed == DCOL_NONE || lo > hi) continue;
                                const int clo = (lo + 1) / 2, chi = hi / 2;
                                if (clo <= chi) cd[(size_t)I + (size_t)cN[0] * J] = clo | (chi << 16);
                            }
                        C.qdcol.emplace_back();
                        C.qdcol.back().upload(al, cd, s);
                        q1.dcol = C.qdcol.back().p;
                    }
                    launch_q1_stencil(q1, Sc, s);
                }
            } else {
                const double *Sf = Fl.S64.p + 27 * Fl.soff[i];
                launch_rap(fN[0], fN[1], fN[2], Sf, cN[0], cN[1], cN[2], Sc, s);
            }
            launch_stencil_invdiag(Sc, ccnt[i], C.invd64.p + coff[i], s);
        }
        if (ctot > 0) {
            convert_plain((int64_t)27 * ctot, C.S64.p, C.S32.p, s);
            convert_plain(ctot, C.invd64.p, C.invd32.p, s);
        }
        std::vector<LevelDev> g64(n), g32(n);
        for (int i = 0; i < n; i++) {
            LevelDev g{};
            g.NX = C.dims[3 * i]; g.NY = C.dims[3 * i + 1]; g.NZ = C.dims[3 * i + 2];
            g.off = coff[i]; g.n = ccnt[i];
            g.S = C.S64.p + 27 * coff[i];
            g64[i] = g;
            g.S = C.S32.p + 27 * coff[i];
            g32[i] = g;
        }
        C.h64 = g64;
        C.g64.upload(al, g64, s);
        C.g32.upload(al, g32, s);
        // dense inverses of the instances that end on this level
        std::vector<CoarseDev> cd;
        int64_t row0 = 0;
        for (int i = 0; i < n; i++) {
            if (!C.present[i] || C.cont[i]) continue;
            const int64_t nn = ccnt[i];
            std::vector<double> st((size_t)27 * nn);
            HTS_HIP(hipMemcpy(st.data(), C.S64.p + 27 * coff[i], st.size() * sizeof(double), hipMemcpyDeviceToHost));
            const int NX = C.dims[3 * i], NY = C.dims[3 * i + 1], NZ = C.dims[3 * i + 2];
            std::vector<double> A((size_t)nn * nn, 0.0);
            for (int64_t r = 0; r < nn; r++) {
                int i0 = (int)(r % NX), j0 = (int)((r / NX) % NY), k0 = (int)(r / ((int64_t)NX * NY));
                for (int c = 0; c < 27; c++) {
                    int a = i0 + c % 3 - 1, b = j0 + (c / 3) % 3 - 1, d = k0 + c / 9 - 1;
                    if (a < 0 || a >= NX || b < 0 || b >= NY || d < 0 || d >= NZ) continue;
                    A[(size_t)r * nn + a + (int64_t)NX * (b + (int64_t)NY * d)] += st[(size_t)c * nn + r];
                }
            }
            if (!invert_spd_banded(A, (int)nn, NX * NY + NX + 1)) invert_dense(A, (int)nn);
            C.Ainv.emplace_back();
            C.Ainv.back().upload(al, A, s);
            CoarseDev e{};
            e.Ainv = C.Ainv.back().p;
            e.n = nn;
            e.off = coff[i];
            e.row0 = row0;
            e.inst = i;
            row0 += nn;
            cd.push_back(e);
        }
        C.ncd = (int)cd.size();
        C.crows = row0;
        if (!cd.empty()) C.cd.upload(al, cd, s);
        sync(s);
    }
    // smoothers on every level with continuing instances
    for (size_t l = 0; l < H.lev.size(); l++)
        if (H.lev[l].nch > 0) build_smoother(H, (int)l, 2 * H.deg, l == 0 ? H.ratio : H.ratio_coarse);
    sync(s);
}

// ---------------------------------------------------------------- V-cycle
template <typename T>
void Batch::smooth(Hier &H, int l, int steps, int first, const T *b, T *&cur, T *&oth)
{
    Level &L = H.lev[l];
    EpiArgs<T> ep{};
    ep.b = b;
    ep.d = PK(T, L.d64, L.d32);
    ep.invd = PK(T, L.invd64, L.invd32);
    ep.S = L.cheb.p;
    for (int k = 0; k < steps; k++) {
        ep.s1 = S_CHEB + 2 * (first + k);
        ep.s2 = ep.s1 + 1;
        apply_lvl<T>(H, l, EPI_CHEB, true, cur, oth, ep);
        std::swap(cur, oth);
    }
}

template <typename T>
void Batch::vcycle(Hier &H, int l, const T *b, T *x)
{
    Level &L = H.lev[l];
    if (L.ncd > 0) launch_coarse_solve<T>(L.cd.p, L.ncd, L.crows, active.p, b, x, s);
    if (L.nch == 0) return;
    const int deg = H.deg;
    T *xb = PK(T, L.xb64, L.xb32);
    T *cur = xb, *oth = x;   // 2*deg - 1 swaps end in x
    cheb_from_zero<T>(H, l, deg, b, cur, oth);
    // residual, restriction, coarse correction
    EpiArgs<T> ep{};
    ep.b = b;
    T *t = PK(T, L.t64, L.t32);
    apply_lvl<T>(H, l, EPI_RESID, true, cur, t, ep);
    Level &C = H.lev[l + 1];
    const OpDev *fops = (l == 0) ? H.ops.d64.p : nullptr;
    // the Q1 level under a Q2 fine level is re-discretised with its Dirichlet
    // vertices eliminated; Galerkin levels keep them as coupled unknowns
    const int mask_coarse = (l == 0 && p == 2) ? 1 : 0;
    launch_restrict<T>(L.g64.p, C.g64.p, fops, C.ch_all_ext, C.nch_all, active.p, t, PK(T, C.b64, C.b32), mask_coarse,
                       s);
    vcycle<T>(H, l + 1, PK(T, C.b64, C.b32), PK(T, C.x64, C.x32));
    launch_prolong_add<T>(L.g64.p, C.g64.p, fops, L.ch_ext, L.nch, active.p, PK(T, C.x64, C.x32), cur, s);
    // post-smoothing restarts the Chebyshev recurrence (first coefficient pair has c1 = 0)
    smooth<T>(H, l, deg, 0, b, cur, oth);
    if (cur != x) {
        VecCtx vc{L.ch_ext, L.nch, active.p, S.p, s};
        vcopy<T>(vc, cur, x);
    }
}

// deg Chebyshev steps on level l from x = 0, leaving the result in cur
// after deg - 1 swaps of (cur, oth).  The first two steps run as one
// operator pass (EPI_CHEB0) where the level's kernel has that epilogue
// (Q1 and stencil levels), else the first step is its own kernel.
template <typename T>
void Batch::cheb_from_zero(Hier &H, int l, int deg, const T *b, T *&cur, T *&oth)
{
    Level &L = H.lev[l];
    if (deg >= 2 && !(l == 0 && p == 2)) {
        EpiArgs<T> ep{};
        ep.b = b;
        ep.d = PK(T, L.d64, L.d32);
        ep.invd = PK(T, L.invd64, L.invd32);
        ep.S = L.cheb.p;
        ep.s0 = S_CHEB + 1;
        ep.s1 = S_CHEB + 2;
        ep.s2 = S_CHEB + 3;
        apply_lvl<T>(H, l, EPI_CHEB0, true, cur, oth, ep);
        std::swap(cur, oth);
        smooth<T>(H, l, deg - 2, 2, b, cur, oth);
        return;
    }
    launch_cheb0<T>(L.ch_ext, L.nch, active.p, L.cheb.p, S_CHEB + 1, PK(T, L.invd64, L.invd32), b,
                    PK(T, L.d64, L.d32), cur, s);
    smooth<T>(H, l, deg - 1, 1, b, cur, oth);
}

template <typename T>
void Batch::cheb_prec(Hier &H, const T *b, T *x)
{
    Level &L = H.lev[0];
    const int deg = H.deg;
    T *xb = PK(T, L.xb64, L.xb32);
    T *cur = ((deg - 1) % 2 == 0) ? x : xb;
    T *oth = (cur == x) ? xb : x;
    cheb_from_zero<T>(H, 0, deg, b, cur, oth);
}

// ------------------------------------------------------------------- CG
template <typename T>
int Batch::cg(const Tables &A, const std::function<void(const T *, T *)> &M, const T *b, T *x, int maxit,
              bool flexible, int check_every, bool x0_zero)
{
    T *r = PK(T, this->r, r32), *z = PK(T, this->z, z32), *pv = PK(T, pp, p32), *q = PK(T, this->q, q32);
    T *ro = flexible ? PK(T, rold, rold32) : nullptr;
    VecCtx v = vctx();
    EpiArgs<T> ep{};
    ep.b = b;
    ep.partial = partial.p;
    exported_last = false;
    if (x0_zero) {
        // r = b - A 0 = b: a copy and a norm instead of an operator pass
        vcopy<T>(v, b, r);
        vdot<T>(v, b, b, nullptr, partial.p);
        vreduce(rch, partial.p, 2, RED_CG_INIT, 0, S.p, active.p, maxit, 0.0, nullptr, s);
    } else {
        apply_op<T>(A, EPI_RESID_NORM, true, x, r, ep);
        vreduce(rwk[A.field][prec_of<T>()], partial.p, 1, RED_CG_INIT, 0, S.p, active.p, maxit, 0.0, nullptr, s);
    }
    const bool hook = std::is_same<T, double>::value && cg_hook;
    const bool graphed = use_graph && !hook && !g_timing.on;
    // (replayed chunks skip instances that converged at the start, so only
    // the eager loop checks here)
    if (!graphed && !any_active()) {
        exported_last = true;
        return 0;
    }
    if (hook) cg_hook(reinterpret_cast<const double *>(x), 0);
    M(r, z);
    vdot<T>(v, r, z, nullptr, partial.p);
    vreduce(rch, partial.p, 2, RED_STORE, S_RZ, S.p, active.p, 0, 0.0, nullptr, s);
    vcopy<T>(v, z, pv);
    if (graphed) {
        // Chunks replayed as graphs with a host check between them: the first
        // chunk as long as the previous solve of this system took, then
        // chunks of one (or check_every) iteration.  Every chunk ends right
        // after a convergence check, so a chunk of the right length launches
        // no preconditioner application past convergence; the later chunks
        // start with the preconditioner and the direction update that the
        // eager loop runs at the end of an iteration.
        char key[256];
        std::snprintf(key, sizeof key, "cg%d|%d|%p|%p|%p|%d|%d", (int)sizeof(T), A.field, (const void *)&A,
                      (const void *)b, (const void *)x, maxit, flexible ? 1 : 0);
        // the preconditioner closure is identified by its target, not its address
        const std::string base = std::string(key) + "|" + graph_tag;
        // iteration history per outer refinement step: later refinement
        // steps usually need far fewer iterations than the first
        const std::string hkey = base + "|o" + std::to_string(hist_tag);
        auto hist = last_iters.find(hkey);
        int K = hist != last_iters.end() ? hist->second : 4;
        int done = 0;
        while (done < maxit) {
            K = std::max(1, std::min(K, maxit - done));
            if (chunk_cap > 0) K = std::min(K, chunk_cap);
            const std::string mode = chunk_mode ? chunk_mode() : std::string();
            const bool lead = done > 0;
            replay(base + mode + (lead ? "|c" : "|f") + std::to_string(K), [&] {
                VecCtx vg = vctx();
                for (int c = 0; c < K; c++) {
                    if (c > 0 || lead) {
                        M(r, z);
                        vdot<T>(vg, z, r, ro, partial.p);
                        vreduce(rch, partial.p, 2, RED_CG_BETA, 0, S.p, active.p, 0, 0.0, nullptr, s);
                        vaxpby<T>(vg, 1.0, -1, z, 1.0, S_BETA, pv);
                    }
                    EpiArgs<T> e2{};
                    e2.partial = partial.p;
                    apply_op<T>(A, EPI_DOT, true, pv, q, e2);
                    vreduce(rwk[A.field][prec_of<T>()], partial.p, 1, RED_CG_ALPHA, 0, S.p, active.p, 0, 0.0, nullptr, s);
                    vcg_update<T>(vg, x, r, pv, q, ro, partial.p);
                    vreduce(rch, partial.p, 2, RED_CG_CONV, 0, S.p, active.p, maxit, 0.0, nullptr, s);
                }
            });
            done += K;
            if (!any_active()) break;
            K = std::max(1, check_every);
        }
        // every chunk ends with an export: the slots are those of the last one
        slots_from_export();
        exported_last = true;
        int used = 0;
        for (int i = 0; i < n; i++) used = std::max(used, (int)hS[(size_t)i * NSLOT + S_ITER]);
        // a solve in which no instance iterated (all converged at the start)
        // keeps the chunk length, so that it captures no new graph
        if (used > 0) last_iters[hkey] = used;
        return done;
    }
    int it = 0;
    for (it = 1; it <= maxit; it++) {
        EpiArgs<T> e2{};
        e2.partial = partial.p;
        apply_op<T>(A, EPI_DOT, true, pv, q, e2);
        vreduce(rwk[A.field][prec_of<T>()], partial.p, 1, RED_CG_ALPHA, 0, S.p, active.p, 0, 0.0, nullptr, s);
        vcg_update<T>(v, x, r, pv, q, ro, partial.p);
        if (hook) cg_hook(reinterpret_cast<const double *>(x), it);
        vreduce(rch, partial.p, 2, RED_CG_CONV, 0, S.p, active.p, maxit, 0.0, nullptr, s);
        static const bool verbose = env_or("HTS_VERBOSE", 0.0) > 1.0;
        if (verbose) {
            download_S();
            std::fprintf(stderr, "[hts] cg it %d rr %.6e rr0 %.6e\n", it, hS[S_RR], hS[S_RR0]);
        }
        if (it % std::max(1, check_every) == 0 || it == maxit)
            if (!any_active()) {
                exported_last = true;
                break;
            }
        M(r, z);
        vdot<T>(v, z, r, ro, partial.p);
        vreduce(rch, partial.p, 2, RED_CG_BETA, 0, S.p, active.p, 0, 0.0, nullptr, s);
        vaxpby<T>(v, 1.0, -1, z, 1.0, S_BETA, pv);
    }
    return it;
}

// ---------------------------------------------------------------- FGMRES
template <typename T>
void Batch::fgmres(const Tables &A, const std::function<void(const T *, T *)> &M, const T *b, T *x, int maxit,
                   int mres, int check_every, bool x0_zero)
{
    ensure_gmres(mres);
    T *V = PK(T, V64, V32), *Z = PK(T, Z64, Z32);
    const int64_t ld = ntot;
    VecCtx v = vctx();
    for (int cycle = 0; cycle < 1000; cycle++) {
        EpiArgs<T> ep{};
        ep.b = b;
        ep.partial = partial.p;
        if (x0_zero && cycle == 0) {
            // V_0 = b - A 0 = b
            vcopy<T>(v, b, V);
            vdot<T>(v, b, b, nullptr, partial.p);
            vreduce(rch, partial.p, 2, RED_STORE, S_RR, S.p, active.p, 0, 0.0, nullptr, s);
        } else {
            apply_op<T>(A, EPI_RESID_NORM, true, x, V, ep);
            vreduce(rwk[A.field][prec_of<T>()], partial.p, 1, RED_STORE, S_RR, S.p, active.p, 0, 0.0, nullptr, s);
        }
        // which instances take part (S_CYC) is read back with the first
        // check of the Arnoldi steps, not on its own
        gm_begin(n, active.p, S.p, gg.p, mres, gkdim.p, s);
        vaxpby<T>(v, 1.0, S_SCALE, V, 0.0, -1, V);
        // one Arnoldi step; every kernel skips instances whose cycle ended
        auto step_j = [&](int j) {
            VecCtx vj = vctx();
            T *Vj = V + (int64_t)j * ld, *w = V + (int64_t)(j + 1) * ld, *Zj = Z + (int64_t)j * ld;
            M(Vj, Zj);
            EpiArgs<T> e2{};
            apply_op<T>(A, EPI_STORE, true, Zj, w, e2);
            vmultidot<T>(vj, V, ld, j + 1, w, partial.p, j + 1);
            vreduce(rch, partial.p, j + 1, RED_NONE, 0, S.p, active.p, 0, 0.0, gh1.p, s);
            vorth_update<T>(vj, V, ld, j + 1, gh1.p, j + 1, w, 1, partial.p, j + 2);
            // the second pass's sums, the Hessenberg column and the norm
            // (from |w'|^2 - |h2|^2) in one kernel, then the second
            // projection and the normalisation in one pass
            const ArnArgs arn{j, mres, maxit, 0, gh1.p, gH.p, gcs.p, gsn.p, gg.p, gkdim.p};
            vreduce_arnoldi(rch, partial.p, j + 2, S.p, active.p, arn, gh2.p, s);
            vorth_update<T>(vj, V, ld, j + 1, gh2.p, j + 2, w, 0, nullptr, 0, S_SCALE);
        };
        if (use_graph && !g_timing.on) {
            // the whole cycle as one graph, in chunks of K steps with a host
            // check between them: the first as long as the previous cycle of
            // this system, then one (or check_every) step at a time
            char key[256];
            std::snprintf(key, sizeof key, "gm%d|%d|%p|%p|%p|%d|%d", (int)sizeof(T), A.field, (const void *)&A,
                          (const void *)b, (const void *)x, maxit, mres);
            const std::string base = std::string(key) + "|" + graph_tag;
            const std::string hkey = base + "|o" + std::to_string(hist_tag);
            auto hist = last_iters.find(hkey);
            int K = hist != last_iters.end() ? hist->second : 8;
            int j0 = 0;
            for (; j0 < mres;) {
                const int j1 = std::min(mres, j0 + std::max(1, K));
                replay(base + "|" + std::to_string(j0) + "-" + std::to_string(j1), [&] {
                    for (int j = j0; j < j1; j++) step_j(j);
                });
                j0 = j1;
                if (!any_active()) break;
                K = std::max(1, check_every);
            }
        } else {
            for (int j = 0; j < mres; j++) {
                step_j(j);
                if ((j + 1) % std::max(1, check_every) == 0 || j == mres - 1)
                    if (!any_active()) break;
            }
        }
        // both loops end with an export
        slots_from_export();
        std::vector<int32_t> cyc(n, 0);
        bool any = false;
        for (int i = 0; i < n; i++) {
            cyc[i] = hS[(size_t)i * NSLOT + S_CYC] == 1.0;
            any |= cyc[i] != 0;
        }
        if (!any) break;
        if (use_graph && !g_timing.on && cycle == 0) {
            char key[256];
            std::snprintf(key, sizeof key, "gm%d|%d|%p|%p|%p|%d|%d", (int)sizeof(T), A.field, (const void *)&A,
                          (const void *)b, (const void *)x, maxit, mres);
            const std::string hkey = std::string(key) + "|" + graph_tag + "|o" + std::to_string(hist_tag);
            int used = 0;
            for (int i = 0; i < n; i++)
                if (cyc[i]) used = std::max(used, (int)hS[(size_t)i * NSLOT + S_ITER]);
            last_iters[hkey] = std::max(1, std::min(used, mres));
        }
        // x += Z y for every instance that took part in this cycle (neither
        // kernel writes the slots, so the export that ended the Arnoldi steps
        // still holds them)
        set_active(cyc);
        gm_solve(n, active.p, mres, gH.p, gg.p, gkdim.p, gy.p, s);
        vbasis_update<T, T>(v, Z, ld, gkdim.p, gy.p, mres, 1.0, -1, x);
        slots_from_export();
        std::vector<int32_t> again(n, 0);
        bool more = false;
        for (int i = 0; i < n; i++) {
            if (cyc[i] && hS[(size_t)i * NSLOT + S_STATUS] == 1.0) {
                again[i] = 1;
                more = true;
            }
        }
        // (without a next cycle the caller sets the flags it needs before
        // its next launch)
        if (!more) break;
        set_active(again);
    }
    exported_last = true;
}

void Batch::ensure_gmres(int mres)
{
    if (gm_m == mres) return;
    drop_graphs();
    gm_m = mres;
    V64.alloc(al, (size_t)(mres + 1) * ntot);
    Z64.alloc(al, (size_t)mres * ntot);
    V32.alloc(al, (size_t)(mres + 1) * ntot);
    Z32.alloc(al, (size_t)mres * ntot);
    V64.zero(s); Z64.zero(s); V32.zero(s); Z32.zero(s);
    gH.alloc(al, (size_t)n * (mres + 1) * mres);
    gcs.alloc(al, (size_t)n * mres);
    gsn.alloc(al, (size_t)n * mres);
    gg.alloc(al, (size_t)n * (mres + 1));
    gy.alloc(al, (size_t)n * mres);
    gh1.alloc(al, (size_t)n * (mres + 2));
    gh2.alloc(al, (size_t)n * (mres + 2));
    gkdim.alloc(al, n);
    gkdim.zero(s);
}

// ---------------------------------------------------- field solve (outer)
// FP64 defect correction around an inner Krylov solve in FP64 or FP32:
//   r = b - A64 x;  stop when ||r|| <= rtol ||b||;  d ~ A^{-1} (r / ||r||);
//   x += ||r|| d.  The outer test is the true FP64 residual of every mode.
FieldStats Batch::solve_field(int field, Hier *mg, const Tables &A, double *b64, double *x64,
                              const hts_solver_opts &o, std::vector<int32_t> participants, Hier *hprec)
{
    FieldStats st;
    st.status.assign(n, 1);
    st.iters.assign(n, 0);
    st.outer.assign(n, 0);
    st.relres.assign(n, 0.0);
    st.fallbacks.assign(n, 0);
    const bool fp32 = o.mode == HTS_MODE_FP32_REFINED;
    const bool learned = o.mode == HTS_MODE_LEARNED && field == 0;
    use_graph = o.use_graph != 0;
    if (learned && !o.nn) throw Error(HTS_ERR_ARG, "learned mode needs opts.nn");
    if (learned && !mg) throw Error(HTS_ERR_STATE, "learned mode needs the multigrid fallback");
    const double rtol = o.rtol > 0 ? o.rtol : 1e-8;
    const int maxit = std::max(1, o.max_iter);
    hipEvent_t e0, e1;
    HTS_HIP(hipEventCreate(&e0));
    HTS_HIP(hipEventCreate(&e1));
    HTS_HIP(hipEventRecord(e0, s));
    // the device flags equal participants on entry: both callers set them
    // with the right-hand side, and nothing launched since changes them
    VecCtx vall = vctx();
    vdot<double>(vall, b64, b64, nullptr, partial.p);
    vreduce(rch, partial.p, 2, RED_NONE, 0, S.p, active.p, 0, 0.0, redout.p, s);
    set_otol(n, active.p, S.p, redout.p, 2, rtol * rtol, s);
    std::vector<int32_t> outer = participants;
    int total_inner = 0;
    bool fresh = false;   // the last export holds the final slots
    // The device flags equal outer at the top of every outer step: the
    // participants on entry (the norm and tolerance launches above only read
    // them) and outer as set at the end of the previous step (the update
    // there only reads them).
    for (int oit = 0; oit < 40; oit++) {
        EpiArgs<double> ep{};
        ep.b = b64;
        ep.partial = partial.p;
        apply_op<double>(A, EPI_RESID_NORM, true, x64, this->y.p, ep);
        vreduce(rwk[A.field][0], partial.p, 1, RED_NONE, 0, S.p, active.p, 0, 0.0, redout.p, s);
        outer_check(n, active.p, S.p, redout.p, s);
        HTS_HIP(hipEventRecord(e1, s));
        // The first check is read back with the inner solve's last export
        // (the inner kernels skip the instances it deactivated), which saves
        // a host round trip; later checks are read at once.
        const bool defer = oit == 0 && !learned;
        const std::vector<int32_t> prev = outer;
        if (!defer) {
            outer = get_active();
            fresh = true;
            bool any = false;
            for (int a : outer) any |= a != 0;
            if (!any) break;
            fresh = false;
            for (int i = 0; i < n; i++)
                if (outer[i]) st.outer[i]++;
        }
        // inner system: A d = r / ||r||
        hist_tag = oit;
        const double fl = fp32 ? std::pow(std::max(o.inner_rtol, 1e-6), 2) : 0.0;
        set_inner_tol(n, active.p, S.p, fl, 0.25, s);
        VecCtx v = vctx();
        if (fp32) {
            vconvert<double, float>(v, 1.0, S_OINV, this->y.p, b32.p);
            vfill<float>(v, x32.p, 0.0f);
            auto M = [&](const float *r_, float *z_) {
                if (mg) vcycle<float>(*mg, 0, r_, z_);
                else if (hprec->tensor) tmass_prec<float>(*hprec, r_, z_);
                else cheb_prec<float>(*hprec, r_, z_);
            };
            graph_tag = (mg ? "mg" : "cheb") + std::to_string((uintptr_t)(mg ? mg : hprec));
            if (field == 0) cg<float>(A, M, b32.p, x32.p, maxit, false, o.check_every, true);
            else fgmres<float>(A, M, b32.p, x32.p, maxit, std::max(2, std::min(o.gmres_restart, 60)), o.check_every,
                                 true);
        } else {
            // inner RHS r / ||r||; the Krylov work vectors are r, z, pp, q, rold
            vaxpby<double>(v, 1.0, S_OINV, this->y.p, 0.0, -1, inner_b.p);
            vfill<double>(v, inner_x.p, 0.0);
            auto M = [&](const double *r_, double *z_) {
                if (mg) vcycle<double>(*mg, 0, r_, z_);
                else if (hprec->tensor) tmass_prec<double>(*hprec, r_, z_);
                else cheb_prec<double>(*hprec, r_, z_);
            };
            graph_tag = (mg ? "mg" : "cheb") + std::to_string((uintptr_t)(mg ? mg : hprec));
            if (learned) {
                // Flexible CG with the network as preconditioner; the
                // fallback rule runs on the device (nn_gate_*: two
                // consecutive weak iterations or a non-finite residual or
                // network output send the instance to the V-cycle for the
                // rest of this inner solve), so an application needs no
                // host round trip and the loop can be replayed as a graph.
                nn_prepare(o.nn, *this);
                nn_gate_init(n, S.p, s);
                graph_tag = "nn" + std::to_string(nn_serial(o.nn)) + "|" + std::to_string((uintptr_t)mg);
                // Once every instance still iterating has fallen back (as the
                // exports between chunks or iterations show), the network's
                // gated launches are left out: the remaining chunks are plain
                // V-cycle-preconditioned iterations.
                const uint32_t seq0 = exp_seq;
                auto all_fell_back = [&]() {
                    if (exp_seq == seq0) return false;
                    for (int i = 0; i < n; i++)
                        if (hact[i] && hexpS[(size_t)i * NSLOT + S_NN_FB] == 0.0) return false;
                    return true;
                };
                chunk_mode = [&]() { return all_fell_back() ? std::string("|mg") : std::string("|nn"); };
                // short chunks while the network is in use, so that a
                // fallback is seen (and its gated launches dropped) soon
                chunk_cap = 2;
                auto ML = [&](const double *r_, double *z_) {
                    if (all_fell_back()) {
                        vcycle<double>(*mg, 0, r_, z_);
                        return;
                    }
                    nn_gate_begin(n, active.p, S.p, nn_use.p, nn_mg.p, act_save.p, s);
                    for (int i = 0; i < n; i++) nn_precondition(o.nn, *this, i, r_, z_, nn_use.p + i);
                    vdot<double>(vctx(), z_, z_, nullptr, partial.p);
                    vreduce(rch, partial.p, 2, RED_STORE, S_TMP2, S.p, active.p, 0, 0.0, nullptr, s);
                    nn_gate_check(n, S.p, nn_use.p, nn_mg.p, active.p, s);
                    vcycle<double>(*mg, 0, r_, z_);   // the fallback instances only
                    nn_gate_end(n, act_save.p, active.p, s);
                };
                cg<double>(A, ML, inner_b.p, inner_x.p, maxit, true, 1, true);
                chunk_mode = nullptr;
                chunk_cap = 0;
            } else if (field == 0) {
                cg<double>(A, M, inner_b.p, inner_x.p, maxit, false, o.check_every, true);
            } else
                fgmres<double>(A, M, inner_b.p, inner_x.p, maxit, std::max(2, std::min(o.gmres_restart, 60)),
                               o.check_every, true);
        }
        if (inner_hook && field == 0 && !fp32) {
            inner_hook(A, inner_x.p);
            exported_last = false;
        }
        if (exported_last) slots_from_export();
        else download_S();
        if (defer) {
            bool any = false;
            for (int i = 0; i < n; i++) {
                outer[i] = prev[i] && hS[(size_t)i * NSLOT + S_OSTATUS] == 1.0;
                any |= outer[i] != 0;
                if (outer[i]) st.outer[i]++;
            }
            if (!any) {
                fresh = true;   // hS is current: nothing was queued after its export
                break;
            }
        }
        for (int i = 0; i < n; i++)
            if (outer[i]) {
                st.iters[i] += (int)hS[(size_t)i * NSLOT + S_ITER];
                total_inner += (int)hS[(size_t)i * NSLOT + S_ITER];
                if (learned) st.fallbacks[i] += (int)hS[(size_t)i * NSLOT + S_NN_NFB];
                const double ist = hS[(size_t)i * NSLOT + S_STATUS];
                if (ist == -6.0) st.status[i] = -6;
            }
        set_active(outer);
        if (fp32) vadd_scaled<float>(vctx(), 1.0, S_ONORM, x32.p, x64);
        else vadd_scaled<double>(vctx(), 1.0, S_ONORM, inner_x.p, x64);
        bool stop = true;
        for (int i = 0; i < n; i++)
            if (outer[i] && st.status[i] != -6 && st.iters[i] < maxit) stop = false;
        if (stop) {
            // final judge with the last update
            apply_op<double>(A, EPI_RESID_NORM, true, x64, this->y.p, ep);
            vreduce(rwk[A.field][0], partial.p, 1, RED_NONE, 0, S.p, active.p, 0, 0.0, redout.p, s);
            outer_check(n, active.p, S.p, redout.p, s);
            HTS_HIP(hipEventRecord(e1, s));
            outer = get_active();
            fresh = true;
            break;
        }
    }
    if (fresh) {
        slots_from_export();
    } else {
        HTS_HIP(hipEventRecord(e1, s));
        download_S();
    }
    HTS_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    HTS_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    st.ms = ms;
    for (int i = 0; i < n; i++) {
        if (!participants[i]) { st.status[i] = 0; continue; }
        const double orr = hS[(size_t)i * NSLOT + S_ORR], obb = hS[(size_t)i * NSLOT + S_OBB];
        st.relres[i] = obb > 0 ? std::sqrt(orr / obb) : std::sqrt(orr);
        const double os = hS[(size_t)i * NSLOT + S_OSTATUS];
        if (st.status[i] == -6 || os == -6.0) st.status[i] = HTS_ERR_BREAKDOWN;
        else if (os == 0.0) st.status[i] = HTS_OK;
        else st.status[i] = HTS_ERR_NOT_CONVERGED;
    }
    (void)total_inner;
    return st;
}

// ------------------------------------------------------------- one step
void Batch::set_time(const std::vector<double> &tnew, const std::vector<double> &fscale,
                     const std::vector<double> *xtra, const std::vector<double> *xtra2)
{
    const int slots[4] = {S_TNEW, S_FSCALE, S_XTRA, S_XTRA2};
    const double *vals[4] = {tnew.data(), fscale.data(), xtra ? xtra->data() : nullptr,
                             xtra2 ? xtra2->data() : nullptr};
    vset_slots(slots, xtra ? (xtra2 ? 4 : 3) : 2, vals, n, S.p, s);
}

// Factors of each instance's initial guess X^n + c1 (X^n - X^{n-1}) +
// c2 (X^{n-1} - X^{n-2}): the value at t^n + dt of the polynomial through
// the known levels (Lagrange form at the times 0, -h1, -(h1 + h2) relative to
// t^n; three levels: quadratic, two: linear, one: X^n).  extrapolate = 1
// stops at the linear one.
void Batch::xtra_factors(int field, double dt, const hts_solver_opts &o, std::vector<double> &c1,
                         std::vector<double> &c2) const
{
    c1.assign(n, 0.0);
    c2.assign(n, 0.0);
    if (o.extrapolate <= 0 || !(dt > 0.0)) return;
    for (int i = 0; i < n; i++) {
        const double h1 = m[i]->hist_dt[field], h2 = m[i]->hist_dt2[field];
        if (!(h1 > 0.0)) continue;
        if (o.extrapolate >= 2 && h2 > 0.0) {
            const double Ln = (dt + h1) * (dt + h1 + h2) / (h1 * (h1 + h2));
            const double Lpp = dt * (dt + h1) / ((h1 + h2) * h2);
            c1[i] = Ln - 1.0;
            c2[i] = -Lpp;
        } else {
            c1[i] = dt / h1;
        }
    }
}

void Batch::pressure_rhs(Hier &H, bool steady)
{
    std::vector<int32_t> all(n, 1);
    set_active(all);
    VecCtx v = vctx(false);
    launch_dirichlet_values(H.ops.d64.p, bc[0].p, ch.p, nch, S.p, g.p, s);
    EpiArgs<double> ep{};
    if (!steady) apply_op<double>(massP, EPI_STORE, false, Pn.p, b.p, ep);
    else vfill<double>(v, b.p, 0.0);
    apply_op<double>(H.ops, EPI_STORE, false, g.p, y.p, ep);
    vrhs_combine(v, y.p, ld0.p, S_FSCALE, b.p);
    launch_sources(srows[0].p, srowptr[0].p, sents[0].p, nsrows[0], ssrc[0].p, S.p, b.p, s);
    vmask<double>(v, H.ops.d64.p, b.p, 0.0);
}

void Batch::heat_rhs(Hier &H)
{
    std::vector<int32_t> all(n, 1);
    set_active(all);
    VecCtx v = vctx(false);
    launch_source_values(lsrc.p, nlsrc, S.p, lcoef.p, s);
    launch_dirichlet_values(H.ops.d64.p, bc[1].p, ch.p, nch, S.p, g.p, s);
    EpiArgs<double> ep{};
    apply_op<double>(massH, EPI_STORE, false, Tn.p, b.p, ep);
    apply_op<double>(H.ops, EPI_STORE, false, g.p, y.p, ep);
    vrhs_combine(v, y.p, ld1.p, S_FSCALE, b.p);
    launch_sources(srows[1].p, srowptr[1].p, sents[1].p, nsrows[1], ssrc[1].p, S.p, b.p, s);
    vmask<double>(v, H.ops.d64.p, b.p, 0.0);
}

// State in and out of the batch vectors, one launch per field for up to 128
// instances (a copy per instance would cost one launch each).
void Batch::gather_state()
{
    if (alias_state) return;
    std::vector<double *> P(n), T(n);
    for (int i = 0; i < n; i++) {
        P[i] = m[i]->P.p;
        T[i] = m[i]->T.p;
    }
    vgather_scatter(ch.p, hch, P, off, Pn.p, true, s);
    vgather_scatter(ch.p, hch, T, off, Tn.p, true, s);
    bool hist = false, hist2 = false;
    for (int i = 0; i < n; i++) {
        hist |= m[i]->hist_dt[0] > 0.0 || m[i]->hist_dt[1] > 0.0;
        hist2 |= m[i]->hist_dt2[0] > 0.0 || m[i]->hist_dt2[1] > 0.0;
    }
    if (hist) {
        for (int i = 0; i < n; i++) {
            P[i] = m[i]->Pprev.p;
            T[i] = m[i]->Tprev.p;
        }
        vgather_scatter(ch.p, hch, P, off, Pp.p, true, s);
        vgather_scatter(ch.p, hch, T, off, Tp.p, true, s);
    }
    if (hist2) {
        for (int i = 0; i < n; i++) {
            P[i] = m[i]->Pprev2.p;
            T[i] = m[i]->Tprev2.p;
        }
        vgather_scatter(ch.p, hch, P, off, Ppp.p, true, s);
        vgather_scatter(ch.p, hch, T, off, Tpp.p, true, s);
    }
}

void Batch::scatter_state()
{
    if (alias_state) {
        export_state();   // completion wait
        return;
    }
    std::vector<double *> P(n), T(n);
    for (int i = 0; i < n; i++) {
        P[i] = m[i]->P.p;
        T[i] = m[i]->T.p;
    }
    vgather_scatter(ch.p, hch, P, off, Pn.p, false, s);
    vgather_scatter(ch.p, hch, T, off, Tn.p, false, s);
    bool hist = false, hist2 = false;
    for (int i = 0; i < n; i++) {
        hist |= m[i]->hist_dt[0] > 0.0 || m[i]->hist_dt[1] > 0.0;
        hist2 |= m[i]->hist_dt2[0] > 0.0 || m[i]->hist_dt2[1] > 0.0;
    }
    if (hist) {
        for (int i = 0; i < n; i++) {
            P[i] = m[i]->Pprev.p;
            T[i] = m[i]->Tprev.p;
        }
        vgather_scatter(ch.p, hch, P, off, Pp.p, false, s);
        vgather_scatter(ch.p, hch, T, off, Tp.p, false, s);
    }
    if (hist2) {
        for (int i = 0; i < n; i++) {
            P[i] = m[i]->Pprev2.p;
            T[i] = m[i]->Tprev2.p;
        }
        vgather_scatter(ch.p, hch, P, off, Ppp.p, false, s);
        vgather_scatter(ch.p, hch, T, off, Tpp.p, false, s);
    }
    export_state();   // completion wait (spin on the export's sequence number)
}

// Solve the pressure of every instance at t_i + dt into P1 (steady or transient).
FieldStats Batch::solve_pressure(double dt, bool steady_all, const hts_solver_opts &o)
{
    std::vector<double> tn(n), fs(n);
    bool steady = steady_all;
    for (int i = 0; i < n; i++) {
        const bool st_i = steady_all || m[i]->B <= 0.0;
        if (i > 0 && st_i != steady) throw Error(HTS_ERR_UNSUPPORTED, "mixed steady/transient pressure in a batch");
        steady = st_i;
    }
    for (int i = 0; i < n; i++) {
        tn[i] = m[i]->t + (steady_all ? 0.0 : dt);
        fs[i] = steady ? 1.0 : dt * m[i]->B;
    }
    std::vector<double> xf, xf2;
    xtra_factors(0, steady_all ? 0.0 : dt, o, xf, xf2);
    set_time(tn, fs, &xf, &xf2);
    Hier &H = pressure_hier(steady, dt, o);
    pressure_rhs(H, steady);
    VecCtx v = vctx(false);
    vextrapolate(v, S_XTRA, S_XTRA2, H.ops.d64.p, Pn.p, Pp.p, Ppp.p, x.p);
    std::vector<int32_t> all(n, 1);
    FieldStats st = solve_field(0, &H, H.ops, b.p, x.p, o, all, nullptr);
    std::vector<int32_t> a(n, 1);
    set_active(a);
    vadd(vctx(false), x.p, g.p, P1.p);
    return st;
}

FieldStats Batch::solve_heat(double dt, const hts_solver_opts &o)
{
    std::vector<double> tn(n), fs(n);
    for (int i = 0; i < n; i++) {
        tn[i] = m[i]->t + dt;
        fs[i] = dt;
    }
    std::vector<double> xf, xf2;
    xtra_factors(1, dt, o, xf, xf2);
    set_time(tn, fs, &xf, &xf2);
    std::vector<int32_t> all(n, 1);
    // every instance's flag is set: the pressure solve of the same step
    // ends by setting them all (the preconditioner set-up below needs them)
    VecCtx v = vctx(false);
    vpiezo32(v, massH.d64.p, P1.p, P32.p);
    // line coefficients before the preconditioner setup reads the operator
    launch_source_values(lsrc.p, nlsrc, S.p, lcoef.p, s);
    Hier &H = heat_prec(dt, o);
    heat_rhs(H);
    vextrapolate(v, S_XTRA, S_XTRA2, H.ops.d64.p, Tn.p, Tp.p, Tpp.p, x.p);
    FieldStats st = solve_field(1, H.multigrid ? &H : nullptr, H.ops, b.p, x.p, o, all, &H);
    set_active(all);
    vadd(vctx(false), x.p, g.p, T1.p);
    return st;
}

// One backward-Euler step for every instance; commits only when all solves
// of all instances converged.
int Batch::step(double dt, const hts_solver_opts &o, std::vector<hts_step_stats> *stats)
{
    FieldStats sp = solve_pressure(dt, false, o);
    FieldStats sh = solve_heat(dt, o);
    int rc = HTS_OK;
    for (int i = 0; i < n; i++) {
        if (sp.status[i] != HTS_OK) rc = rc == HTS_OK ? sp.status[i] : rc;
        if (sh.status[i] != HTS_OK) rc = rc == HTS_OK ? sh.status[i] : rc;
    }
    if (stats) {
        stats->resize(n);
        for (int i = 0; i < n; i++) {
            hts_step_stats &x = (*stats)[i];
            std::memset(&x, 0, sizeof(x));
            x.iters[0] = sp.iters[i]; x.iters[1] = sh.iters[i];
            x.outer[0] = sp.outer[i]; x.outer[1] = sh.outer[i];
            x.relres[0] = sp.relres[i]; x.relres[1] = sh.relres[i];
            x.status[0] = sp.status[i]; x.status[1] = sh.status[i];
            x.time_ms[0] = sp.ms; x.time_ms[1] = sh.ms;
            x.fallbacks = sp.fallbacks[i];
        }
    }
    if (rc == HTS_OK) {
        std::vector<int32_t> all(n, 1);
        set_active(all);
        VecCtx v = vctx(false);
        vshift(v, P1.p, Pn.p, Pp.p, Ppp.p);
        vshift(v, T1.p, Tn.p, Tp.p, Tpp.p);
        for (int i = 0; i < n; i++) {
            m[i]->t += dt;
            for (int f = 0; f < 2; f++) {
                m[i]->hist_dt2[f] = m[i]->hist_dt[f];
                m[i]->hist_dt[f] = dt;
            }
        }
    }
    // no wait here: the statistics came from the solvers' exports, and the
    // caller's scatter of the state waits for the stream
    return rc;
}

std::shared_ptr<Batch> solo_batch(hts_mesh *m)
{
    prepare_mesh(m);
    auto it = m->batches.find("solo");
    if (it != m->batches.end()) return it->second;
    auto B = build_batch({m});
    m->batches["solo"] = B;
    return B;
}

// Batches of several meshes, kept for the next call with the same meshes in
// the same order (hierarchies, dense coarse inverses, captured graphs and
// iteration history survive between calls); the four most recent are kept.
namespace {
struct MultiEntry {
    std::vector<hts_mesh *> ms;
    std::shared_ptr<Batch> B;
};
std::mutex g_multi_mu;
std::vector<MultiEntry> g_multi;
constexpr size_t MULTI_KEEP = 4;
}  // namespace

std::shared_ptr<Batch> multi_batch(const std::vector<hts_mesh *> &ms)
{
    for (hts_mesh *m : ms) prepare_mesh(m);
    {
        std::lock_guard<std::mutex> lk(g_multi_mu);
        for (size_t i = 0; i < g_multi.size(); i++)
            if (g_multi[i].ms == ms) {
                MultiEntry e = std::move(g_multi[i]);
                g_multi.erase(g_multi.begin() + (long)i);
                g_multi.push_back(std::move(e));
                return g_multi.back().B;
            }
    }
    auto B = build_batch(ms);
    std::shared_ptr<Batch> old;
    {
        std::lock_guard<std::mutex> lk(g_multi_mu);
        if (g_multi.size() >= MULTI_KEEP) {
            old = std::move(g_multi.front().B);
            g_multi.erase(g_multi.begin());
        }
        g_multi.push_back({ms, B});
    }
    return B;
}

void forget_batches(hts_mesh *m)
{
    m->batches.clear();
    std::vector<std::shared_ptr<Batch>> drop;
    {
        std::lock_guard<std::mutex> lk(g_multi_mu);
        for (size_t i = 0; i < g_multi.size();) {
            if (std::find(g_multi[i].ms.begin(), g_multi[i].ms.end(), m) != g_multi[i].ms.end()) {
                drop.push_back(std::move(g_multi[i].B));
                g_multi.erase(g_multi.begin() + (long)i);
            } else {
                i++;
            }
        }
    }
    for (auto &B : drop)
        if (B) (void)hipStreamSynchronize(B->s);
}

template void Batch::vcycle<double>(Hier &, int, const double *, double *);
template void Batch::vcycle<float>(Hier &, int, const float *, float *);

}  // namespace hts

// =================================================================== C ABI
using namespace hts;

static hts_solver_opts opts_or_default(const hts_solver_opts *o)
{
    hts_solver_opts d;
    hts_default_opts(&d);
    return o ? *o : d;
}

static void check_ready(hts_mesh *m)
{
    if (!m) throw Error(HTS_ERR_ARG, "null mesh");
    if (!m->has_mat) throw Error(HTS_ERR_STATE, "materials not set");
}

extern "C" {

hts_status hts_kernel_timing(int32_t enable, hts_kernel_times out[2][2])
{
    return guard_call([&] {
        if (enable) {
            for (auto &r : g_timing.recs) {
                g_timing.pool.push_back(r.a);
                g_timing.pool.push_back(r.b);
            }
            g_timing.recs.clear();
            g_timing.on = true;
            return;
        }
        g_timing.on = false;
        hts_kernel_times t[2][2];
        std::memset(t, 0, sizeof(t));
        for (auto &r : g_timing.recs) {
            HTS_HIP(hipEventSynchronize(r.b));
            float ms = 0.0f;
            HTS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
            hts_kernel_times &c = t[r.field][r.prec];
            c.launches++;
            c.ms += ms;
            c.bytes += r.bytes;
            c.flops += r.flops;
            g_timing.pool.push_back(r.a);
            g_timing.pool.push_back(r.b);
        }
        g_timing.recs.clear();
        if (out) std::memcpy(out, t, sizeof(t));
    });
}

hts_status hts_apply_operator(hts_mesh *m, hts_field field, hts_precision prec, double dt, const void *x_dev,
                              void *y_dev)
{
    return guard_call([&] {
        check_ready(m);
        if (field != 0 && field != 1) throw Error(HTS_ERR_ARG, "bad field");
        if (prec != HTS_FP64 && prec != HTS_FP32) throw Error(HTS_ERR_ARG, "bad precision");
        if (!x_dev || !y_dev || x_dev == y_dev) throw Error(HTS_ERR_ARG, "x and y must be distinct device buffers");
        HTS_HIP(hipSetDevice(m->desc.device));
        auto B = solo_batch(m);
        Batch &b = *B;
        std::vector<int32_t> all(1, 1);
        b.set_active(all);
        const bool steady = field == 0 && (dt <= 0.0 || m->B <= 0.0);
        Tables &t = b.apply_tables(field, dt, steady);
        if (field == 1) {
            HTS_HIP(hipMemcpyAsync(b.P1.p, m->P.p, m->nnode * sizeof(double), hipMemcpyDeviceToDevice, b.s));
            VecCtx v = b.vctx(false);
            vpiezo32(v, b.massH.d64.p, b.P1.p, b.P32.p);
            std::vector<double> tn(1, m->t + dt), fs(1, dt);
            b.set_time(tn, fs);
            launch_source_values(b.lsrc.p, b.nlsrc, b.S.p, b.lcoef.p, b.s);
        }
        if (prec == HTS_FP64) {
            EpiArgs<double> ep{};
            b.apply_op<double>(t, EPI_STORE, true, (const double *)x_dev, (double *)y_dev, ep);
        } else {
            EpiArgs<float> ep{};
            b.apply_op<float>(t, EPI_STORE, true, (const float *)x_dev, (float *)y_dev, ep);
        }
    });
}

// Time the fine-level operators of each mesh for several z-chunk depths
// (the depth of node planes one workgroup marches through) and keep the
// fastest per (degree, field, node dims).
hts_status hts_autotune(hts_mesh *const *meshes, int32_t n)
{
    return guard_call([&] {
        if (!meshes || n < 1) throw Error(HTS_ERR_ARG, "no meshes");
        for (int i = 0; i < n; i++) check_ready(meshes[i]);
        tuned_zc(1, 0, 0, 0, 0, 0);   // load the cache file once
        for (int i = 0; i < n; i++) {
            hts_mesh *m = meshes[i];
            HTS_HIP(hipSetDevice(m->desc.device));
            auto B = solo_batch(m);
            Batch &b = *B;
            const double dt = 86400.0;
            HTS_HIP(hipMemcpyAsync(b.P1.p, m->P.p, m->nnode * sizeof(double), hipMemcpyDeviceToDevice, b.s));
            std::vector<int32_t> all(1, 1);
            b.set_active(all);
            VecCtx v = b.vctx(false);
            vpiezo32(v, b.massH.d64.p, b.P1.p, b.P32.p);
            std::vector<double> tn(1, m->t + dt), fs(1, dt);
            b.set_time(tn, fs);
            launch_source_values(b.lsrc.p, b.nlsrc, b.S.p, b.lcoef.p, b.s);
            vfill<double>(v, b.inner_x.p, 1.0);
            vfill<float>(v, b.x32.p, 1.0f);
            hipEvent_t e0, e1, e2;
            HTS_HIP(hipEventCreate(&e0));
            HTS_HIP(hipEventCreate(&e1));
            HTS_HIP(hipEventCreate(&e2));
            for (int f = 0; f < 2; f++) {
                Tables &t = b.apply_tables(f, dt, f == 0 && m->B <= 0.0);
                const int cands[] = {2, 3, 4, 5, 6, 8, 10, 12, 16, 24, 32, 48, 64};
                double best[2] = {1e30, 1e30};
                int bz[2] = {0, 0};
                std::vector<int> tried;
                for (int zc : cands) {
                    if (zc > m->N[2] && bz[0] > 0) break;
                    // Q2 depths are rounded up to whole cell layers
                    const int eff = zc_for(m, f, 0, 1, zc);
                    if (std::find(tried.begin(), tried.end(), eff) != tried.end()) continue;
                    tried.push_back(eff);
                    b.zc_force[f][0] = b.zc_force[f][1] = zc;
                    b.build_work();
                    EpiArgs<double> e64{};
                    e64.b = b.inner_x.p;
                    EpiArgs<float> e32{};
                    e32.b = b.x32.p;
                    for (int w = 0; w < 2; w++) {
                        b.apply_op<double>(t, EPI_RESID, true, b.inner_x.p, b.y.p, e64);
                        b.apply_op<float>(t, EPI_RESID, true, b.x32.p, b.y32.p, e32);
                    }
                    // each precision timed on its own (their kernels differ in
                    // registers and occupancy, so their best depths differ)
                    HTS_HIP(hipEventRecord(e0, b.s));
                    for (int r = 0; r < 10; r++) b.apply_op<double>(t, EPI_RESID, true, b.inner_x.p, b.y.p, e64);
                    HTS_HIP(hipEventRecord(e1, b.s));
                    for (int r = 0; r < 10; r++) b.apply_op<float>(t, EPI_RESID, true, b.x32.p, b.y32.p, e32);
                    HTS_HIP(hipEventRecord(e2, b.s));
                    HTS_HIP(hipEventSynchronize(e2));
                    float ms[2] = {0.0f, 0.0f};
                    HTS_HIP(hipEventElapsedTime(&ms[0], e0, e1));
                    HTS_HIP(hipEventElapsedTime(&ms[1], e1, e2));
                    static const bool verbose = env_or("HTS_VERBOSE", 0.0) > 0.0;
                    if (verbose)
                        std::fprintf(stderr, "[hts] autotune q%d field %d %dx%dx%d z-depth %d: %d blocks, %.2f us FP64, "
                                     "%.2f us FP32\n", m->p, f, m->N[0], m->N[1], m->N[2], zc, b.nwork[f][0],
                                     100.0 * ms[0], 100.0 * ms[1]);
                    for (int pr = 0; pr < 2; pr++)
                        if (ms[pr] < best[pr]) {
                            best[pr] = ms[pr];
                            bz[pr] = zc;
                        }
                }
                b.zc_force[f][0] = b.zc_force[f][1] = 0;
                for (int pr = 0; pr < 2; pr++)
                    set_tuned_zc(kernel_degree(m), f, pr, m->N[0], m->N[1], m->N[2], bz[pr]);
            }
            (void)hipEventDestroy(e2);
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
        }
        save_tuning();
        for (int i = 0; i < n; i++) forget_batches(meshes[i]);
    });
}

hts_status hts_solve_steady_pressure(hts_mesh *m, const hts_solver_opts *opts, hts_step_stats *stats)
{
    return guard_call([&] {
        check_ready(m);
        HTS_HIP(hipSetDevice(m->desc.device));
        hts_solver_opts o = opts_or_default(opts);
        if (o.mode == HTS_MODE_LEARNED) o.mode = HTS_MODE_FP64;
        auto B = solo_batch(m);
        B->gather_state();
        FieldStats st = B->solve_pressure(0.0, true, o);
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            stats->iters[0] = st.iters[0];
            stats->outer[0] = st.outer[0];
            stats->relres[0] = st.relres[0];
            stats->status[0] = st.status[0];
            stats->time_ms[0] = st.ms;
        }
        if (st.status[0] != HTS_OK) throw Error(st.status[0], "steady pressure solve failed");
        HTS_HIP(hipMemcpyAsync(m->P.p, B->P1.p, m->nnode * sizeof(double), hipMemcpyDeviceToDevice, B->s));
        HTS_HIP(hipStreamSynchronize(B->s));
        m->has_state[0] = true;
        m->hist_dt[0] = m->hist_dt2[0] = 0.0;   // not a time step: no previous levels
    });
}

hts_status hts_solve_step(hts_mesh *m, double dt, const hts_solver_opts *opts, hts_step_stats *stats)
{
    return guard_call([&] {
        check_ready(m);
        if (!(dt > 0.0)) throw Error(HTS_ERR_ARG, "dt must be > 0");
        HTS_HIP(hipSetDevice(m->desc.device));
        hts_solver_opts o = opts_or_default(opts);
        auto B = solo_batch(m);
        B->gather_state();
        std::vector<hts_step_stats> st;
        int rc = B->step(dt, o, &st);
        if (stats) *stats = st[0];
        if (rc == HTS_OK) B->scatter_state();
        if (rc != HTS_OK) throw Error(rc, "time step did not converge");
    });
}

hts_status hts_advance(hts_mesh *const *meshes, int32_t n, int32_t n_steps, double dt, const hts_solver_opts *opts,
                       hts_step_stats *stats)
{
    return guard_call([&] {
        if (!meshes || n < 1) throw Error(HTS_ERR_ARG, "no meshes");
        if (n_steps < 0) throw Error(HTS_ERR_ARG, "n_steps must be >= 0");
        if (!(dt > 0.0)) throw Error(HTS_ERR_ARG, "dt must be > 0");
        std::vector<hts_mesh *> ms(meshes, meshes + n);
        for (hts_mesh *m : ms) check_ready(m);
        {
            std::vector<hts_mesh *> u = ms;
            std::sort(u.begin(), u.end());
            if (std::adjacent_find(u.begin(), u.end()) != u.end()) throw Error(HTS_ERR_ARG, "a mesh appears twice");
        }
        HTS_HIP(hipSetDevice(ms[0]->desc.device));
        hts_solver_opts o = opts_or_default(opts);
        std::shared_ptr<Batch> B = n == 1 ? solo_batch(ms[0]) : multi_batch(ms);
        B->gather_state();
        std::vector<hts_step_stats> st;
        int rc = HTS_OK;
        for (int k = 0; k < n_steps; k++) {
            rc = B->step(dt, o, &st);
            if (rc != HTS_OK) break;
        }
        B->scatter_state();
        if (stats && !st.empty())
            for (int i = 0; i < n; i++) stats[i] = st[i];
        if (rc != HTS_OK) throw Error(rc, "a time step did not converge");
    });
}

}  // extern "C"

namespace hts {
template void Batch::apply_op<double>(const Tables &, int, bool, const double *, double *, EpiArgs<double>);
}  // namespace hts
