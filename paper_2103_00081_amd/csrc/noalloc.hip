// hts_apply_operator without device allocation: every buffer the apply needs
// beyond the mesh's own data and the caller's x and y (the operator
// descriptors, the work list, the time slots and line-source coefficients of
// the heat operator, and the FP32 piezometric pressure it reads) lives in one
// statically sized device array per GPU.  For callers that cannot allocate
// (code under graph capture, tight loops, harnesses that forbid it).
#include <cstring>
#include <functional>
#include <mutex>

#include "bc.h"
#include "internal.h"
#include "vec.h"

namespace hts {
hts_status guard_call(const std::function<void()> &f);
template <typename T>
void launch_apply(int degree, int field, int epi, bool masked, bool graded, const OpDev *ops, const WorkItem *work,
                  int nwork, const T *x, T *y, const EpiArgs<T> &ep, hipStream_t s);

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)40 << 20;   // 40 MiB per GPU
// Device scratch of the allocation-free entry point.  In host code this name
// is a host-side stand-in: only the address returned by hipGetSymbolAddress
// (kept per device in g_ptr) is passed to kernels and copies.
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEV = 64;
std::mutex g_mu;
unsigned char *g_ptr[MAX_DEV] = {};

unsigned char *scratch_ptr(int dev)
{
    if (dev < 0 || dev >= MAX_DEV) throw Error(HTS_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw Error(HTS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_ptr[dev] = static_cast<unsigned char *>(p);
    }
    return g_ptr[dev];
}

// Small host structures reach the device as kernel arguments (no host
// buffer, no copy engine): one blob of up to 2 KiB per launch.
constexpr int BLOB = 2048;
struct Blob {
    unsigned char b[BLOB];
};

__global__ void k_put(unsigned char *__restrict__ dst, Blob blob, int nbytes)
{
    for (int i = threadIdx.x; i < nbytes; i += blockDim.x) dst[i] = blob.b[i];
}

void put(unsigned char *dst, const void *src, size_t nbytes, hipStream_t s)
{
    const unsigned char *p = static_cast<const unsigned char *>(src);
    for (size_t o = 0; o < nbytes; o += BLOB) {
        Blob b;
        const int n = (int)std::min<size_t>(BLOB, nbytes - o);
        std::memcpy(b.b, p + o, (size_t)n);
        k_put<<<dim3(1), dim3(256), 0, s>>>(dst + o, b, n);
        HTS_LAUNCH_CHECK();
    }
}

// work item w: tile (w % ntx, (w / ntx) % nty), node planes [z0, z0 + zc)
__global__ void k_make_work(WorkItem *__restrict__ w, int ntx, int nty, int zc, int NZ, int total)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= total) return;
    WorkItem it{};
    it.inst = 0;
    it.tx = b % ntx;
    it.ty = (b / ntx) % nty;
    it.z0 = (b / (ntx * nty)) * zc;
    it.z1 = min(NZ, it.z0 + zc);
    it.slot = b;
    w[b] = it;
}

// chunk c: nodes [c * len, min(n, (c + 1) * len)) of instance 0
__global__ void k_make_chunks(Chunk *__restrict__ c, int64_t n, int64_t len, int nchunk)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nchunk) return;
    Chunk ch{};
    ch.inst = 0;
    ch.beg = (int64_t)i * len;
    ch.end = min(n, ch.beg + len);
    c[i] = ch;
}

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace
}  // namespace hts

using namespace hts;

extern "C" hts_status hts_apply_operator_noalloc(hts_mesh *m, hts_field field, hts_precision prec, double dt,
                                                 const void *x_dev, void *y_dev)
{
    return guard_call([&] {
        if (!m) throw Error(HTS_ERR_ARG, "null mesh");
        if (!m->has_mat) throw Error(HTS_ERR_STATE, "materials not set");
        if (m->dirty)
            throw Error(HTS_ERR_STATE, "mesh data not prepared: call hts_apply_operator, hts_autotune or a solve "
                                       "once after changing the mesh");
        if (field != 0 && field != 1) throw Error(HTS_ERR_ARG, "bad field");
        if (prec != HTS_FP64 && prec != HTS_FP32) throw Error(HTS_ERR_ARG, "bad precision");
        if (!x_dev || !y_dev || x_dev == y_dev) throw Error(HTS_ERR_ARG, "x and y must be distinct device buffers");
        if (field == 1 && !m->has_state[0]) throw Error(HTS_ERR_STATE, "pressure state not set");
        const hipStream_t s = m->stream;
        const bool fp32 = prec == HTS_FP32;
        const bool steady = field == 0 && (dt <= 0.0 || m->B <= 0.0);
        const int ox = tile_own_x(kernel_degree(m), field), oy = tile_own_y(kernel_degree(m), field);
        const int ntx = (m->N[0] + ox - 1) / ox, nty = (m->N[1] + oy - 1) / oy;
        const int zc = zc_for(m, field, fp32 ? 1 : 0, (int64_t)ntx * nty, 0);
        const int64_t nzc = (m->N[2] + zc - 1) / zc;
        const int64_t nwork = (int64_t)ntx * nty * nzc;
        const int nsrc = field == 1 ? (int)m->line_srcs.size() : 0;
        const int64_t clen = 1024;
        const int64_t nchunk = (field == 1 && fp32) ? (m->nnode + clen - 1) / clen : 0;
        // layout, 256-byte aligned pieces
        size_t o = 0;
        const size_t o_ops = o;    o += up256(2 * sizeof(OpDev));
        const size_t o_S = o;      o += up256(NSLOT * sizeof(double));
        const size_t o_src = o;    o += up256((size_t)std::max(1, nsrc) * sizeof(SrcDev));
        const size_t o_coef = o;   o += up256((size_t)std::max(1, nsrc) * sizeof(double));
        const size_t o_work = o;   o += up256((size_t)nwork * sizeof(WorkItem));
        const size_t o_chunk = o;  o += up256((size_t)nchunk * sizeof(Chunk));
        const size_t o_p32 = o;    o += up256((size_t)(nchunk ? m->nnode : 0) * sizeof(float));
        if (o > SCRATCH_BYTES || nwork > INT32_MAX)
            throw Error(HTS_ERR_ARG, "mesh too large for the allocation-free apply: needs " + std::to_string(o) +
                                         " bytes of the " + std::to_string(SCRATCH_BYTES) + "-byte scratch");
        HTS_HIP(hipSetDevice(m->desc.device));
        unsigned char *base = scratch_ptr(m->desc.device);
        OpDev *ops = reinterpret_cast<OpDev *>(base + o_ops);
        double *S = reinterpret_cast<double *>(base + o_S);
        SrcDev *srcs = reinterpret_cast<SrcDev *>(base + o_src);
        double *coef = reinterpret_cast<double *>(base + o_coef);
        WorkItem *work = reinterpret_cast<WorkItem *>(base + o_work);
        Chunk *chunks = reinterpret_cast<Chunk *>(base + o_chunk);
        float *P32 = reinterpret_cast<float *>(base + o_p32);

        // descriptors: [0] FP64, [1] FP32, as the solo batch builds them
        OpDev h[2];
        for (int q = 0; q < 2; q++) {
            h[q] = make_op(m, field, q == 1, dt, steady, false);
            h[q].off = 0;
            if (field == 1) {
                h[q].P = q == 1 ? (const void *)(nchunk ? P32 : nullptr) : (const void *)m->P.p;
                h[q].lcoef = coef;
                if (q == 1) h[q].rho_g = 0.0;   // the FP32 pressure is piezometric
            }
        }
        put(base + o_ops, h, sizeof(h), s);
        k_make_work<<<dim3((unsigned)((nwork + 255) / 256)), dim3(256), 0, s>>>(work, ntx, nty, zc, m->N[2],
                                                                               (int)nwork);
        HTS_LAUNCH_CHECK();
        if (field == 1) {
            // time slots of instance 0, then the line-source coefficients at t + dt
            double hS[NSLOT];
            for (int i = 0; i < NSLOT; i++) hS[i] = 0.0;
            hS[S_TNEW] = m->t + dt;
            hS[S_FSCALE] = dt;
            put(base + o_S, hS, sizeof(hS), s);
            if (nsrc > 0) {
                std::vector<SrcDev> ls(m->line_srcs);
                for (SrcDev &sd : ls) sd.inst = 0;
                put(base + o_src, ls.data(), ls.size() * sizeof(SrcDev), s);
                launch_source_values(srcs, nsrc, S, coef, s);
            }
            if (nchunk) {
                k_make_chunks<<<dim3((unsigned)((nchunk + 255) / 256)), dim3(256), 0, s>>>(chunks, m->nnode, clen,
                                                                                         (int)nchunk);
                HTS_LAUNCH_CHECK();
                VecCtx v{chunks, (int)nchunk, nullptr, S, s};
                vpiezo32(v, ops, m->P.p, P32);
            }
        }
        if (!fp32) {
            EpiArgs<double> ep{};
            launch_apply<double>(kernel_degree(m), field, EPI_STORE, true, m->graded, ops, work, (int)nwork,
                                 static_cast<const double *>(x_dev), static_cast<double *>(y_dev), ep, s);
        } else {
            EpiArgs<float> ep{};
            launch_apply<float>(kernel_degree(m), field, EPI_STORE, true, m->graded, ops + 1, work, (int)nwork,
                                static_cast<const float *>(x_dev), static_cast<float *>(y_dev), ep, s);
        }
    });
}
