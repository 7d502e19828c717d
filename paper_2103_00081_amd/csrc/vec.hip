// Vector kernels of the Krylov solvers over batched (concatenated) vectors.
//
// A batch vector holds the nodes of all instances back to back.  It is cut
// into chunks that never straddle an instance; one 256-thread block handles
// one chunk, so per-instance scalars (alpha, beta, ...) are read once per
// block.  Dot products are two-stage and deterministic: each block writes
// one FP64 partial per component, then k_reduce sums an instance's partials
// in a fixed order and applies the solver's scalar update.  Inactive
// (converged) instances are skipped by every kernel.
#include "common.h"
#include "dev_util.h"
#include "vec.h"

#include <algorithm>

namespace hts {

namespace {

constexpr int VB = 256;

// A chunk holds at most EPT * VB nodes, so a thread has at most EPT of them:
// e[u] = beg + tid + u VB, present if below end.  The kernels read all of a
// thread's operands before they store anything, at indices clamped to the
// chunk's last node (c[u]), so every load can be in flight at once; values
// of absent nodes are dropped.
constexpr int EPT = 4;
static_assert(CHUNK_LEN <= EPT * VB && CHUNK_LEN_COARSE <= EPT * VB, "chunks longer than EPT nodes per thread");

struct Lanes {
    int64_t e[EPT], c[EPT];
    bool in[EPT];
};

__device__ __forceinline__ Lanes chunk_lanes(const Chunk &ch)
{
    Lanes l;
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        l.e[u] = ch.beg + threadIdx.x + u * VB;
        l.in[u] = l.e[u] < ch.end;
        l.c[u] = l.in[u] ? l.e[u] : ch.end - 1;
    }
    return l;
}

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return r;
}

#define CHUNK_PROLOGUE                                                   \
    const Chunk ch = chunks[blockIdx.x];                                 \
    if (active && !active[ch.inst]) return;                              \
    const double *Si = S + (int64_t)ch.inst * NSLOT;                     \
    (void)Si;

template <typename T>
__global__ __launch_bounds__(VB) void k_fill(const Chunk *__restrict__ chunks, const int32_t *active,
                                             const double *S, T *__restrict__ y, T v)
{
    CHUNK_PROLOGUE
    for (int64_t e = ch.beg + threadIdx.x; e < ch.end; e += VB) y[e] = v;
}

template <typename T>
__global__ __launch_bounds__(VB) void k_copy(const Chunk *__restrict__ chunks, const int32_t *active,
                                             const double *S, const T *__restrict__ x, T *__restrict__ y)
{
    CHUNK_PROLOGUE
    const Lanes l = chunk_lanes(ch);
    T v[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) v[u] = x[l.c[u]];
#pragma unroll
    for (int u = 0; u < EPT; u++)
        if (l.in[u]) y[l.e[u]] = v[u];
}

// y = a * x + b * y with a = sa * S[ia] (ia < 0: a = sa), same for b
template <typename T>
__global__ __launch_bounds__(VB) void k_axpby(const Chunk *__restrict__ chunks, const int32_t *active,
                                              const double *S, double sa, int ia, const T *__restrict__ x,
                                              double sb, int ib, T *__restrict__ y)
{
    CHUNK_PROLOGUE
    const T a = T(ia >= 0 ? sa * Si[ia] : sa);
    const T b = T(ib >= 0 ? sb * Si[ib] : sb);
    const Lanes l = chunk_lanes(ch);
    T xv[EPT], yv[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) xv[u] = x[l.c[u]];
    if (b == T(0)) {
#pragma unroll
        for (int u = 0; u < EPT; u++)
            if (l.in[u]) y[l.e[u]] = a * xv[u];
    } else {
#pragma unroll
        for (int u = 0; u < EPT; u++) yv[u] = y[l.c[u]];
#pragma unroll
        for (int u = 0; u < EPT; u++)
            if (l.in[u]) y[l.e[u]] = a * xv[u] + b * yv[u];
    }
}

// z = d .* r (Jacobi)
template <typename T>
__global__ __launch_bounds__(VB) void k_jacobi(const Chunk *__restrict__ chunks, const int32_t *active,
                                               const double *S, double c, int ic, const T *__restrict__ d,
                                               const T *__restrict__ r, T *__restrict__ z)
{
    CHUNK_PROLOGUE
    const T a = T(ic >= 0 ? c * Si[ic] : c);
    const Lanes l = chunk_lanes(ch);
    T dv[EPT], rv[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        dv[u] = d[l.c[u]];
        rv[u] = r[l.c[u]];
    }
#pragma unroll
    for (int u = 0; u < EPT; u++)
        if (l.in[u]) z[l.e[u]] = a * dv[u] * rv[u];
}

// partial[blk*2 + 0] = x.y (and partial[blk*2+1] = x.w if w)
template <typename T>
__global__ __launch_bounds__(VB) void k_dot(const Chunk *__restrict__ chunks, const int32_t *active,
                                            const double *S, const T *__restrict__ x, const T *__restrict__ y,
                                            const T *__restrict__ w, double *partial)
{
    __shared__ double sh[4];
    CHUNK_PROLOGUE
    double a = 0.0, b = 0.0;
    const Lanes l = chunk_lanes(ch);
    T xv[EPT], yv[EPT], wv[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        xv[u] = x[l.c[u]];
        yv[u] = y[l.c[u]];
        wv[u] = w ? w[l.c[u]] : T(0);
    }
#pragma unroll
    for (int u = 0; u < EPT; u++)
        if (l.in[u]) {
            const double xe = (double)xv[u];
            a += xe * (double)yv[u];
            if (w) b += xe * (double)wv[u];
        }
    a = block_sum(a, sh);
    if (w) b = block_sum(b, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = a;
        partial[2 * blockIdx.x + 1] = b;
    }
}

// CG: x += alpha p; r -= alpha q; (r_old = r before); partial = r.r
template <typename T>
__global__ __launch_bounds__(VB) void k_cg_update(const Chunk *__restrict__ chunks, const int32_t *active,
                                                  const double *S, T *__restrict__ x, T *__restrict__ r,
                                                  const T *__restrict__ p, const T *__restrict__ q,
                                                  T *__restrict__ r_old, double *partial)
{
    __shared__ double sh[4];
    CHUNK_PROLOGUE
    const T al = T(Si[S_ALPHA]);
    double a = 0.0;
    const Lanes l = chunk_lanes(ch);
    T xv[EPT], rv[EPT], pv[EPT], qv[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        xv[u] = x[l.c[u]];
        rv[u] = r[l.c[u]];
        pv[u] = p[l.c[u]];
        qv[u] = q[l.c[u]];
    }
#pragma unroll
    for (int u = 0; u < EPT; u++)
        if (l.in[u]) {
            const int64_t e = l.e[u];
            x[e] = xv[u] + al * pv[u];
            T re = rv[u];
            if (r_old) r_old[e] = re;
            re -= al * qv[u];
            r[e] = re;
            a += (double)re * (double)re;
        }
    a = block_sum(a, sh);
    if (threadIdx.x == 0) partial[2 * blockIdx.x] = a;
}

// GMRES: multi-dot h_i = V_i . w for i < nv (V_i = V + i*ld)
// Sums over the block of NC per-thread values at once (component c in
// a[c], c < nc): each wave reduces by shuffles, then thread c adds the four
// wave sums in wave order and writes out[c].  Fixed order: deterministic.
template <int NC>
__device__ __forceinline__ void block_multi_sum(const double (&a)[NC], int nc, double (*sh)[NC], double *out)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NC; c++) {
        if (c < nc) {
            const double v = wave_sum(a[c]);
            if (lane == 0) sh[w][c] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) {
        const int c = threadIdx.x;
        out[c] = (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]);
    }
}

// The basis kernels also clamp the vector index to nv - 1; the clamped
// terms are discarded by their factors (0 weight, 0 coefficient) or by never
// being written out, so the sums keep the order of the plain loop.

// Partials of V_i . w (i < nv) in one pass over the chunk: every thread
// keeps NB running sums (NB >= nv, compile-time bucket; sums i >= nv are
// not written out).
template <typename T, int NB>
__global__ __launch_bounds__(VB) void k_multidot(const Chunk *__restrict__ chunks, const int32_t *active,
                                                 const double *S, const T *__restrict__ V, int64_t ld,
                                                 int nv, const T *__restrict__ w, double *partial,
                                                 int ncomp)
{
    __shared__ double sh[4][NB];
    CHUNK_PROLOGUE
    double a[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) a[i] = 0.0;
    const int64_t last = ch.end - 1;
    constexpr int UN = NB <= 16 ? EPT : 1;
#pragma unroll UN
    for (int u = 0; u < EPT; u++) {
        const int64_t e = ch.beg + threadIdx.x + u * VB;
        const int64_t ec = e < ch.end ? e : last;
        const double we = e < ch.end ? (double)w[ec] : 0.0;
#pragma unroll
        for (int i = 0; i < NB; i++) a[i] += (double)V[(int64_t)(i < nv ? i : nv - 1) * ld + ec] * we;
    }
    block_multi_sum<NB>(a, nv, sh, partial + (int64_t)blockIdx.x * ncomp);
}

// GMRES: w -= sum_i h_i V_i (h per instance: H + inst*hld), then partials of
// V_i . w (i < nv, if dots) and w . w (component nv, or 0 without dots),
// taken on the stored (type T) values of the new w in the same pass.
template <typename T, int NB>
__global__ __launch_bounds__(VB) void k_orth_update(const Chunk *__restrict__ chunks, const int32_t *active,
                                                    const double *S, const T *__restrict__ V, int64_t ld,
                                                    int nv, const double *__restrict__ H, int hld,
                                                    T *__restrict__ w, int dots, double *partial,
                                                    int ncomp, int scale_slot)
{
    __shared__ double sh[4][NB + 1];
    __shared__ double hs[NB];
    CHUNK_PROLOGUE
    if (threadIdx.x < NB) hs[threadIdx.x] = (int)threadIdx.x < nv ? H[(int64_t)ch.inst * hld + threadIdx.x] : 0.0;
    __syncthreads();
    const double sc = scale_slot >= 0 ? Si[scale_slot] : 1.0;
    double a[NB], aw = 0.0;
#pragma unroll
    for (int i = 0; i < NB; i++) a[i] = 0.0;
    const bool sums = partial != nullptr;
    const int64_t last = ch.end - 1;
    constexpr int UN = NB <= 16 ? EPT : 1;
#pragma unroll UN
    for (int u = 0; u < EPT; u++) {
        const int64_t e = ch.beg + threadIdx.x + u * VB;
        const bool in = e < ch.end;
        const int64_t ec = in ? e : last;
        double v[NB];
        double acc = (double)w[ec];
#pragma unroll
        for (int i = 0; i < NB; i++) {
            v[i] = (double)V[(int64_t)(i < nv ? i : nv - 1) * ld + ec];
            acc -= hs[i] * v[i];
        }
        const T wn = T(scale_slot >= 0 ? acc * sc : acc);
        if (in) w[e] = wn;
        if (sums && in) {
            const double wd = (double)wn;
            if (dots) {
                // long bases read V again (cache hits) rather than hold it
                if constexpr (NB > 24) asm volatile("" ::: "memory");
#pragma unroll
                for (int i = 0; i < NB; i++)
                    a[i] += (NB > 24 ? (double)V[(int64_t)(i < nv ? i : nv - 1) * ld + ec] : v[i]) * wd;
            }
            aw += wd * wd;
        }
    }
    if (!sums) return;
    // components: the nv dots (if dots), then w . w; wave sums into sh[w][c]
    // (w . w at column NB), then thread c adds the four waves in order
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (dots) {
#pragma unroll
        for (int c = 0; c < NB; c++)
            if (c < nv) {
                const double r = wave_sum(a[c]);
                if (lane == 0) sh[wv][c] = r;
            }
    }
    {
        const double r = wave_sum(aw);
        if (lane == 0) sh[wv][NB] = r;
    }
    __syncthreads();
    const int nd = dots ? nv : 0;
    double *out = partial + (int64_t)blockIdx.x * ncomp;
    if ((int)threadIdx.x < nd) {
        const int c = threadIdx.x;
        out[c] = (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]);
    } else if ((int)threadIdx.x == nd) {
        out[nd] = (sh[0][NB] + sh[1][NB]) + (sh[2][NB] + sh[3][NB]);
    }
}

// x += sum_{i < kdim[inst]} y_i Z_i   (y per instance: Y + inst*yld)
template <typename T, typename TX>
__global__ __launch_bounds__(VB) void k_basis_update(const Chunk *__restrict__ chunks, const int32_t *active,
                                                     const double *S, const T *__restrict__ Z, int64_t ld,
                                                     const int32_t *kdim, const double *__restrict__ Yc,
                                                     int yld, double scale, int iscale, TX *__restrict__ x)
{
    __shared__ double ys[64];
    const Chunk ch = chunks[blockIdx.x];
    if (active && !active[ch.inst]) return;
    const int kd = kdim[ch.inst];
    const double sc = iscale >= 0 ? scale * S[(int64_t)ch.inst * NSLOT + iscale] : scale;
    if (threadIdx.x < kd) ys[threadIdx.x] = Yc[(int64_t)ch.inst * yld + threadIdx.x] * sc;
    __syncthreads();
    for (int64_t e = ch.beg + threadIdx.x; e < ch.end; e += VB) {
        double acc = 0.0;
        for (int i = 0; i < kd; i++) acc += ys[i] * (double)Z[(int64_t)i * ld + e];
        x[e] = TX((double)x[e] + acc);
    }
}

// y (type TY) = c * x (type TX), c = sc * S[ic] or sc
template <typename TX, typename TY>
__global__ __launch_bounds__(VB) void k_convert(const Chunk *__restrict__ chunks, const int32_t *active,
                                                const double *S, double sc, int ic, const TX *__restrict__ x,
                                                TY *__restrict__ y)
{
    CHUNK_PROLOGUE
    const double c = ic >= 0 ? sc * Si[ic] : sc;
    const Lanes l = chunk_lanes(ch);
    TX xv[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) xv[u] = x[l.c[u]];
#pragma unroll
    for (int u = 0; u < EPT; u++)
        if (l.in[u]) y[l.e[u]] = TY(c * (double)xv[u]);
}

// x (FP64) += c * d (type T)
template <typename T>
__global__ __launch_bounds__(VB) void k_add_scaled(const Chunk *__restrict__ chunks, const int32_t *active,
                                                   const double *S, double sc, int ic, const T *__restrict__ d,
                                                   double *__restrict__ x)
{
    CHUNK_PROLOGUE
    const double c = ic >= 0 ? sc * Si[ic] : sc;
    const Lanes l = chunk_lanes(ch);
    T dv[EPT];
    double xv[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        dv[u] = d[l.c[u]];
        xv[u] = x[l.c[u]];
    }
#pragma unroll
    for (int u = 0; u < EPT; u++)
        if (l.in[u]) x[l.e[u]] = xv[u] + c * (double)dv[u];
}

// Initial guess from the last time levels: x = Xn + c1 (Xn - Xp) +
// c2 (Xp - Xpp), c1 = S[slot1], c2 = S[slot2] of the instance; with both 0
// it copies Xn (the older levels are then not read); constrained nodes of
// ops (if given) get 0.
__global__ __launch_bounds__(VB) void k_extrapolate(const Chunk *__restrict__ chunks, const int32_t *active,
                                                    const double *S, int slot1, int slot2,
                                                    const OpDev *__restrict__ ops, const double *__restrict__ Xn,
                                                    const double *__restrict__ Xp, const double *__restrict__ Xpp,
                                                    double *__restrict__ x)
{
    CHUNK_PROLOGUE
    const double c1 = Si[slot1], c2 = Si[slot2];
    const bool lin = c1 != 0.0 || c2 != 0.0, quad = c2 != 0.0;
    const Lanes l = chunk_lanes(ch);
    double a[EPT], b[EPT], q[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        a[u] = Xn[l.c[u]];
        b[u] = lin ? Xp[l.c[u]] : 0.0;
        q[u] = quad ? Xpp[l.c[u]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < EPT; u++)
        if (l.in[u]) {
            double v = a[u];
            if (lin) v = a[u] + c1 * (a[u] - b[u]);
            if (quad) v += c2 * (b[u] - q[u]);
            if (ops) {
                const OpDev &o = ops[ch.inst];
                if (node_constrained(o, l.e[u] - o.off)) v = 0.0;
            }
            x[l.e[u]] = v;
        }
}

// Right-hand side assembly: b = (b - y) + c ld, c = S[slot] of the instance
__global__ __launch_bounds__(VB) void k_rhs_combine(const Chunk *__restrict__ chunks, const int32_t *active,
                                                    const double *S, const double *__restrict__ y,
                                                    const double *__restrict__ ld, int slot, double *__restrict__ b)
{
    CHUNK_PROLOGUE
    const double c = Si[slot];
    const Lanes l = chunk_lanes(ch);
    double bv[EPT], yv[EPT], lv[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        bv[u] = b[l.c[u]];
        yv[u] = y[l.c[u]];
        lv[u] = ld[l.c[u]];
    }
#pragma unroll
    for (int u = 0; u < EPT; u++)
        if (l.in[u]) b[l.e[u]] = c * lv[u] + (bv[u] - yv[u]);
}

// z = x + y
__global__ __launch_bounds__(VB) void k_add(const Chunk *__restrict__ chunks, const int32_t *active,
                                            const double *S, const double *__restrict__ x,
                                            const double *__restrict__ y, double *__restrict__ z)
{
    CHUNK_PROLOGUE
    const Lanes l = chunk_lanes(ch);
    double xv[EPT], yv[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        xv[u] = x[l.c[u]];
        yv[u] = y[l.c[u]];
    }
#pragma unroll
    for (int u = 0; u < EPT; u++)
        if (l.in[u]) z[l.e[u]] = xv[u] + yv[u];
}

// Xpp = Xp, Xp = Xn, Xn = X1 (commit of a step, keeping two older levels)
__global__ __launch_bounds__(VB) void k_shift(const Chunk *__restrict__ chunks, const int32_t *active,
                                              const double *S, const double *__restrict__ X1,
                                              double *__restrict__ Xn, double *__restrict__ Xp,
                                              double *__restrict__ Xpp)
{
    CHUNK_PROLOGUE
    const Lanes l = chunk_lanes(ch);
    double a[EPT], b[EPT], c[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        a[u] = X1[l.c[u]];
        b[u] = Xn[l.c[u]];
        c[u] = Xp[l.c[u]];
    }
#pragma unroll
    for (int u = 0; u < EPT; u++)
        if (l.in[u]) {
            Xpp[l.e[u]] = c[u];
            Xp[l.e[u]] = b[u];
            Xn[l.e[u]] = a[u];
        }
}

// y[n] = v at constrained nodes of instance (n in chunk), others untouched
template <typename T>
__global__ __launch_bounds__(VB) void k_mask(const Chunk *__restrict__ chunks, const int32_t *active,
                                             const double *S, const OpDev *__restrict__ ops,
                                             T *__restrict__ y, T v)
{
    CHUNK_PROLOGUE
    const OpDev &o = ops[ch.inst];
    for (int64_t e = ch.beg + threadIdx.x; e < ch.end; e += VB)
        if (node_constrained(o, e - o.off)) y[e] = v;
}

// FP32 pressure for the heat operator in piezometric form:
// P32 = (P - P[node 0]) + rho_w g z, so that q = -k grad(P32) without the
// cancellation between grad P and rho_w g e_z.
__global__ __launch_bounds__(VB) void k_piezo32(const Chunk *__restrict__ chunks, const OpDev *__restrict__ ops,
                                                const double *__restrict__ P, float *__restrict__ P32)
{
    const Chunk ch = chunks[blockIdx.x];
    const OpDev &o = ops[ch.inst];
    const double ref = P[o.off];
    const double dz = o.hz / o.p;
    const int64_t pl = (int64_t)o.NX * o.NY;
    for (int64_t e = ch.beg + threadIdx.x; e < ch.end; e += VB) {
        const int64_t k = (e - o.off) / pl;
        double zk = o.zn ? o.zn[k] - o.zn[0] : k * dz;
        if (o.xyz) zk = o.xyz[3 * (e - o.off) + 2] - o.xyz[2];   // general hexahedra
        P32[e] = (float)((P[e] - ref) + o.rho_g * zk);
    }
}

// ---------------------------------------------------------------- reduce
// pre: S_RZ, S_TOL2, S_ITER of the instance, read before the partial sums
__device__ void scalar_op(int op, int inst, const double *v, const double *pre, double *S, int32_t *active,
                          int maxit, int slot, double aux)
{
    double *Si = S + (int64_t)inst * NSLOT;
    auto stop = [&](int status) {
        Si[S_STATUS] = status;
        if (active) active[inst] = 0;
    };
    switch (op) {
    case RED_STORE:
        Si[slot] = v[0];
        break;
    case RED_STORE2:
        Si[slot] = v[0];
        Si[slot + 1] = v[1];
        break;
    case RED_CG_ALPHA: {
        const double pq = v[0];
        Si[S_PQ] = pq;
        if (!(pq > 0.0) || !isfinite(pq)) {
            Si[S_ALPHA] = 0.0;
            stop(-6);
        } else {
            Si[S_ALPHA] = pre[0] / pq;
        }
        break;
    }
    case RED_CG_CONV: {
        const double rr = v[0];
        const double iter = pre[2] + 1.0;
        Si[S_RR] = rr;
        Si[S_ITER] = iter;
        if (!isfinite(rr)) stop(-6);
        else if (rr <= pre[1]) stop(0);
        else if (iter >= maxit) stop(-5);
        break;
    }
    case RED_CG_BETA: {   // v0 = z.r (new), v1 = z.r_old (flexible)
        const double rzn = v[0];
        const double num = rzn - v[1];
        const double rz = pre[0];
        Si[S_BETA] = (rz != 0.0 && isfinite(num)) ? num / rz : 0.0;
        Si[S_RZ] = rzn;
        if (!isfinite(rzn)) stop(-6);
        break;
    }
    case RED_SET_TOL:     // v0 = b.b; aux = rtol^2
        Si[S_BB] = v[0];
        Si[S_TOL2] = aux * v[0];
        break;
    case RED_INVSQRT:     // S[slot] = v0, S[slot+1] = 1/sqrt(v0)
        Si[slot] = v[0];
        Si[slot + 1] = v[0] > 0.0 ? 1.0 / sqrt(v[0]) : 0.0;
        break;
    case RED_CG_INIT: {   // v0 = r.r of the initial residual
        Si[S_RR] = v[0];
        Si[S_RR0] = v[0];
        Si[S_ITER] = 0.0;
        Si[S_STATUS] = 1.0;
        if (!isfinite(v[0])) stop(-6);
        else if (v[0] <= pre[1]) stop(0);
        break;
    }
    default:
        break;
    }
}

// One block per instance.  The loads that do not depend on each other (the
// instance's flag, its segment and the scalar slots the update reads) are
// issued together, then the partial sums; a kernel of a few dependent memory
// latencies in the solver's critical path.
constexpr int RB = 1024;   // threads of the final reduction (one block per instance)
constexpr int RU = 8;      // loads in flight per thread

__global__ __launch_bounds__(RB) void k_reduce(const double *__restrict__ partial, int ncomp,
                                               const int32_t *__restrict__ seg_ptr, int single, int op,
                                               int slot, double *S, int32_t *active, int maxit, double aux,
                                               double *out, ArnArgs arn)
{
    __shared__ double vals[64];
    __shared__ double rows[RB];
    const int inst = blockIdx.x;
    const int on = active ? active[inst] : 1;
    const int b = single >= 0 ? 0 : seg_ptr[inst], n = (single >= 0 ? single : seg_ptr[inst + 1]) - b;
    double pre[3] = {0.0, 0.0, 0.0};
    if (threadIdx.x == 0) {
        const double *Si = S + (int64_t)inst * NSLOT;
        pre[0] = Si[S_RZ];
        pre[1] = Si[S_TOL2];
        pre[2] = Si[S_ITER];
    }
    // The partials are rows of ncomp values.  Thread t takes component
    // c = t % ncomp of rows r0, r0 + R, r0 + 2R, ... (r0 = t / ncomp,
    // R = RB / ncomp rows per pass), so each pass reads R * ncomp consecutive
    // values; RU loads go out together.  Then a wave per component adds the
    // R row sums in row order.  Fixed order throughout: deterministic.
    const int R = RB / ncomp;
    const int t = threadIdx.x, c = t % ncomp, r0 = t / ncomp;
    double a = 0.0;
    if (r0 < R) {
        const double *pc = partial + (int64_t)b * ncomp + c;
        for (int r = r0; r < n; r += RU * R) {
            double p[RU];
#pragma unroll
            for (int u = 0; u < RU; u++) p[u] = r + u * R < n ? pc[(int64_t)(r + u * R) * ncomp] : 0.0;
#pragma unroll
            for (int u = 0; u < RU; u++)
                if (r + u * R < n) a += p[u];
        }
    }
    rows[t] = a;
    __syncthreads();
    const int lane = t & 63, w = t >> 6;
    for (int cc = w; cc < ncomp; cc += RB / 64) {
        double v = 0.0;
        for (int r = lane; r < R; r += 64) v += rows[r * ncomp + cc];
        v = wave_sum(v);
        if (lane == 0) vals[cc] = v;
    }
    __syncthreads();
    if (!on) {   // the same for the whole block
        // a CG solve that finds the instance already inactive counts no
        // iteration for it (no stale count from an earlier solve)
        if (op == RED_CG_INIT && threadIdx.x == 0) S[(int64_t)inst * NSLOT + S_ITER] = 0.0;
        return;
    }
    if (threadIdx.x == 0 && out)
        for (int c = 0; c < ncomp; c++) out[(int64_t)inst * ncomp + c] = vals[c];
    // FGMRES: the second-pass coefficients and |w'|^2 go straight into the
    // Arnoldi column update of this instance (the whole block takes part)
    if (op == RED_ARNOLDI) arnoldi_column(inst, active, S, arn, vals, rows, rows + 64, rows + 128);
    else if (threadIdx.x == 0) scalar_op(op, inst, vals, pre, S, active, maxit, slot, aux);
}

// Copy between the batch vector (chunk ranges) and the per-instance arrays of
// instances g0 .. g0 + PtrBlock::N - 1: to_batch ? batch = inst : inst = batch.
__global__ __launch_bounds__(VB) void k_gather_scatter(const Chunk *__restrict__ chunks, PtrBlock pb, int g0,
                                                       double *__restrict__ batch, int to_batch)
{
    const Chunk ch = chunks[blockIdx.x];
    const int g = ch.inst - g0;
    double *p = pb.p[g];
    const int64_t off = pb.off[g];
    for (int64_t e = ch.beg + threadIdx.x; e < ch.end; e += VB) {
        if (to_batch) batch[e] = p[e - off];
        else p[e - off] = batch[e];
    }
}

// Per-instance flags set from the host: the values travel as a kernel
// argument, so no host buffer has to stay untouched until a copy runs.
__global__ __launch_bounds__(VB) void k_set_flags(FlagBlock f, int beg, int cnt, int32_t *__restrict__ dst)
{
    if ((int)threadIdx.x < cnt) dst[beg + threadIdx.x] = f.v[threadIdx.x];
}

// Scalar slots and flags written straight into host-visible memory, then a
// sequence number once all of them are visible system-wide (the host waits
// for that number instead of a stream synchronisation).
__global__ __launch_bounds__(VB) void k_export(const double *__restrict__ S, int nS,
                                               const int32_t *__restrict__ act, int n, double *hs,
                                               int32_t *ha, uint32_t *seq_ptr, uint32_t seq)
{
    for (int i = threadIdx.x; i < nS; i += VB) hs[i] = S[i];
    for (int i = threadIdx.x; i < n; i += VB) ha[i] = act[i];
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence_system();
        __hip_atomic_store(seq_ptr, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// S[i * NSLOT + slot[j]] = v[j][i] for the instances beg .. beg + cnt - 1
__global__ __launch_bounds__(VB) void k_set_slots(SlotBlock b, int beg, int cnt, int nslots, double *__restrict__ S)
{
    const int i = threadIdx.x;
    if (i >= cnt) return;
    for (int j = 0; j < nslots; j++) S[(int64_t)(beg + i) * NSLOT + b.slot[j]] = b.v[j][i];
}

}  // namespace

// ---------------------------------------------------------------- host API
#define GRID dim3((unsigned)v.nchunk), dim3(VB), 0, v.stream

template <typename T>
void vfill(const VecCtx &v, T *y, T val) { k_fill<T><<<GRID>>>(v.chunks, v.active, v.S, y, val); HTS_LAUNCH_CHECK(); }
void vextrapolate(const VecCtx &v, int slot1, int slot2, const OpDev *ops, const double *Xn, const double *Xp,
                  const double *Xpp, double *x)
{
    k_extrapolate<<<GRID>>>(v.chunks, v.active, v.S, slot1, slot2, ops, Xn, Xp, Xpp, x);
    HTS_LAUNCH_CHECK();
}
void vrhs_combine(const VecCtx &v, const double *y, const double *ld, int slot, double *b)
{
    k_rhs_combine<<<GRID>>>(v.chunks, v.active, v.S, y, ld, slot, b);
    HTS_LAUNCH_CHECK();
}
void vadd(const VecCtx &v, const double *x, const double *y, double *z)
{
    k_add<<<GRID>>>(v.chunks, v.active, v.S, x, y, z);
    HTS_LAUNCH_CHECK();
}
void vshift(const VecCtx &v, const double *X1, double *Xn, double *Xp, double *Xpp)
{
    k_shift<<<GRID>>>(v.chunks, v.active, v.S, X1, Xn, Xp, Xpp);
    HTS_LAUNCH_CHECK();
}
template <typename T>
void vcopy(const VecCtx &v, const T *x, T *y) { k_copy<T><<<GRID>>>(v.chunks, v.active, v.S, x, y); HTS_LAUNCH_CHECK(); }
template <typename T>
void vaxpby(const VecCtx &v, double a, int ia, const T *x, double b, int ib, T *y)
{
    k_axpby<T><<<GRID>>>(v.chunks, v.active, v.S, a, ia, x, b, ib, y);
    HTS_LAUNCH_CHECK();
}
template <typename T>
void vjacobi(const VecCtx &v, double c, int ic, const T *d, const T *r, T *z)
{
    k_jacobi<T><<<GRID>>>(v.chunks, v.active, v.S, c, ic, d, r, z);
    HTS_LAUNCH_CHECK();
}
template <typename T>
void vdot(const VecCtx &v, const T *x, const T *y, const T *w, double *partial)
{
    k_dot<T><<<GRID>>>(v.chunks, v.active, v.S, x, y, w, partial);
    HTS_LAUNCH_CHECK();
}
template <typename T>
void vcg_update(const VecCtx &v, T *x, T *r, const T *p, const T *q, T *r_old, double *partial)
{
    k_cg_update<T><<<GRID>>>(v.chunks, v.active, v.S, x, r, p, q, r_old, partial);
    HTS_LAUNCH_CHECK();
}
template <typename T>
void vmultidot(const VecCtx &v, const T *V, int64_t ld, int nv, const T *w, double *partial, int ncomp)
{
    if (nv < 1 || nv > 64) throw Error(-1, "vmultidot: 1..64 vectors");
#define HTS_MDOT(NB) k_multidot<T, NB><<<GRID>>>(v.chunks, v.active, v.S, V, ld, nv, w, partial, ncomp)
    if (nv <= 4) HTS_MDOT(4);
    else if (nv <= 8) HTS_MDOT(8);
    else if (nv <= 12) HTS_MDOT(12);
    else if (nv <= 16) HTS_MDOT(16);
    else if (nv <= 24) HTS_MDOT(24);
    else if (nv <= 32) HTS_MDOT(32);
    else if (nv <= 48) HTS_MDOT(48);
    else HTS_MDOT(64);
#undef HTS_MDOT
    HTS_LAUNCH_CHECK();
}
template <typename T>
void vorth_update(const VecCtx &v, const T *V, int64_t ld, int nv, const double *H, int hld, T *w, int dots,
                  double *partial, int ncomp, int scale_slot)
{
    if (scale_slot >= 0 && partial) throw Error(-1, "vorth_update: scaling takes no partial sums");
    if (nv < 1 || nv > 64) throw Error(-1, "vorth_update: 1..64 vectors");
#define HTS_ORTH(NB) k_orth_update<T, NB><<<GRID>>>(v.chunks, v.active, v.S, V, ld, nv, H, hld, w, dots, partial, ncomp, scale_slot)
    if (nv <= 4) HTS_ORTH(4);
    else if (nv <= 8) HTS_ORTH(8);
    else if (nv <= 12) HTS_ORTH(12);
    else if (nv <= 16) HTS_ORTH(16);
    else if (nv <= 24) HTS_ORTH(24);
    else if (nv <= 32) HTS_ORTH(32);
    else if (nv <= 48) HTS_ORTH(48);
    else HTS_ORTH(64);
#undef HTS_ORTH
    HTS_LAUNCH_CHECK();
}
template <typename T, typename TX>
void vbasis_update(const VecCtx &v, const T *Z, int64_t ld, const int32_t *kdim, const double *Y, int yld,
                   double scale, int iscale, TX *x)
{
    k_basis_update<T, TX><<<GRID>>>(v.chunks, v.active, v.S, Z, ld, kdim, Y, yld, scale, iscale, x);
    HTS_LAUNCH_CHECK();
}
template <typename TX, typename TY>
void vconvert(const VecCtx &v, double sc, int ic, const TX *x, TY *y)
{
    k_convert<TX, TY><<<GRID>>>(v.chunks, v.active, v.S, sc, ic, x, y);
    HTS_LAUNCH_CHECK();
}
template <typename T>
void vadd_scaled(const VecCtx &v, double sc, int ic, const T *d, double *x)
{
    k_add_scaled<T><<<GRID>>>(v.chunks, v.active, v.S, sc, ic, d, x);
    HTS_LAUNCH_CHECK();
}
template <typename T>
void vmask(const VecCtx &v, const OpDev *ops, T *y, T val)
{
    k_mask<T><<<GRID>>>(v.chunks, v.active, v.S, ops, y, val);
    HTS_LAUNCH_CHECK();
}

void vpiezo32(const VecCtx &v, const OpDev *ops64, const double *P, float *P32)
{
    k_piezo32<<<GRID>>>(v.chunks, ops64, P, P32);
    HTS_LAUNCH_CHECK();
}

void vreduce(const RedCtx &r, const double *partial, int ncomp, int op, int slot, double *S, int32_t *active,
             int maxit, double aux, double *out, hipStream_t s)
{
    if (ncomp < 1 || ncomp > 64) throw Error(-1, "vreduce: 1..64 components");
    k_reduce<<<dim3((unsigned)r.nseg), dim3(RB), 0, s>>>(partial, ncomp, r.seg_ptr, r.single, op, slot, S,
                                                          active, maxit, aux, out, ArnArgs{});
    HTS_LAUNCH_CHECK();
}

void vreduce_arnoldi(const RedCtx &r, const double *partial, int ncomp, double *S, int32_t *active,
                     const ArnArgs &arn, double *out, hipStream_t s)
{
    if (ncomp < 1 || ncomp > 64) throw Error(-1, "vreduce: 1..64 components");
    k_reduce<<<dim3((unsigned)r.nseg), dim3(RB), 0, s>>>(partial, ncomp, r.seg_ptr, r.single, RED_ARNOLDI, 0, S,
                                                          active, 0, 0.0, out, arn);
    HTS_LAUNCH_CHECK();
}

void vgather_scatter(const Chunk *chunks, const std::vector<Chunk> &hchunks, const std::vector<double *> &ptrs,
                     const std::vector<int64_t> &off, double *batch, bool to_batch, hipStream_t s)
{
    const int n = (int)ptrs.size();
    size_t c0 = 0;
    for (int g0 = 0; g0 < n; g0 += PtrBlock::N) {
        const int g1 = std::min(n, g0 + PtrBlock::N);
        PtrBlock pb{};
        for (int i = g0; i < g1; i++) {
            pb.p[i - g0] = ptrs[i];
            pb.off[i - g0] = off[i];
        }
        size_t c1 = c0;
        while (c1 < hchunks.size() && hchunks[c1].inst < g1) c1++;
        if (c1 > c0)
            k_gather_scatter<<<dim3((unsigned)(c1 - c0)), dim3(VB), 0, s>>>(chunks + c0, pb, g0, batch,
                                                                          to_batch ? 1 : 0);
        HTS_LAUNCH_CHECK();
        c0 = c1;
    }
}

void vset_flags(const int32_t *flags, int n, int32_t *dst, hipStream_t s)
{
    for (int beg = 0; beg < n; beg += FlagBlock::N) {
        FlagBlock f{};
        const int cnt = std::min(FlagBlock::N, n - beg);
        for (int i = 0; i < cnt; i++) f.v[i] = flags[beg + i];
        k_set_flags<<<dim3(1), dim3(VB), 0, s>>>(f, beg, cnt, dst);
        HTS_LAUNCH_CHECK();
    }
}

void vexport(const double *S, int nS, const int32_t *act, int n, double *hs, int32_t *ha, uint32_t *seq_ptr,
             uint32_t seq, hipStream_t s)
{
    k_export<<<dim3(1), dim3(VB), 0, s>>>(S, nS, act, n, hs, ha, seq_ptr, seq);
    HTS_LAUNCH_CHECK();
}

void vset_slots(const int *slots, int nslots, const double *const *vals, int n, double *S, hipStream_t s)
{
    if (nslots > SlotBlock::NS) throw Error(-1, "too many slots");   // -1: invalid argument
    for (int beg = 0; beg < n; beg += SlotBlock::N) {
        SlotBlock b{};
        const int cnt = std::min(SlotBlock::N, n - beg);
        for (int j = 0; j < nslots; j++) {
            b.slot[j] = slots[j];
            for (int i = 0; i < cnt; i++) b.v[j][i] = vals[j][beg + i];
        }
        k_set_slots<<<dim3(1), dim3(VB), 0, s>>>(b, beg, cnt, nslots, S);
        HTS_LAUNCH_CHECK();
    }
}

#define INST(T)                                                                                          \
    template void vfill<T>(const VecCtx &, T *, T);                                                      \
    template void vcopy<T>(const VecCtx &, const T *, T *);                                              \
    template void vaxpby<T>(const VecCtx &, double, int, const T *, double, int, T *);                   \
    template void vjacobi<T>(const VecCtx &, double, int, const T *, const T *, T *);                    \
    template void vdot<T>(const VecCtx &, const T *, const T *, const T *, double *);                    \
    template void vcg_update<T>(const VecCtx &, T *, T *, const T *, const T *, T *, double *);          \
    template void vmultidot<T>(const VecCtx &, const T *, int64_t, int, const T *, double *, int);       \
    template void vorth_update<T>(const VecCtx &, const T *, int64_t, int, const double *, int, T *, int, \
                                  double *, int, int);                                                   \
    template void vbasis_update<T, double>(const VecCtx &, const T *, int64_t, const int32_t *,          \
                                           const double *, int, double, int, double *);                 \
    template void vbasis_update<T, float>(const VecCtx &, const T *, int64_t, const int32_t *,           \
                                          const double *, int, double, int, float *);                   \
    template void vadd_scaled<T>(const VecCtx &, double, int, const T *, double *);                      \
    template void vmask<T>(const VecCtx &, const OpDev *, T *, T);
INST(double)
INST(float)
template void vconvert<double, float>(const VecCtx &, double, int, const double *, float *);
template void vconvert<float, double>(const VecCtx &, double, int, const float *, double *);
template void vconvert<double, double>(const VecCtx &, double, int, const double *, double *);
template void vconvert<float, float>(const VecCtx &, double, int, const float *, float *);

}  // namespace hts
