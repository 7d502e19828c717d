// Geometric multigrid kernels: 2:1 coarsening of the structured node grid,
// trilinear prolongation P (fine constrained nodes masked), restriction
// R = P^T, Galerkin coarse operators A_c = P^T A P stored as 27-point
// stencils, Chebyshev-Jacobi smoothing fused with the stencil product, and a
// dense FP64 solve on the coarsest level.
//
// Coarsening along one axis with Nf fine nodes (last = Nf - 1): coarse node I
// sits on fine node min(2I, last); a fine node is either on a coarse node
// (even index, or the last node) or the midpoint of two coarse nodes.  Odd
// cell counts therefore coarsen too (the last coarse cell spans one fine
// cell).
#include "common.h"
#include "dev_util.h"
#include "mg.h"

namespace hts {

namespace {

__device__ __forceinline__ double pw1(int i, int I, int Nf)
{
    const int last = Nf - 1;
    if ((i & 1) == 0 || i == last) return ((i + 1) >> 1) == I ? 1.0 : 0.0;
    return (((i - 1) >> 1) == I || ((i + 1) >> 1) == I) ? 0.5 : 0.0;
}

__device__ __forceinline__ int fpos(int I, int Nf) { return min(2 * I, Nf - 1); }

// parents of fine node i: count, indices, weights
__device__ __forceinline__ int parents(int i, int Nf, int *P, double *W)
{
    const int last = Nf - 1;
    if ((i & 1) == 0 || i == last) {
        P[0] = (i + 1) >> 1;
        W[0] = 1.0;
        return 1;
    }
    P[0] = (i - 1) >> 1;
    P[1] = (i + 1) >> 1;
    W[0] = W[1] = 0.5;
    return 2;
}

// the same with always two entries: a single parent is repeated with weight 0
__device__ __forceinline__ void parents2(int i, int Nf, int *P, double *W)
{
    const bool one = (i & 1) == 0 || i == Nf - 1;
    P[0] = one ? (i + 1) >> 1 : (i - 1) >> 1;
    P[1] = one ? P[0] : (i + 1) >> 1;
    W[0] = one ? 1.0 : 0.5;
    W[1] = one ? 0.0 : 0.5;
}

template <typename T, int EPI>
__global__ __launch_bounds__(256) void k_stencil(const LevelDev *__restrict__ lev, const Chunk *__restrict__ chunks,
                                                 const int32_t *active, const T *__restrict__ X, T *__restrict__ Y,
                                                 EpiArgs<T> ep)
{
    const Chunk ch = chunks[blockIdx.x];
    if (active && !active[ch.inst]) return;
    const LevelDev &L = lev[ch.inst];
    const T HTS_GLOBAL *__restrict__ St = gptr<T>(L.S);
    const int NX = L.NX, NY = L.NY, NZ = L.NZ;
    const int64_t pl = (int64_t)NX * NY;
    const T *Xi = X + L.off;
    const double *Sc = ep.S ? ep.S + (int64_t)ch.inst * NSLOT : nullptr;
    const T c0 = EPI == EPI_CHEB0 ? T(Sc[ep.s0]) : T(0);
    const T *Ii = EPI == EPI_CHEB0 ? ep.invd + L.off : nullptr;
    const T *Bi = EPI == EPI_CHEB0 ? ep.b + L.off : nullptr;
    for (int64_t e = ch.beg + threadIdx.x; e < ch.end; e += 256) {
        // instance-local indices fit 32 bits (meshes have < 2^31 nodes)
        const int n = (int)(e - L.off);
        const int nxy = n / NX, i = n - nxy * NX, k = nxy / NY, j = nxy - k * NY;
        // Neighbours outside the grid have zero coefficients (the assembled
        // and Galerkin stencils never couple to them): their offsets are
        // clamped to the node itself, so every load is unconditional and all
        // 54 of them can be in flight together.
        const int ox[3] = {i > 0 ? -1 : 0, 0, i < NX - 1 ? 1 : 0};
        const int oy[3] = {j > 0 ? -NX : 0, 0, j < NY - 1 ? NX : 0};
        const int oz[3] = {k > 0 ? -(int)pl : 0, 0, k < NZ - 1 ? (int)pl : 0};
        const int ln = (int)L.n;
        T acc = T(0);
#pragma unroll
        for (int dz = 0; dz < 3; dz++)
#pragma unroll
            for (int dy = 0; dy < 3; dy++)
#pragma unroll
                for (int dx = 0; dx < 3; dx++) {
                    const int c = dx + 3 * dy + 9 * dz;
                    const int nb = n + ox[dx] + oy[dy] + oz[dz];
                    // EPI_CHEB0 operand: x0 = c0 D^-1 b
                    const T xv = EPI == EPI_CHEB0 ? c0 * Ii[nb] * Bi[nb] : Xi[nb];
                    acc += St[c * ln + n] * xv;
                }
        if (EPI == EPI_STORE) {
            Y[e] = acc;
        } else if (EPI == EPI_RESID) {
            Y[e] = ep.b[e] - acc;
        } else if (EPI == EPI_CHEB) {
            T r = ep.b[e] - acc;
            T d = T(Sc[ep.s1]) * ep.d[e] + T(Sc[ep.s2]) * ep.invd[e] * r;
            ep.d[e] = d;
            Y[e] = X[e] + d;
        } else if (EPI == EPI_CHEB0) {
            const T x0 = c0 * ep.invd[e] * ep.b[e];
            T r = ep.b[e] - acc;
            T d = T(Sc[ep.s1]) * x0 + T(Sc[ep.s2]) * ep.invd[e] * r;
            ep.d[e] = d;
            Y[e] = x0 + d;
        }
    }
}

// first Chebyshev step from x = 0: d = c D^-1 b, x = d
template <typename T>
__global__ __launch_bounds__(256) void k_cheb0(const Chunk *__restrict__ chunks, const int32_t *active,
                                               const double *S, int slot, const T *__restrict__ invd,
                                               const T *__restrict__ b, T *__restrict__ d, T *__restrict__ x)
{
    const Chunk ch = chunks[blockIdx.x];
    if (active && !active[ch.inst]) return;
    const T c = T(S[(int64_t)ch.inst * NSLOT + slot]);
    for (int64_t e = ch.beg + threadIdx.x; e < ch.end; e += 256) {
        T v = c * invd[e] * b[e];
        d[e] = v;
        x[e] = v;
    }
}

// Fine neighbours of coarse node I along one axis: fine nodes fi - 1 .. fi + 1
// (fi = fpos(I, Nf)), with weight 0 and a clamped index where a node is
// outside the grid or not a child of I.
__device__ __forceinline__ void children(int I, int Nf, int idx[3], double w[3])
{
    const int fi = fpos(I, Nf);
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int i = fi + d - 1;
        const bool in = i >= 0 && i < Nf;
        w[d] = in ? pw1(i, I, Nf) : 0.0;
        idx[d] = in ? i : fi;
    }
}

// coarse b_c = P^T r_f (fine constrained rows excluded when fops != null),
// the fine rows summed z-outer, then y, then x
template <typename T>
__global__ __launch_bounds__(256) void k_restrict(const LevelDev *__restrict__ fine, const LevelDev *__restrict__ coarse,
                                                  const OpDev *__restrict__ fops, const Chunk *__restrict__ cchunks,
                                                  const int32_t *active, const T *__restrict__ rf, T *__restrict__ bc,
                                                  int mask_coarse)
{
    const Chunk ch = cchunks[blockIdx.x];
    if (active && !active[ch.inst]) return;
    const LevelDev &F = fine[ch.inst];
    const LevelDev &Cc = coarse[ch.inst];
    const int fNX = F.NX, fNY = F.NY, fNZ = F.NZ, cNX = Cc.NX, cNY = Cc.NY;
    const int fpl = fNX * fNY;
    const T *rfi = rf + F.off;
    for (int64_t e = ch.beg + threadIdx.x; e < ch.end; e += 256) {
        const int n = (int)(e - Cc.off);
        const int nxy = n / cNX, I = n - nxy * cNX, K = nxy / cNY, J = nxy - K * cNY;
        int xi[3], yi[3], zi[3];
        double wx[3], wy[3], wz[3];
        children(I, fNX, xi, wx);
        children(J, fNY, yi, wy);
        children(K, fNZ, zi, wz);
        // constraint data of the 3 x 3 fine columns
        bool cxy[3][3];
        int lo[3][3], hi[3][3];
        int NZo = 0, m = 0;
#pragma unroll
        for (int b = 0; b < 3; b++)
#pragma unroll
            for (int a = 0; a < 3; a++) {
                cxy[b][a] = false;
                lo[b][a] = 1;
                hi[b][a] = 0;
            }
        if (fops) {
            const OpDev &o = fops[ch.inst];
            NZo = o.NZ;
            m = o.dmask;
#pragma unroll
            for (int b = 0; b < 3; b++)
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    const ColInfo c = col_info(o, xi[a], yi[b]);
                    cxy[b][a] = c.xyc != 0;
                    lo[b][a] = c.dlo;
                    hi[b][a] = c.dhi;
                }
            // a coarse operator with eliminated (identity) rows where the fine
            // node under the coarse node is constrained takes no residual there
            if (mask_coarse) {
                const ColInfo cc = col_info(o, fpos(I, fNX), fpos(J, fNY));
                if (constrained(cc, fpos(K, fNZ), NZo, m)) {
                    bc[e] = T(0);
                    continue;
                }
            }
        }
        // every child is loaded (the indices of absent children are clamped
        // into the grid and their weight is 0; constrained children get weight
        // 0), so the 27 loads are unconditional
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int b = 0; b < 3; b++)
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    double w = wx[a] * wy[b] * wz[c];
                    if (fops) {
                        const int k = zi[c];
                        const bool con = cxy[b][a] || ((m & 16) && k == 0) || ((m & 32) && k == NZo - 1) ||
                                         (k >= lo[b][a] && k <= hi[b][a]);
                        w = con ? 0.0 : w;
                    }
                    acc += w * (double)rfi[xi[a] + yi[b] * fNX + zi[c] * fpl];
                }
        bc[e] = T(acc);
    }
}

// x_f += P x_c (fine constrained nodes untouched when fops != null)
template <typename T>
__global__ __launch_bounds__(256) void k_prolong_add(const LevelDev *__restrict__ fine, const LevelDev *__restrict__ coarse,
                                                     const OpDev *__restrict__ fops, const Chunk *__restrict__ fchunks,
                                                     const int32_t *active, const T *__restrict__ xc, T *__restrict__ xf)
{
    const Chunk ch = fchunks[blockIdx.x];
    if (active && !active[ch.inst]) return;
    const LevelDev &F = fine[ch.inst];
    const LevelDev &Cc = coarse[ch.inst];
    const int fNX = F.NX, fNY = F.NY, fNZ = F.NZ, cNX = Cc.NX;
    const int cpl = Cc.NX * Cc.NY;
    const T *xci = xc + Cc.off;
    for (int64_t e = ch.beg + threadIdx.x; e < ch.end; e += 256) {
        const int n = (int)(e - F.off);
        const int nxy = n / fNX, i = n - nxy * fNX, k = nxy / fNY, j = nxy - k * fNY;
        bool con = false;
        if (fops) {
            const OpDev &o = fops[ch.inst];
            con = constrained(col_info(o, i, j), k, o.NZ, o.dmask);
        }
        // two parents per axis, the second with weight 0 (and the first's
        // index) where there is one: eight unconditional loads
        int Px[2], Py[2], Pz[2];
        double Wx[2], Wy[2], Wz[2];
        parents2(i, fNX, Px, Wx);
        parents2(j, fNY, Py, Wy);
        parents2(k, fNZ, Pz, Wz);
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 2; c++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int a = 0; a < 2; a++)
                    acc += Wx[a] * Wy[b] * Wz[c] * (double)xci[Px[a] + Py[b] * cNX + Pz[c] * cpl];
        if (!con) xf[e] = T((double)xf[e] + acc);
    }
}

// Galerkin A_c = P^T A_f P for one instance; stencils [27][n] in FP64.
__global__ __launch_bounds__(128) void k_rap(int fNX, int fNY, int fNZ, const double *__restrict__ Sf, int64_t fn,
                                             int cNX, int cNY, int cNZ, double *__restrict__ Sc, int64_t cn)
{
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= cn) return;
    const int64_t cpl = (int64_t)cNX * cNY, fpl = (int64_t)fNX * fNY;
    const int I = (int)(n % cNX), J = (int)((n / cNX) % cNY), K = (int)(n / cpl);
    double acc[27];
    for (int e = 0; e < 27; e++) acc[e] = 0.0;
    const int fi = fpos(I, fNX), fj = fpos(J, fNY), fk = fpos(K, fNZ);
    for (int dz = -1; dz <= 1; dz++) {
        const int k = fk + dz;
        if (k < 0 || k >= fNZ) continue;
        const double wz = pw1(k, K, fNZ);
        if (wz == 0.0) continue;
        for (int dy = -1; dy <= 1; dy++) {
            const int j = fj + dy;
            if (j < 0 || j >= fNY) continue;
            const double wy = pw1(j, J, fNY);
            if (wy == 0.0) continue;
            for (int dx = -1; dx <= 1; dx++) {
                const int i = fi + dx;
                if (i < 0 || i >= fNX) continue;
                const double wx = pw1(i, I, fNX);
                if (wx == 0.0) continue;
                const double wI = wx * wy * wz;
                const int64_t row = i + (int64_t)j * fNX + (int64_t)k * fpl;
                for (int c = 0; c < 27; c++) {
                    const double a = Sf[(int64_t)c * fn + row];
                    if (a == 0.0) continue;
                    const int ox = c % 3 - 1, oy = (c / 3) % 3 - 1, oz = c / 9 - 1;
                    const int ji = i + ox, jj = j + oy, jk = k + oz;
                    if (ji < 0 || ji >= fNX || jj < 0 || jj >= fNY || jk < 0 || jk >= fNZ) continue;
                    int Px[2], Py[2], Pz[2];
                    double Wx[2], Wy[2], Wz[2];
                    const int nx_ = parents(ji, fNX, Px, Wx), ny_ = parents(jj, fNY, Py, Wy),
                              nz_ = parents(jk, fNZ, Pz, Wz);
                    for (int cz = 0; cz < nz_; cz++)
                        for (int cy = 0; cy < ny_; cy++)
                            for (int cx = 0; cx < nx_; cx++) {
                                const int ex = Px[cx] - I, ey = Py[cy] - J, ez = Pz[cz] - K;
                                if (ex < -1 || ex > 1 || ey < -1 || ey > 1 || ez < -1 || ez > 1) continue;
                                acc[(ex + 1) + 3 * (ey + 1) + 9 * (ez + 1)] += wI * a * Wx[cx] * Wy[cy] * Wz[cz];
                            }
                }
            }
        }
    }
    if (acc[13] == 0.0) acc[13] = 1.0;   // a coarse function with no free support
    for (int e = 0; e < 27; e++) Sc[(int64_t)e * cn + n] = acc[e];
}

// inverse diagonal of a stencil level (FP64)
__global__ void k_stencil_invdiag(const double *__restrict__ S, int64_t n, double *__restrict__ out)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) out[e] = 1.0 / S[13 * n + e];
}

// dense FP64 coarse solve x = Ainv b: one wave per row
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_solve(const CoarseDev *__restrict__ cd, int ninst, const int32_t *active,
                                                      const T *__restrict__ b, T *__restrict__ x)
{
    const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6, lane = threadIdx.x & 63;
    // find (instance, row) of this wave: rows are numbered across instances
    int k = -1;
    int64_t row = 0;
    for (int s = 0; s < ninst; s++) {
        if (wave >= cd[s].row0 && wave < cd[s].row0 + cd[s].n) { k = s; row = wave - cd[s].row0; break; }
    }
    if (k < 0) return;
    const CoarseDev &C = cd[k];
    if (active && !active[C.inst]) return;
    const double HTS_GLOBAL *A = gptr<double>(C.Ainv) + row * C.n;
    const T *bi = b + C.off;
    const int n = (int)C.n;
    // four independent partial sums per lane, so that four row segments
    // are in flight at once
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int j = lane;
    for (; j + 192 < n; j += 256) {
        a0 += A[j] * (double)bi[j];
        a1 += A[j + 64] * (double)bi[j + 64];
        a2 += A[j + 128] * (double)bi[j + 128];
        a3 += A[j + 192] * (double)bi[j + 192];
    }
    for (; j < n; j += 64) a0 += A[j] * (double)bi[j];
    double acc = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) x[C.off + row] = T(acc);
}

}  // namespace

template <typename T>
void launch_stencil(int epi, const LevelDev *lev, const Chunk *chunks, int nchunk, const int32_t *active, const T *x,
                    T *y, const EpiArgs<T> &ep, hipStream_t s)
{
    if (nchunk <= 0) return;
    dim3 g(nchunk), b(256);
    switch (epi) {
    case EPI_STORE: k_stencil<T, EPI_STORE><<<g, b, 0, s>>>(lev, chunks, active, x, y, ep); break;
    case EPI_RESID: k_stencil<T, EPI_RESID><<<g, b, 0, s>>>(lev, chunks, active, x, y, ep); break;
    case EPI_CHEB: k_stencil<T, EPI_CHEB><<<g, b, 0, s>>>(lev, chunks, active, x, y, ep); break;
    case EPI_CHEB0: k_stencil<T, EPI_CHEB0><<<g, b, 0, s>>>(lev, chunks, active, x, y, ep); break;
    default: throw Error(-1, "bad stencil epilogue");
    }
    HTS_LAUNCH_CHECK();
}

template <typename T>
void launch_cheb0(const Chunk *chunks, int nchunk, const int32_t *active, const double *S, int slot, const T *invd,
                  const T *b, T *d, T *x, hipStream_t s)
{
    if (nchunk <= 0) return;
    k_cheb0<T><<<dim3(nchunk), dim3(256), 0, s>>>(chunks, active, S, slot, invd, b, d, x);
    HTS_LAUNCH_CHECK();
}

template <typename T>
void launch_restrict(const LevelDev *fine, const LevelDev *coarse, const OpDev *fops, const Chunk *cchunks,
                     int nchunk, const int32_t *active, const T *rf, T *bc, int mask_coarse, hipStream_t s)
{
    if (nchunk <= 0) return;
    if (mask_coarse && !fops) throw Error(-1, "coarse masking needs the fine operator descriptors");
    k_restrict<T><<<dim3(nchunk), dim3(256), 0, s>>>(fine, coarse, fops, cchunks, active, rf, bc, mask_coarse);
    HTS_LAUNCH_CHECK();
}

template <typename T>
void launch_prolong_add(const LevelDev *fine, const LevelDev *coarse, const OpDev *fops, const Chunk *fchunks,
                        int nchunk, const int32_t *active, const T *xc, T *xf, hipStream_t s)
{
    if (nchunk <= 0) return;
    k_prolong_add<T><<<dim3(nchunk), dim3(256), 0, s>>>(fine, coarse, fops, fchunks, active, xc, xf);
    HTS_LAUNCH_CHECK();
}

void launch_rap(int fNX, int fNY, int fNZ, const double *Sf, int cNX, int cNY, int cNZ, double *Sc, hipStream_t s)
{
    const int64_t fn = (int64_t)fNX * fNY * fNZ, cn = (int64_t)cNX * cNY * cNZ;
    k_rap<<<dim3((unsigned)((cn + 127) / 128)), dim3(128), 0, s>>>(fNX, fNY, fNZ, Sf, fn, cNX, cNY, cNZ, Sc, cn);
    HTS_LAUNCH_CHECK();
}

void launch_stencil_invdiag(const double *S, int64_t n, double *out, hipStream_t s)
{
    k_stencil_invdiag<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(S, n, out);
    HTS_LAUNCH_CHECK();
}

template <typename T>
void launch_coarse_solve(const CoarseDev *cd, int ninst, int64_t total_rows, const int32_t *active, const T *b,
                         T *x, hipStream_t s)
{
    const int64_t threads = total_rows * 64;
    k_coarse_solve<T><<<dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s>>>(cd, ninst, active, b, x);
    HTS_LAUNCH_CHECK();
}

#define INST(T)                                                                                                  \
    template void launch_stencil<T>(int, const LevelDev *, const Chunk *, int, const int32_t *, const T *, T *,   \
                                    const EpiArgs<T> &, hipStream_t);                                            \
    template void launch_cheb0<T>(const Chunk *, int, const int32_t *, const double *, int, const T *, const T *, \
                                  T *, T *, hipStream_t);                                                        \
    template void launch_restrict<T>(const LevelDev *, const LevelDev *, const OpDev *, const Chunk *, int,       \
                                     const int32_t *, const T *, T *, int, hipStream_t);                              \
    template void launch_prolong_add<T>(const LevelDev *, const LevelDev *, const OpDev *, const Chunk *, int,   \
                                        const int32_t *, const T *, T *, hipStream_t);                           \
    template void launch_coarse_solve<T>(const CoarseDev *, int, int64_t, const int32_t *, const T *, T *,        \
                                         hipStream_t);
INST(double)
INST(float)

}  // namespace hts
