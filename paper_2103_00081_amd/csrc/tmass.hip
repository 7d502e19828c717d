// Separable preconditioner for the heat equation (Eq. 4 at the time steps of
// interest is dominated by its capacity and conduction terms):
//     z = S (B_x^-1 (x) B_y^-1 (x) B_z^-1) S r,   S = diag(cbar_T)^(-1/2),
//     B_d = M_d + alpha K_d,   alpha = dt * median(lambda / c_T),
// where M_d and K_d are the 1D Q1 mass and stiffness matrices along axis d
// (Dirichlet ends replaced by identity rows where that face is
// constrained) and cbar_T the mean capacity of the cells around a node; the
// product differs from M + alpha K by terms of order alpha^2.  Each 1D
// inverse is a Thomas solve along every grid line, with the elimination
// factors of the line precomputed once per axis and instance.
#include "common.h"
#include "dev_util.h"
#include "tmass.h"

namespace hts {

namespace {

// Find the instance whose [beg, end) range of blocks contains block b.
__device__ __forceinline__ int find_inst(const int64_t *__restrict__ beg, int n, int64_t b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (beg[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One wavefront solves up to `lb` lines of one instance along axis AX: the
// lines are staged in LDS with coalesced loads (scaled by S when `first`),
// each lane runs the Thomas recurrences of one line in LDS, and the results
// go back with coalesced stores (scaled by S when `last`).  Krylov vectors
// are zero on constrained rows and faces are identity rows of the 1D
// factors, so only Dirichlet columns need masking, on the z pass, which
// runs along node columns (`last` is the z pass).
template <typename T, int AX>
__global__ __launch_bounds__(64) void k_tmass_sweep(const TMassInst *__restrict__ inst, int ninst,
                                                    const int64_t *__restrict__ bbeg, int lb,
                                                    const int32_t *active, const OpDev *__restrict__ ops,
                                                    const T *__restrict__ in, T *__restrict__ out, int first,
                                                    int last)
{
    extern __shared__ unsigned char tm_smem[];
    T *buf = reinterpret_cast<T *>(tm_smem);
    const int i = find_inst(bbeg, ninst, blockIdx.x);
    if (active && !active[i]) return;
    const TMassInst &I = inst[i];
    const int NX = I.N[0], NY = I.N[1], NZ = I.N[2];
    const int n = I.N[AX];
    const int nlines = AX == 0 ? NY * NZ : (AX == 1 ? NX * NZ : NX * NY);
    const int l0 = (int)(blockIdx.x - bbeg[i]) * lb;
    const int cnt = min(lb, nlines - l0);
    const int ld = n | 1;   // odd row stride: conflict-free column access
    const int lane = threadIdx.x;
    const T *__restrict__ src = in + I.off;
    T *__restrict__ dst = out + I.off;
    const T *__restrict__ sc = static_cast<const T *>(I.s) + I.off;
    const int plane = NX * NY;
    // lane's own line (AX 1, 2): first node and stride
    int base = 0, stride = 1;
    if (AX == 1) {
        const int l = l0 + lane, x = l % NX, k = l / NX;
        base = x + plane * k;
        stride = NX;
    } else if (AX == 2) {
        base = l0 + lane;
        stride = plane;
    }
    // stage
    if (AX == 0) {
        const int tot = cnt * n;
        for (int idx = lane; idx < tot; idx += 64) {
            const int ll = idx / n, e = idx - ll * n;
            const int node = NX * (l0 + ll) + e;
            T v = src[node];
            if (first) v *= sc[node];
            buf[ll * ld + e] = v;
        }
    } else if (lane < cnt) {
        for (int e = 0; e < n; e++) {
            const int node = base + e * stride;
            T v = src[node];
            if (first) v *= sc[node];
            buf[lane * ld + e] = v;
        }
    }
    __syncthreads();
    // solve: forward elimination then back substitution, factors shared by
    // every line of the axis
    if (lane < cnt) {
        const double *__restrict__ fa = I.fac[AX];
        const double *__restrict__ fi = fa + n, *__restrict__ fc = fa + 2 * n;
        T *row = buf + lane * ld;
        T prev = T(0);
        for (int e = 0; e < n; e++) {
            const T v = (row[e] - T(fa[e]) * prev) * T(fi[e]);
            row[e] = v;
            prev = v;
        }
        T nxt = row[n - 1];
        for (int e = n - 2; e >= 0; e--) {
            nxt = row[e] - T(fc[e]) * nxt;
            row[e] = nxt;
        }
    }
    __syncthreads();
    // write back
    if (AX == 0) {
        const int tot = cnt * n;
        for (int idx = lane; idx < tot; idx += 64) {
            const int ll = idx / n, e = idx - ll * n;
            const int node = NX * (l0 + ll) + e;
            T v = buf[ll * ld + e];
            if (last) v *= sc[node];
            dst[node] = v;
        }
    } else if (lane < cnt) {
        ColInfo col;
        col.valid = 0;
        col.xyc = 0;
        col.dlo = 0xFFFF;
        col.dhi = 0;
        if (AX == 2 && last) col = col_info(ops[i], base % NX, base / NX);
        for (int e = 0; e < n; e++) {
            const int node = base + e * stride;
            T v = buf[lane * ld + e];
            if (last) v *= sc[node];
            if (AX == 2 && last && (e >= col.dlo && e <= col.dhi)) v = T(0);
            dst[node] = v;
        }
    }
}

}  // namespace

template <typename T>
void launch_tmass(const TMassInst *inst, int ninst, const int64_t *const bbeg[3], const int64_t nblocks[3],
                  const int lb[3], const int lds[3], const int32_t *active, const OpDev *ops, const T *r, T *z,
                  hipStream_t s)
{
    const dim3 b(64);
    if (nblocks[0] > 0)
        k_tmass_sweep<T, 0><<<dim3((unsigned)nblocks[0]), b, lds[0], s>>>(inst, ninst, bbeg[0], lb[0], active, ops,
                                                                          r, z, 1, 0);
    HTS_LAUNCH_CHECK();
    if (nblocks[1] > 0)
        k_tmass_sweep<T, 1><<<dim3((unsigned)nblocks[1]), b, lds[1], s>>>(inst, ninst, bbeg[1], lb[1], active, ops,
                                                                          z, z, 0, 0);
    HTS_LAUNCH_CHECK();
    if (nblocks[2] > 0)
        k_tmass_sweep<T, 2><<<dim3((unsigned)nblocks[2]), b, lds[2], s>>>(inst, ninst, bbeg[2], lb[2], active, ops,
                                                                          z, z, 0, 1);
    HTS_LAUNCH_CHECK();
}

template void launch_tmass<double>(const TMassInst *, int, const int64_t *const[3], const int64_t[3], const int[3],
                                   const int[3], const int32_t *, const OpDev *, const double *, double *,
                                   hipStream_t);
template void launch_tmass<float>(const TMassInst *, int, const int64_t *const[3], const int64_t[3], const int[3],
                                  const int[3], const int32_t *, const OpDev *, const float *, float *, hipStream_t);

}  // namespace hts
