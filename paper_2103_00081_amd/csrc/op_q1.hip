// Matrix-free Q1 operators of the pressure (Eq. 3) and heat (Eq. 4)
// equations on a uniform box, sum-factorised per cell.
//
// Kernel layout: a 256-thread workgroup owns a 15 x 15 tile of node columns
// and marches upward through a range of node planes.  Each thread handles
// one cell column of the 16 x 16 cells that touch the tile (one-cell halo on
// the low x/y side).  Per cell layer the two node planes are staged in LDS;
// each thread evaluates its cell's 8 outputs by Kronecker sum factorisation
// (1D mass h/6 [2 1; 1 2] and stiffness 1/h [1 -1; -1 1] in each direction,
// 2-point Gauss for the convection term) and writes its four plane-corner
// contributions to LDS; the owner of a node adds the four cell contributions
// in a fixed order.  Every node value is produced by exactly one thread:
// no atomics, bitwise reproducible.
#include "common.h"
#include "dev_util.h"

namespace hts {

namespace {

constexpr int TB = 16;          // cell columns per tile edge
constexpr int OWN = TB - 1;     // owned node columns per tile edge
constexpr int NCOL = (TB + 1) * (TB + 1);

template <typename T>
__device__ __forceinline__ void m1p(T &a, T &b)
{
    // [a; b] <- [2 1; 1 2]/6 [a; b]
    T s = a + b;
    T na = (a + s) * T(1.0 / 6.0);
    T nb = (b + s) * T(1.0 / 6.0);
    a = na;
    b = nb;
}

template <typename T>
__device__ __forceinline__ void k1p(T &a, T &b)
{
    // [a; b] <- [1 -1; -1 1] [a; b]
    T d = a - b;
    a = d;
    b = -d;
}

template <typename T>
__device__ __forceinline__ void g1p(T &a, T &b)
{
    // values at the two Gauss points from nodal values (and its transpose,
    // which is the same symmetric 2x2 matrix)
    const T cg = T(0.28867513459481288225);   // 1 / (2 sqrt 3)
    T s = (a + b) * T(0.5);
    T d = (a - b) * cg;
    a = s + d;
    b = s - d;
}

#define PZ(F, v) F(v[0], v[4]); F(v[1], v[5]); F(v[2], v[6]); F(v[3], v[7]);
#define PY(F, v) F(v[0], v[2]); F(v[1], v[3]); F(v[4], v[6]); F(v[5], v[7]);
#define PX(F, v) F(v[0], v[1]); F(v[2], v[3]); F(v[4], v[5]); F(v[6], v[7]);
#define P2(F, v) F(v[0], v[1]); F(v[2], v[3]); F(v[0], v[2]); F(v[1], v[3]);

// w = mV (M1 x M1 x M1) u + sk (cxx K1xM1xM1 + cyy M1xK1xM1 + czz M1xM1xK1) u
template <typename T>
__device__ __forceinline__ void cell_mass_stiff(const T u[8], T mV, T sk, T cxx, T cyy, T czz, T w[8])
{
    T a[8], b[8];
#pragma unroll
    for (int i = 0; i < 8; i++) { a[i] = u[i]; b[i] = u[i]; }
    PZ(m1p, a);
    PZ(k1p, b);
    T c[8], d[8], e[8];
#pragma unroll
    for (int i = 0; i < 8; i++) { c[i] = a[i]; d[i] = a[i]; e[i] = b[i]; }
    PY(m1p, c);
    PY(k1p, d);
    PY(m1p, e);
    T f[8], g[8];
    const T skx = sk * cxx, sky = sk * cyy, skz = sk * czz;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        f[i] = mV * c[i] + sky * d[i] + skz * e[i];
        g[i] = c[i];
    }
    PX(m1p, f);
    PX(k1p, g);
#pragma unroll
    for (int i = 0; i < 8; i++) w[i] = f[i] + skx * g[i];
}

// w += cw8 sum_q N_a(q) (q_h . grad u)(q), q_h = -k (grad P + rho_g e_z),
// 2 x 2 x 2 Gauss points, cw8 = dt c_w V / 8.
template <typename T>
__device__ __forceinline__ void cell_convect(const T u[8], const T P[8], T kc, T ihx, T ihy, T ihz,
                                            T rho_g, T cw8, T w[8])
{
    T gx[4], gy[4], gz[4], px[4], py[4], pz[4];
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
        for (int t = 0; t < 2; t++) {
            gx[s + 2 * t] = u[1 + 2 * s + 4 * t] - u[2 * s + 4 * t];   // (ay, az)
            gy[s + 2 * t] = u[s + 2 + 4 * t] - u[s + 4 * t];           // (ax, az)
            gz[s + 2 * t] = u[s + 2 * t + 4] - u[s + 2 * t];           // (ax, ay)
            px[s + 2 * t] = P[1 + 2 * s + 4 * t] - P[2 * s + 4 * t];
            py[s + 2 * t] = P[s + 2 + 4 * t] - P[s + 4 * t];
            pz[s + 2 * t] = P[s + 2 * t + 4] - P[s + 2 * t];
        }
    P2(g1p, gx);
    P2(g1p, gy);
    P2(g1p, gz);
    P2(g1p, px);
    P2(g1p, py);
    P2(g1p, pz);
    const T nk = -kc;
    T ax[4], ay[4], az[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        ax[j] = nk * (px[j] * ihx) * (gx[j] * ihx);
        ay[j] = nk * (py[j] * ihy) * (gy[j] * ihy);
        az[j] = nk * (pz[j] * ihz + rho_g) * (gz[j] * ihz);
    }
    P2(g1p, ax);
    P2(g1p, ay);
    P2(g1p, az);
#pragma unroll
    for (int z = 0; z < 2; z++)
#pragma unroll
        for (int y = 0; y < 2; y++)
#pragma unroll
            for (int x = 0; x < 2; x++)
                w[x + 2 * y + 4 * z] += cw8 * (ax[y + 2 * z] + ay[x + 2 * z] + az[x + 2 * y]);
}

template <typename T, int FIELD, int EPI, bool MASKED>
__global__ __launch_bounds__(256) void k_q1_apply(const OpDev *__restrict__ ops,
                                                  const WorkItem *__restrict__ work,
                                                  const T *__restrict__ X, T *__restrict__ Y,
                                                  EpiArgs<T> ep)
{
    __shared__ T xs[2][TB + 1][TB + 2];
    __shared__ T ps[FIELD ? 2 : 1][TB + 1][TB + 2];
    __shared__ T S4[4][TB][TB + 1];
    __shared__ double red[4];

    const WorkItem wi = work[blockIdx.x];
    if (ep.active && !ep.active[wi.inst]) return;
    const OpDev &o = ops[wi.inst];
    const int nx = o.nx, ny = o.ny, nz = o.nz, NZ = o.NZ, m = o.dmask;
    const int64_t plane = (int64_t)o.NX * o.NY;
    const T *__restrict__ Xi = X + o.off;
    T *__restrict__ Yi = Y + o.off;
    const T *__restrict__ Pi = FIELD ? static_cast<const T *>(o.P) : nullptr;
    const T *__restrict__ kk = static_cast<const T *>(o.k);
    const T *__restrict__ lamc = static_cast<const T *>(o.lam);
    const T *__restrict__ cTc = static_cast<const T *>(o.cT);

    const int tid = threadIdx.x, tx = tid % TB, ty = tid / TB;
    const int cx0 = wi.tx * OWN - 1, cy0 = wi.ty * OWN - 1;
    const int cx = cx0 + tx, cy = cy0 + ty;
    const bool cin = cx >= 0 && cx < nx && cy >= 0 && cy < ny;
    const int64_t cbase = cin ? (int64_t)cx + (int64_t)nx * cy : 0;
    const int64_t cplane = (int64_t)nx * ny;

    // node columns staged by this thread (flattened 17 x 17 halo tile)
    ColInfo lc[2];
    int lj[2], li[2];
#pragma unroll
    for (int s = 0; s < 2; s++) {
        int c = tid + s * 256;
        li[s] = c % (TB + 1);
        lj[s] = c / (TB + 1);
        if (c < NCOL) lc[s] = col_info(o, cx0 + li[s], cy0 + lj[s]);
        else lc[s].valid = 0;
    }
    // owned node column
    const bool owner = tx < OWN && ty < OWN;
    const int oi = cx0 + tx + 1, oj = cy0 + ty + 1;
    ColInfo oc = col_info(o, oi, oj);
    const bool own_ok = owner && oc.valid;
    int lr = -1;
    if (FIELD && o.lcol && own_ok) lr = o.lcol[oc.base];

    const T hx = T(o.hx), hy = T(o.hy), hz = T(o.hz);
    const T V = hx * hy * hz;
    const T cxx = hy * hz / hx, cyy = hx * hz / hy, czz = hx * hy / hz;
    const T cs = T(o.cs), cm = T(o.cm);
    const T ihx = T(1) / hx, ihy = T(1) / hy, ihz = T(1) / hz;
    const T rho_g = T(o.rho_g);
    const T cw8 = T(o.cadv) * V * T(0.125);

    auto load_plane = [&](int buf, int k) {
#pragma unroll
        for (int s = 0; s < 2; s++) {
            if (tid + s * 256 >= NCOL) continue;
            T v = T(0), pv = T(0);
            if (lc[s].valid && k >= 0 && k < NZ) {
                int64_t gi = lc[s].base + k * plane;
                v = Xi[gi];
                if (MASKED && constrained(lc[s], k, NZ, m)) v = T(0);
                if (FIELD) pv = Pi[gi];
            }
            xs[buf][lj[s]][li[s]] = v;
            if (FIELD) ps[FIELD ? buf : 0][lj[s]][li[s]] = pv;
        }
    };

    const int kb = wi.z0, ke = wi.z1;
    double acc = 0.0;
    T top[4] = {T(0), T(0), T(0), T(0)};
    int cur = 0;
    load_plane(0, kb - 1);
    for (int L = kb - 1; L < ke; L++) {
        const int nxt = cur ^ 1;
        load_plane(nxt, L + 1);
        const bool lay = cin && L >= 0 && L < nz;
        T kc = T(0), lam = T(0), cT = T(0);
        if (lay) {
            int64_t ci = cbase + (int64_t)L * cplane;
            kc = kk[ci];
            if (FIELD) { lam = lamc[ci]; cT = cTc[ci]; }
        }
        __syncthreads();
        T bot[4] = {T(0), T(0), T(0), T(0)}, tp[4] = {T(0), T(0), T(0), T(0)};
        if (lay) {
            T u[8], w[8];
#pragma unroll
            for (int a = 0; a < 4; a++) {
                u[a] = xs[cur][ty + (a >> 1)][tx + (a & 1)];
                u[a + 4] = xs[nxt][ty + (a >> 1)][tx + (a & 1)];
            }
            if (FIELD == 0) {
                cell_mass_stiff(u, cm * V, cs * kc, cxx, cyy, czz, w);
            } else {
                cell_mass_stiff(u, cT * V, cs * lam, cxx, cyy, czz, w);
                T pp[8];
#pragma unroll
                for (int a = 0; a < 4; a++) {
                    pp[a] = ps[FIELD ? cur : 0][ty + (a >> 1)][tx + (a & 1)];
                    pp[a + 4] = ps[FIELD ? nxt : 0][ty + (a >> 1)][tx + (a & 1)];
                }
                cell_convect(u, pp, kc, ihx, ihy, ihz, rho_g, cw8, w);
            }
#pragma unroll
            for (int a = 0; a < 4; a++) { bot[a] = w[a]; tp[a] = w[a + 4]; }
        }
        const bool emit = L >= kb;
        if (emit) {
#pragma unroll
            for (int a = 0; a < 4; a++) S4[a][ty][tx] = top[a] + bot[a];
        }
#pragma unroll
        for (int a = 0; a < 4; a++) top[a] = tp[a];
        __syncthreads();
        if (emit && own_ok && L < NZ) {
            T v = S4[3][ty][tx] + S4[2][ty][tx + 1] + S4[1][ty + 1][tx] + S4[0][ty + 1][tx + 1];
            const int64_t gi = oc.base + (int64_t)L * plane;
            if (FIELD && lr >= 0) {
                while (o.lrows[lr].col == (int)oc.base && o.lrows[lr].k < L) lr++;
                const LineRow row = o.lrows[lr];
                if (row.col == (int)oc.base && row.k == L && !(MASKED && row.row_constrained)) {
                    T la = T(0);
                    for (int e = row.beg; e < row.end; e++) {
                        const LineEnt en = o.lents[e];
                        if (MASKED && en.col_constrained) continue;
                        la += T(o.lcoef[en.src] * en.w) * Xi[en.col];
                    }
                    v += la;
                }
            }
            const bool con = MASKED && constrained(oc, L, NZ, m);
            if (con) v = Xi[gi];
            if (EPI == EPI_STORE) {
                Yi[gi] = v;
            } else if (EPI == EPI_RESID) {
                Yi[gi] = ep.b[o.off + gi] - v;
            } else if (EPI == EPI_RESID_NORM) {
                T r = ep.b[o.off + gi] - v;
                Yi[gi] = r;
                acc += (double)r * (double)r;
            } else if (EPI == EPI_DOT) {
                Yi[gi] = v;
                acc += (double)Xi[gi] * (double)v;
            } else if (EPI == EPI_CHEB) {
                const double *Sc = ep.S + (int64_t)wi.inst * NSLOT;
                T r = ep.b[o.off + gi] - v;
                T d = T(Sc[ep.s1]) * ep.d[o.off + gi] + T(Sc[ep.s2]) * ep.invd[o.off + gi] * r;
                ep.d[o.off + gi] = d;
                Yi[gi] = Xi[gi] + d;
            }
        }
        cur = nxt;
    }
    if (EPI == EPI_RESID_NORM || EPI == EPI_DOT) {
        double v = wave_sum(acc);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) ep.partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// ----------------------------------------------------------- setup kernels
__global__ void k_q1_inv_diag(OpDev o, double *__restrict__ out)
{
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= o.nnode) return;
    const int NX = o.NX, NY = o.NY;
    int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((int64_t)NX * NY));
    ColInfo c = col_info(o, i, j);
    if (constrained(c, k, o.NZ, o.dmask)) { out[n] = 1.0; return; }
    const double V = o.hx * o.hy * o.hz;
    const double kd = (o.hy * o.hz / o.hx + o.hx * o.hz / o.hy + o.hx * o.hy / o.hz) / 9.0;
    double d = 0.0;
    for (int dz = -1; dz <= 0; dz++)
        for (int dy = -1; dy <= 0; dy++)
            for (int dx = -1; dx <= 0; dx++) {
                int a = i + dx, b = j + dy, cc = k + dz;
                if (a < 0 || a >= o.nx || b < 0 || b >= o.ny || cc < 0 || cc >= o.nz) continue;
                int64_t ci = a + (int64_t)o.nx * (b + (int64_t)o.ny * cc);
                const double *K = static_cast<const double *>(o.k);
                if (o.field == 0) {
                    d += o.cm * V / 27.0 + o.cs * K[ci] * kd;
                } else {
                    const double *L = static_cast<const double *>(o.lam);
                    const double *CT = static_cast<const double *>(o.cT);
                    d += CT[ci] * V / 27.0 + o.cs * L[ci] * kd;
                }
            }
    out[n] = 1.0 / d;
}

__global__ void k_q1_stencil(OpDev o, double *__restrict__ S)
{
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= o.nnode) return;
    const int NX = o.NX, NY = o.NY, NZ = o.NZ;
    int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((int64_t)NX * NY));
    double st[27];
    for (int e = 0; e < 27; e++) st[e] = 0.0;
    ColInfo c = col_info(o, i, j);
    if (constrained(c, k, NZ, o.dmask)) {
        st[13] = 1.0;
    } else {
        const double h[3] = {o.hx, o.hy, o.hz};
        for (int dz = -1; dz <= 0; dz++)
            for (int dy = -1; dy <= 0; dy++)
                for (int dx = -1; dx <= 0; dx++) {
                    int cx = i + dx, cy = j + dy, cz = k + dz;
                    if (cx < 0 || cx >= o.nx || cy < 0 || cy >= o.ny || cz < 0 || cz >= o.nz) continue;
                    int64_t ci = cx + (int64_t)o.nx * (cy + (int64_t)o.ny * cz);
                    double mc, sc;
                    if (o.field == 0) {
                        mc = o.cm;
                        sc = o.cs * static_cast<const double *>(o.k)[ci];
                    } else {
                        mc = static_cast<const double *>(o.cT)[ci];
                        sc = o.cs * static_cast<const double *>(o.lam)[ci];
                    }
                    const int a[3] = {-dx, -dy, -dz};   // local corner of node n in the cell
                    for (int bz = 0; bz < 2; bz++)
                        for (int by = 0; by < 2; by++)
                            for (int bx = 0; bx < 2; bx++) {
                                int gi = cx + bx, gj = cy + by, gk = cz + bz;
                                ColInfo cb = col_info(o, gi, gj);
                                if (constrained(cb, gk, NZ, o.dmask)) continue;
                                const int b[3] = {bx, by, bz};
                                double mm[3], kk[3];
                                for (int d = 0; d < 3; d++) {
                                    bool same = a[d] == b[d];
                                    mm[d] = h[d] * (same ? 1.0 / 3.0 : 1.0 / 6.0);
                                    kk[d] = (same ? 1.0 : -1.0) / h[d];
                                }
                                double v = mc * mm[0] * mm[1] * mm[2] +
                                           sc * (kk[0] * mm[1] * mm[2] + mm[0] * kk[1] * mm[2] +
                                                 mm[0] * mm[1] * kk[2]);
                                int e = (gi - i + 1) + 3 * (gj - j + 1) + 9 * (gk - k + 1);
                                st[e] += v;
                            }
                }
    }
    for (int e = 0; e < 27; e++) S[(int64_t)e * o.nnode + n] = st[e];
}

__global__ void k_q1_cell_loads(OpDev o, const double *__restrict__ alpha,
                                const double *__restrict__ beta, double *__restrict__ y)
{
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= o.nnode) return;
    const int NX = o.NX, NY = o.NY;
    int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((int64_t)NX * NY));
    const double V8 = o.hx * o.hy * o.hz / 8.0, A4 = o.hx * o.hy / 4.0;
    double s = 0.0;
    for (int dz = -1; dz <= 0; dz++)
        for (int dy = -1; dy <= 0; dy++)
            for (int dx = -1; dx <= 0; dx++) {
                int cx = i + dx, cy = j + dy, cz = k + dz;
                if (cx < 0 || cx >= o.nx || cy < 0 || cy >= o.ny || cz < 0 || cz >= o.nz) continue;
                int64_t ci = cx + (int64_t)o.nx * (cy + (int64_t)o.ny * cz);
                if (alpha) s += alpha[ci] * V8;
                // node is the top corner (az = 1) when the cell lies below it
                if (beta) s += beta[ci] * A4 * (dz == -1 ? 1.0 : -1.0);
            }
    y[n] = s;
}

}  // namespace

// ---------------------------------------------------------------- launchers
template <typename T, int FIELD, bool MASKED>
static void dispatch_epi(int epi, const OpDev *ops, const WorkItem *work, int nwork, const T *x, T *y,
                         const EpiArgs<T> &ep, hipStream_t s)
{
    dim3 g(nwork), b(256);
    switch (epi) {
    case EPI_STORE: k_q1_apply<T, FIELD, EPI_STORE, MASKED><<<g, b, 0, s>>>(ops, work, x, y, ep); break;
    case EPI_RESID: k_q1_apply<T, FIELD, EPI_RESID, MASKED><<<g, b, 0, s>>>(ops, work, x, y, ep); break;
    case EPI_RESID_NORM:
        k_q1_apply<T, FIELD, EPI_RESID_NORM, MASKED><<<g, b, 0, s>>>(ops, work, x, y, ep);
        break;
    case EPI_DOT: k_q1_apply<T, FIELD, EPI_DOT, MASKED><<<g, b, 0, s>>>(ops, work, x, y, ep); break;
    case EPI_CHEB: k_q1_apply<T, FIELD, EPI_CHEB, MASKED><<<g, b, 0, s>>>(ops, work, x, y, ep); break;
    default: throw Error(-1, "bad epilogue");
    }
}

template <typename T>
void launch_q1(int field, int epi, bool masked, const OpDev *ops, const WorkItem *work, int nwork,
               const T *x, T *y, const EpiArgs<T> &ep, hipStream_t s)
{
    if (nwork <= 0) return;
    if (field == 0) {
        if (masked) dispatch_epi<T, 0, true>(epi, ops, work, nwork, x, y, ep, s);
        else dispatch_epi<T, 0, false>(epi, ops, work, nwork, x, y, ep, s);
    } else {
        if (masked) dispatch_epi<T, 1, true>(epi, ops, work, nwork, x, y, ep, s);
        else dispatch_epi<T, 1, false>(epi, ops, work, nwork, x, y, ep, s);
    }
    HTS_LAUNCH_CHECK();
}

template void launch_q1<double>(int, int, bool, const OpDev *, const WorkItem *, int, const double *,
                                double *, const EpiArgs<double> &, hipStream_t);
template void launch_q1<float>(int, int, bool, const OpDev *, const WorkItem *, int, const float *,
                               float *, const EpiArgs<float> &, hipStream_t);

void launch_q1_inv_diag(const OpDev &op, double *inv_diag, hipStream_t s)
{
    int64_t nb = (op.nnode + 255) / 256;
    k_q1_inv_diag<<<dim3((unsigned)nb), dim3(256), 0, s>>>(op, inv_diag);
    HTS_LAUNCH_CHECK();
}

void launch_q1_stencil(const OpDev &op, double *S, hipStream_t s)
{
    int64_t nb = (op.nnode + 127) / 128;
    k_q1_stencil<<<dim3((unsigned)nb), dim3(128), 0, s>>>(op, S);
    HTS_LAUNCH_CHECK();
}

void launch_q1_cell_loads(const OpDev &op, const double *alpha, const double *beta, double *y,
                          hipStream_t s)
{
    int64_t nb = (op.nnode + 255) / 256;
    k_q1_cell_loads<<<dim3((unsigned)nb), dim3(256), 0, s>>>(op, alpha, beta, y);
    HTS_LAUNCH_CHECK();
}

}  // namespace hts
