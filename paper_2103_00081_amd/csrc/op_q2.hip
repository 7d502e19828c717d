// Matrix-free Q2 operators of the pressure (Eq. 3) and heat (Eq. 4)
// equations on a uniform box (27-node hexahedra, 3-point Gauss rules).
//
// Kernel layout: a 256-thread workgroup owns the nodes of a 15 x 15 tile of
// cell columns (30 x 30 node columns) and marches upward through its range of
// node planes one cell layer at a time.  Each thread handles one cell column
// of the 16 x 16 cells that touch the owned nodes (one-cell halo on the low
// x/y side).  Per cell layer the three node planes of the layer are staged in
// LDS; each thread evaluates its cell's 27 outputs:
//   mass and stiffness by Kronecker sum factorisation with the 1D Q2
//   matrices  h/30 [4 2 -1; 2 16 2; -1 2 4]  and  1/(3h) [7 -8 1; -8 16 -8;
//   1 -8 7]  (exact for cellwise-constant coefficients);
//   the convection term at the 27 Gauss points from the gradients of T and P
//   (sum-factorised values and derivatives of the 1D basis).
// The cell writes its bottom- and middle-plane contributions to LDS and keeps
// its top plane for the next layer; the owner of a node adds the (up to
// four) cell contributions of its plane in a fixed order.  No atomics,
// bitwise reproducible, same epilogues as the Q1 kernel.
#include "common.h"
#include "dev_util.h"

namespace hts {

namespace {

constexpr int TC = 16;            // cell columns per tile edge
constexpr int OWNC = TC - 1;      // owned cells per tile edge
constexpr int NL = 2 * TC + 1;    // node columns per tile edge staged in LDS
constexpr int OWNN = 2 * OWNC;    // owned node columns per tile edge
constexpr int NOWN = OWNN * OWNN; // owned node columns per tile
constexpr int NSTAGE = NL * NL;   // staged node columns per tile
constexpr int SPT = (NSTAGE + 255) / 256;   // staged columns per thread
constexpr int OPT = (NOWN + 255) / 256;     // owned columns per thread

// 1D Q2 basis on [0, 1] with nodes 0, 1/2, 1 at the 3 Gauss points
constexpr double SQ35 = 0.77459666924148337704;   // sqrt(3/5)
constexpr double G0 = 0.5 - 0.5 * SQ35, G2 = 0.5 + 0.5 * SQ35;
constexpr double bN0(double x) { return (2 * x - 1) * (x - 1); }
constexpr double bN1(double x) { return 4 * x * (1 - x); }
constexpr double bN2(double x) { return x * (2 * x - 1); }
constexpr double dN0(double x) { return 4 * x - 3; }
constexpr double dN1(double x) { return 4 - 8 * x; }
constexpr double dN2(double x) { return 4 * x - 1; }

template <typename T>
struct Q2Tab {
    // B[q][i] = N_i(g_q), D[q][i] = N_i'(g_q), W[q] Gauss weights on [0, 1]
    static constexpr T B[3][3] = {{T(bN0(G0)), T(bN1(G0)), T(bN2(G0))},
                                  {T(0), T(1), T(0)},
                                  {T(bN0(G2)), T(bN1(G2)), T(bN2(G2))}};
    static constexpr T D[3][3] = {{T(dN0(G0)), T(dN1(G0)), T(dN2(G0))},
                                  {T(-1), T(0), T(1)},
                                  {T(dN0(G2)), T(dN1(G2)), T(dN2(G2))}};
    static constexpr T W[3] = {T(5.0 / 18.0), T(8.0 / 18.0), T(5.0 / 18.0)};
    // reference mass (h = 1) and stiffness (h = 1)
    static constexpr T M[3][3] = {{T(4.0 / 30), T(2.0 / 30), T(-1.0 / 30)},
                                  {T(2.0 / 30), T(16.0 / 30), T(2.0 / 30)},
                                  {T(-1.0 / 30), T(2.0 / 30), T(4.0 / 30)}};
    static constexpr T K[3][3] = {{T(7.0 / 3), T(-8.0 / 3), T(1.0 / 3)},
                                  {T(-8.0 / 3), T(16.0 / 3), T(-8.0 / 3)},
                                  {T(1.0 / 3), T(-8.0 / 3), T(7.0 / 3)}};
};

// The cell's 27 nodal values are read through an accessor (from the staged
// LDS planes) one z-plane at a time, so that only the 27 outputs and a few
// 9-value planes are live in registers.

// w = mV (M x M x M) u + sk (cxx K x M x M + cyy M x K x M + czz M x M x K) u
// (first factor along x), accumulated over the z-planes j of u:
//   p_j = (M_x M_y) u_j,  q_j = mV p_j + skx (K_x M_y) u_j + sky (M_x K_y) u_j,
//   w_k += M_z[k][j] q_j + skz K_z[k][j] p_j.
template <typename T, typename UAt>
__device__ __forceinline__ void q2_mass_stiff(const UAt &uat, T mV, T sk, T cxx, T cyy, T czz, T w[27])
{
    using Q = Q2Tab<T>;
    const T sky = sk * cyy, skz = sk * czz, skx = sk * cxx;
#pragma unroll
    for (int i = 0; i < 27; i++) w[i] = T(0);
#pragma unroll
    for (int j = 0; j < 3; j++) {
        // one node plane's values at a time (no hoisting of the next plane's reads)
        asm volatile("" ::: "memory");
        T v[9];
#pragma unroll
        for (int i = 0; i < 9; i++) v[i] = uat(i + 9 * j);
        // y pass (per x index a): my = M_y v, ky = K_y v
        T my[9], ky[9];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int r = 0; r < 3; r++) {
                my[a + 3 * r] = Q::M[r][0] * v[a] + Q::M[r][1] * v[a + 3] + Q::M[r][2] * v[a + 6];
                ky[a + 3 * r] = Q::K[r][0] * v[a] + Q::K[r][1] * v[a + 3] + Q::K[r][2] * v[a + 6];
            }
        // x pass (per y index b)
        T pj[9], qj[9];
#pragma unroll
        for (int b = 0; b < 3; b++)
#pragma unroll
            for (int r = 0; r < 3; r++) {
                const T pm = Q::M[r][0] * my[3 * b] + Q::M[r][1] * my[3 * b + 1] + Q::M[r][2] * my[3 * b + 2];
                const T kx = Q::K[r][0] * my[3 * b] + Q::K[r][1] * my[3 * b + 1] + Q::K[r][2] * my[3 * b + 2];
                const T mk = Q::M[r][0] * ky[3 * b] + Q::M[r][1] * ky[3 * b + 1] + Q::M[r][2] * ky[3 * b + 2];
                pj[r + 3 * b] = pm;
                qj[r + 3 * b] = mV * pm + skx * kx + sky * mk;
            }
        // z accumulation
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const T mz = Q::M[k][j], kz = skz * Q::K[k][j];
#pragma unroll
            for (int i = 0; i < 9; i++) w[i + 9 * k] += mz * qj[i] + kz * pj[i];
        }
    }
}

// w_a += cw sum_q W_q N_a(q) (q_h . grad u)(q), q_h = -k (grad P + rho_g e_z),
// cw = dt c_w V; 3 x 3 x 3 Gauss points, one z-plane of points at a time:
// the plane's z-contractions of P and u (values and z-derivatives at the 9
// node columns), then per row of points (fixed qy) the y- and x-contractions,
// the integrand at the three points of the row and its projection back onto
// the x and y basis functions, accumulated over the rows; the plane's sums
// go to the 27 outputs through the z basis values.  Only one plane's
// contractions and one row's values are live at a time.
template <typename T, typename UAt, typename PAt>
__device__ __forceinline__ void q2_convect(const UAt &uat, const PAt &pat, T kc, T ihx, T ihy, T ihz, T rho_g,
                                          T cw, T w[27])
{
    using Q = Q2Tab<T>;
    const T s0 = -kc * cw;
#pragma unroll 1
    for (int qz = 0; qz < 3; qz++) {
        // keeps the LDS reads of the nodal values inside the loop (read again
        // per plane of points instead of 54 values held across it)
        asm volatile("" ::: "memory");
        const T bz0 = Q::B[qz][0], bz1 = Q::B[qz][1], bz2 = Q::B[qz][2];
        const T dz0 = Q::D[qz][0], dz1 = Q::D[qz][1], dz2 = Q::D[qz][2];
        const T sz = s0 * Q::W[qz];
        T fp[9], fpz[9], fu[9], fuz[9];
#pragma unroll
        for (int ij = 0; ij < 9; ij++) {
            const T p0 = pat(ij), p1 = pat(ij + 9), p2 = pat(ij + 18);
            fp[ij] = bz0 * p0 + bz1 * p1 + bz2 * p2;
            fpz[ij] = dz0 * p0 + dz1 * p1 + dz2 * p2;
            const T u0 = uat(ij), u1 = uat(ij + 9), u2 = uat(ij + 18);
            fu[ij] = bz0 * u0 + bz1 * u1 + bz2 * u2;
            fuz[ij] = dz0 * u0 + dz1 * u1 + dz2 * u2;
        }
        T sacc[9];
#pragma unroll
        for (int i = 0; i < 9; i++) sacc[i] = T(0);
#pragma unroll
        for (int qy = 0; qy < 3; qy++) {
            T yp[3], ypd[3], ypz[3], yu[3], yud[3], yuz[3];
#pragma unroll
            for (int i = 0; i < 3; i++) {
                yp[i] = Q::B[qy][0] * fp[i] + Q::B[qy][1] * fp[i + 3] + Q::B[qy][2] * fp[i + 6];
                ypd[i] = Q::D[qy][0] * fp[i] + Q::D[qy][1] * fp[i + 3] + Q::D[qy][2] * fp[i + 6];
                ypz[i] = Q::B[qy][0] * fpz[i] + Q::B[qy][1] * fpz[i + 3] + Q::B[qy][2] * fpz[i + 6];
                yu[i] = Q::B[qy][0] * fu[i] + Q::B[qy][1] * fu[i + 3] + Q::B[qy][2] * fu[i + 6];
                yud[i] = Q::D[qy][0] * fu[i] + Q::D[qy][1] * fu[i + 3] + Q::D[qy][2] * fu[i + 6];
                yuz[i] = Q::B[qy][0] * fuz[i] + Q::B[qy][1] * fuz[i + 3] + Q::B[qy][2] * fuz[i + 6];
            }
            T a[3];
#pragma unroll
            for (int qx = 0; qx < 3; qx++) {
                const T gpx = Q::D[qx][0] * yp[0] + Q::D[qx][1] * yp[1] + Q::D[qx][2] * yp[2];
                const T gpy = Q::B[qx][0] * ypd[0] + Q::B[qx][1] * ypd[1] + Q::B[qx][2] * ypd[2];
                const T gpz = Q::B[qx][0] * ypz[0] + Q::B[qx][1] * ypz[1] + Q::B[qx][2] * ypz[2];
                const T gux = Q::D[qx][0] * yu[0] + Q::D[qx][1] * yu[1] + Q::D[qx][2] * yu[2];
                const T guy = Q::B[qx][0] * yud[0] + Q::B[qx][1] * yud[1] + Q::B[qx][2] * yud[2];
                const T guz = Q::B[qx][0] * yuz[0] + Q::B[qx][1] * yuz[1] + Q::B[qx][2] * yuz[2];
                const T sw = sz * (Q::W[qx] * Q::W[qy]);
                const T cxq = sw * ((gpx * ihx) * ihx);
                const T cyq = sw * ((gpy * ihy) * ihy);
                const T czq = sw * ((gpz * ihz + rho_g) * ihz);
                a[qx] = cxq * gux + cyq * guy + czq * guz;
            }
            // back onto the x basis functions, then the y basis functions of this row
#pragma unroll
            for (int i = 0; i < 3; i++) {
                const T t = Q::B[0][i] * a[0] + Q::B[1][i] * a[1] + Q::B[2][i] * a[2];
#pragma unroll
                for (int j = 0; j < 3; j++) sacc[i + 3 * j] += Q::B[qy][j] * t;
            }
        }
#pragma unroll
        for (int ij = 0; ij < 9; ij++) {
            w[ij] += bz0 * sacc[ij];
            w[ij + 9] += bz1 * sacc[ij];
            w[ij + 18] += bz2 * sacc[ij];
        }
    }
}

// Compact node-column data of the apply kernel (two registers per column
// instead of ColInfo's six): bf = instance-local node column index (bits
// 0..29), bit 30 valid, bit 31 constrained by an x/y face; dl = packed
// constrained z-range.  A node plane has fewer than 2^30 columns: a mesh
// has fewer than 2^31 nodes (checked when it is created) and at least two
// node planes.
struct ColQ {
    uint32_t bf;
    int32_t dl;
    __device__ __forceinline__ int base() const { return (int)(bf & 0x3FFFFFFFu); }
    __device__ __forceinline__ bool valid() const { return (bf >> 30) & 1u; }
    __device__ __forceinline__ bool xyc() const { return bf >> 31; }
};
__device__ __forceinline__ static ColQ colq(const OpDev &o, int i, int j)
{
    const ColInfo c = col_info(o, i, j);
    ColQ q;
    q.bf = (uint32_t)c.base | (c.valid ? 1u << 30 : 0u) | (c.xyc ? 1u << 31 : 0u);
    q.dl = c.dlo | (c.dhi << 16);
    return q;
}
__device__ __forceinline__ static bool constrained_q(const ColQ &c, int k, int NZ, int m)
{
    const int lo = c.dl & 0xFFFF, hi = (c.dl >> 16) & 0xFFFF;
    return c.xyc() || ((m & 16) && k == 0) || ((m & 32) && k == NZ - 1) || (k >= lo && k <= hi);
}

template <typename T, int FIELD, int EPI, bool MASKED, bool GRADED>
__global__ __launch_bounds__(256) void k_q2_apply(const OpDev *__restrict__ ops,
                                                  const WorkItem *__restrict__ work,
                                                  const T *__restrict__ X, T *__restrict__ Y,
                                                  EpiArgs<T> ep)
{
    __shared__ T xs[3][NL][NL + 1];
    __shared__ T ps[FIELD ? 3 : 1][FIELD ? NL : 1][FIELD ? NL + 1 : 1];
    // heat: one node plane of cell contributions at a time (keeps the
    // workgroup's LDS under half a CU's); pressure: two
    constexpr bool ONEP = FIELD == 1;
    __shared__ T C[ONEP ? 1 : 2][9][256];
    __shared__ double red[4];

    const WorkItem wi = work[blockIdx.x];
    if (ep.active && !ep.active[wi.inst]) return;
    const OpDev &o = ops[wi.inst];
    const int nx = o.nx, ny = o.ny, nz = o.nz, NZ = o.NZ, m = o.dmask;
    const int64_t plane = (int64_t)o.NX * o.NY;
    const T *__restrict__ Xi = X + o.off;
    T *__restrict__ Yi = Y + o.off;
    const T HTS_GLOBAL *__restrict__ Pi = gptr<T>(FIELD ? o.P : nullptr);
    const T HTS_GLOBAL *__restrict__ kk = gptr<T>(o.k);
    const T HTS_GLOBAL *__restrict__ lamc = gptr<T>(o.lam);
    const T HTS_GLOBAL *__restrict__ cTc = gptr<T>(o.cT);
    const T *__restrict__ Bi = (EPI == EPI_RESID || EPI == EPI_RESID_NORM || EPI == EPI_CHEB) ? ep.b + o.off : nullptr;
    T *__restrict__ Di = EPI == EPI_CHEB ? ep.d + o.off : nullptr;
    const T *__restrict__ Ii = EPI == EPI_CHEB ? ep.invd + o.off : nullptr;

    const int tid = threadIdx.x, tx = tid % TC, ty = tid / TC;
    const int cx0 = wi.tx * OWNC - 1, cy0 = wi.ty * OWNC - 1;   // first (halo) cell of the tile
    const int cx = cx0 + tx, cy = cy0 + ty;
    const bool cin = cx >= 0 && cx < nx && cy >= 0 && cy < ny;
    const int64_t cbase = cin ? (int64_t)cx + (int64_t)nx * cy : 0;
    const int64_t cplane = (int64_t)nx * ny;
    const int nx0 = 2 * cx0, ny0 = 2 * cy0;                     // node of local column 0

    // staged node columns of this thread: column tid + 256 s of the staged
    // 33 x 33 (local coordinates recomputed where used)
    ColQ sc[SPT];
#pragma unroll
    for (int s = 0; s < SPT; s++) {
        const int c = tid + 256 * s;
        if (c < NSTAGE) sc[s] = colq(o, nx0 + c % NL, ny0 + c / NL);
        else sc[s] = ColQ{0u, DCOL_NONE};
    }
    // owned node columns of this thread: column tid + 256 s of the owned
    // 30 x 30 (local columns 2 .. 31)
    ColQ oc[OPT];
    int lr[OPT];
#pragma unroll
    for (int s = 0; s < OPT; s++) {
        const int c = tid + 256 * s;
        if (c < NOWN) oc[s] = colq(o, nx0 + 2 + c % OWNN, ny0 + 2 + c / OWNN);
        else oc[s] = ColQ{0u, DCOL_NONE};
        lr[s] = -1;
        if (FIELD && o.lcol && oc[s].valid()) lr[s] = gptr<int32_t>(o.lcol)[oc[s].base()];
    }

    const T hx = T(o.hx), hy = T(o.hy), hz = T(o.hz);
    const T V = hx * hy * hz;
    const T cxx = hy * hz / hx, cyy = hx * hz / hy, czz = hx * hy / hz;
    // graded meshes: this thread's cell column sizes (the layer height is
    // read per layer and the factors formed there)
    const bool graded = GRADED && o.hzs != nullptr;
    T ghx = hx, ghy = hy;
    if (graded) {
        ghx = T(o.hxs[cx < 0 ? 0 : (cx >= nx ? nx - 1 : cx)]);
        ghy = T(o.hys[cy < 0 ? 0 : (cy >= ny ? ny - 1 : cy)]);
    }
    const T cs = T(o.cs), cm = T(o.cm);
    const T ihx = T(1) / hx, ihy = T(1) / hy, ihz = T(1) / hz;
    const T rho_g = T(o.rho_g);
    const T cw = T(o.cadv) * V;
    T c1 = T(0), c2 = T(0);
    if (EPI == EPI_CHEB) {
        const double *Sc = ep.S + (int64_t)wi.inst * NSLOT;
        c1 = T(Sc[ep.s1]);
        c2 = T(Sc[ep.s2]);
    }

    // node plane k (k >= -2) lives in LDS slot (k + 6) % 3
    auto stage = [&](int k) {
        const int b = (k + 6) % 3;
        const int kc = k < 0 ? 0 : (k >= NZ ? NZ - 1 : k);
#pragma unroll
        for (int s = 0; s < SPT; s++) {
            const int c = tid + 256 * s;
            if (c >= NSTAGE) continue;
            const int li = c % NL, lj = c / NL;
            const bool val = sc[s].valid();
            const bool in = val && k >= 0 && k < NZ;
            const int64_t gi = val ? (int64_t)sc[s].base() + kc * plane : 0;
            bool keep = in;
            if (MASKED) keep = keep && !constrained_q(sc[s], k, NZ, m);
            const T xv = Xi[gi];
            xs[b][lj][li] = keep ? xv : T(0);
            if (FIELD) {
                const T pv = Pi[gi];
                ps[FIELD ? b : 0][FIELD ? lj : 0][FIELD ? li : 0] = in ? pv : T(0);
            }
        }
    };

    // pressure: the two node planes of the next cell layer are loaded into
    // registers while this layer is computed (the heat kernel has no
    // registers to spare for it and stages synchronously)
    constexpr bool PF = FIELD == 0;
    T nxa[PF ? SPT : 1], nxb[PF ? SPT : 1];
    auto fetch = [&](int k, T *dst) {
        const int kc = k < 0 ? 0 : (k >= NZ ? NZ - 1 : k);
#pragma unroll
        for (int s = 0; s < SPT; s++) {
            const int64_t gi = sc[s].valid() ? (int64_t)sc[s].base() + kc * plane : 0;
            dst[s] = Xi[gi];
        }
    };
    auto put = [&](int k, const T *src) {
        const int b = (k + 6) % 3;
#pragma unroll
        for (int s = 0; s < SPT; s++) {
            const int c = tid + 256 * s;
            if (c >= NSTAGE) continue;
            bool keep = sc[s].valid() && k >= 0 && k < NZ;
            if (MASKED) keep = keep && !constrained_q(sc[s], k, NZ, m);
            xs[b][c / NL][c % NL] = keep ? src[s] : T(0);
        }
    };

    const int z0 = wi.z0, z1 = wi.z1;            // owned node planes, z0 even
    const int L0 = z0 / 2 - 1, L1 = (z1 - 1) / 2;  // cell layers marched
    double acc = 0.0;
    // pressure: the cell's top-plane contributions wait in registers for the
    // next layer; heat: in the thread's own slots of C
    T top[ONEP ? 1 : 9];
#pragma unroll
    for (int a = 0; a < (ONEP ? 1 : 9); a++) top[a] = T(0);
    if (ONEP) {
#pragma unroll
        for (int a = 0; a < 9; a++) C[0][a][tid] = T(0);
    }

    // the owners of node plane P0 = 2L + h add the cell contributions in Cp
    auto gather = [&](int h, int L, const T (*Cp)[256]) {
        const int P0 = 2 * L + h;
        if (P0 < z0 || P0 >= z1 || P0 >= NZ) return;
#pragma unroll
        for (int s = 0; s < OPT; s++) {
            const int c = tid + 256 * s;
            if (c >= NOWN || !oc[s].valid()) continue;
            // cells around the node: x index i (local node column li)
            const int li = 2 + c % OWNN, lj = 2 + c / OWNN;
            int cxs[2], ixs[2], ncx, cys[2], iys[2], ncy;
            if (li & 1) { cxs[0] = li >> 1; ixs[0] = 1; ncx = 1; }
            else { cxs[0] = (li >> 1) - 1; ixs[0] = 2; cxs[1] = li >> 1; ixs[1] = 0; ncx = 2; }
            if (lj & 1) { cys[0] = lj >> 1; iys[0] = 1; ncy = 1; }
            else { cys[0] = (lj >> 1) - 1; iys[0] = 2; cys[1] = lj >> 1; iys[1] = 0; ncy = 2; }
            T v = T(0);
            for (int b = 0; b < ncy; b++)
                for (int a = 0; a < ncx; a++) {
                    const int cell = cxs[a] + TC * cys[b];
                    v += Cp[ixs[a] + 3 * iys[b]][cell];
                }
            const int64_t gi = (int64_t)oc[s].base() + (int64_t)P0 * plane;
            if (FIELD && lr[s] >= 0) {
                const LineRow HTS_GLOBAL *rows = gptr<LineRow>(o.lrows);
                const LineEnt HTS_GLOBAL *ents = gptr<LineEnt>(o.lents);
                const double HTS_GLOBAL *lco = gptr<double>(o.lcoef);
                int r = lr[s];
                while (rows[r].col == oc[s].base() && rows[r].k < P0) r++;
                lr[s] = r;
                if (rows[r].col == oc[s].base() && rows[r].k == P0 && !(MASKED && rows[r].row_constrained)) {
                    T la = T(0);
                    for (int e = rows[r].beg; e < rows[r].end; e++) {
                        if (MASKED && ents[e].col_constrained) continue;
                        la += T(lco[ents[e].src] * ents[e].w) * Xi[ents[e].col];
                    }
                    v += la;
                }
            }
            T ex = T(0);
            if (EPI == EPI_CHEB || EPI == EPI_DOT || MASKED) ex = Xi[gi];
            if (MASKED && constrained_q(oc[s], P0, NZ, m)) v = ex;
            if (EPI == EPI_STORE) {
                Yi[gi] = v;
            } else if (EPI == EPI_RESID) {
                Yi[gi] = Bi[gi] - v;
            } else if (EPI == EPI_RESID_NORM) {
                const T r = Bi[gi] - v;
                Yi[gi] = r;
                acc += (double)r * (double)r;
            } else if (EPI == EPI_DOT) {
                Yi[gi] = v;
                acc += (double)ex * (double)v;
            } else if (EPI == EPI_CHEB) {
                const T r = Bi[gi] - v;
                const T d = c1 * Di[gi] + c2 * Ii[gi] * r;
                Di[gi] = d;
                Yi[gi] = ex + d;
            }
        }
    };

    stage(2 * L0);
    if (PF) {
        fetch(2 * L0 + 1, nxa);
        fetch(2 * L0 + 2, nxb);
    }
    for (int L = L0; L <= L1; L++) {
        if (PF) {
            put(2 * L + 1, nxa);
            put(2 * L + 2, nxb);
        } else {
            stage(2 * L + 1);
            stage(2 * L + 2);
        }
        T ck = T(0), cl = T(0), cc = T(0);
        const bool lay = cin && L >= 0 && L < nz;
        if (lay) {
            const int64_t ci = cbase + (int64_t)L * cplane;
            ck = kk[ci];
            if (FIELD) { cl = lamc[ci]; cc = cTc[ci]; }
        }
        if (PF && L < L1) {
            fetch(2 * L + 3, nxa);
            fetch(2 * L + 4, nxb);
        }
        __syncthreads();
        T w[27];
        if (lay) {
            // node a + 3 b + 9 c of the cell: staged plane 2L + c, local column (2 tx + a, 2 ty + b)
            const int s0 = (2 * L + 6) % 3, s1 = (2 * L + 7) % 3, s2 = (2 * L + 8) % 3;
            auto uat = [&](int i) -> T {
                const int c = i / 9, b = (i / 3) % 3, a = i % 3;
                return xs[c == 0 ? s0 : (c == 1 ? s1 : s2)][2 * ty + b][2 * tx + a];
            };
            T lV = V, lcxx = cxx, lcyy = cyy, lczz = czz, lihx = ihx, lihy = ihy, lihz = ihz, lcw = cw;
            if (graded) {
                const T lhz = T(o.hzs[L]);
                lV = ghx * ghy * lhz;
                lcxx = ghy * lhz / ghx;
                lcyy = ghx * lhz / ghy;
                lczz = ghx * ghy / lhz;
                lihx = T(1) / ghx;
                lihy = T(1) / ghy;
                lihz = T(1) / lhz;
                lcw = T(o.cadv) * lV;
            }
            if (FIELD == 0) {
                q2_mass_stiff(uat, cm * lV, cs * ck, lcxx, lcyy, lczz, w);
            } else {
                q2_mass_stiff(uat, cc * lV, cs * cl, lcxx, lcyy, lczz, w);
                auto pat = [&](int i) -> T {
                    const int c = i / 9, b = (i / 3) % 3, a = i % 3;
                    return ps[FIELD ? (c == 0 ? s0 : (c == 1 ? s1 : s2)) : 0][FIELD ? 2 * ty + b : 0]
                             [FIELD ? 2 * tx + a : 0];
                };
                q2_convect(uat, pat, ck, lihx, lihy, lihz, rho_g, lcw, w);
            }
        } else {
#pragma unroll
            for (int a = 0; a < 27; a++) w[a] = T(0);
        }
        if (!ONEP) {
            // both planes at once, one barrier
#pragma unroll
            for (int a = 0; a < 9; a++) {
                C[0][a][tid] = top[a] + w[a];
                C[ONEP ? 0 : 1][a][tid] = w[a + 9];
                top[a] = w[a + 18];
            }
            __syncthreads();
            gather(0, L, C[0]);
            gather(1, L, C[ONEP ? 0 : 1]);
        } else {
            // node plane 2L: the previous layer's top contributions (already in
            // the thread's slots) plus this layer's bottom ones
#pragma unroll
            for (int a = 0; a < 9; a++) C[0][a][tid] += w[a];
            __syncthreads();
            gather(0, L, C[0]);
            __syncthreads();
#pragma unroll
            for (int a = 0; a < 9; a++) C[0][a][tid] = w[a + 9];
            __syncthreads();
            gather(1, L, C[0]);
            __syncthreads();
#pragma unroll
            for (int a = 0; a < 9; a++) C[0][a][tid] = w[a + 18];
        }
    }
    if (EPI == EPI_RESID_NORM || EPI == EPI_DOT) {
        double v = wave_sum(acc);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) ep.partial[wi.slot] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// ----------------------------------------------------------- setup kernels
// cells around node index g along one axis with the node's local index in each
__device__ __forceinline__ int q2_cells(int g, int ncell, int *c, int *loc)
{
    int n = 0;
    if (g & 1) {
        c[0] = g >> 1; loc[0] = 1; n = 1;
    } else {
        if ((g >> 1) - 1 >= 0) { c[n] = (g >> 1) - 1; loc[n] = 2; n++; }
        if ((g >> 1) < ncell) { c[n] = g >> 1; loc[n] = 0; n++; }
    }
    return n;
}

// size of cell c along axis d (graded meshes: from the per-axis tables)
__device__ __forceinline__ static double cell_h(const OpDev &o, int d, int c)
{
    if (d == 0) return o.hxs ? o.hxs[c] : o.hx;
    if (d == 1) return o.hys ? o.hys[c] : o.hy;
    return o.hzs ? o.hzs[c] : o.hz;
}

__global__ void k_q2_inv_diag(OpDev o, double *__restrict__ out)
{
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= o.nnode) return;
    const int NX = o.NX, NY = o.NY;
    int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((int64_t)NX * NY));
    ColInfo c = col_info(o, i, j);
    if (constrained(c, k, o.NZ, o.dmask)) { out[n] = 1.0; return; }
    const double md[3] = {4.0 / 30, 16.0 / 30, 4.0 / 30}, kd[3] = {7.0 / 3, 16.0 / 3, 7.0 / 3};
    int cx[2], lx[2], cy[2], ly[2], cz[2], lz[2];
    const int nxc = q2_cells(i, o.nx, cx, lx), nyc = q2_cells(j, o.ny, cy, ly), nzc = q2_cells(k, o.nz, cz, lz);
    double d = 0.0;
    for (int c3 = 0; c3 < nzc; c3++)
        for (int b = 0; b < nyc; b++)
            for (int a = 0; a < nxc; a++) {
                const int64_t ci = cx[a] + (int64_t)o.nx * (cy[b] + (int64_t)o.ny * cz[c3]);
                const double hx = cell_h(o, 0, cx[a]), hy = cell_h(o, 1, cy[b]), hz = cell_h(o, 2, cz[c3]);
                const double V = hx * hy * hz;
                const double cxx = hy * hz / hx, cyy = hx * hz / hy, czz = hx * hy / hz;
                const double mx = md[lx[a]], my = md[ly[b]], mz = md[lz[c3]];
                const double kx = kd[lx[a]], ky = kd[ly[b]], kz = kd[lz[c3]];
                double mc, sc;
                if (o.field == 0) {
                    mc = o.cm;
                    sc = o.cs * static_cast<const double *>(o.k)[ci];
                } else {
                    mc = static_cast<const double *>(o.cT)[ci];
                    sc = o.cs * static_cast<const double *>(o.lam)[ci];
                }
                d += mc * V * mx * my * mz + sc * (cxx * kx * my * mz + cyy * mx * ky * mz + czz * mx * my * kz);
            }
    out[n] = 1.0 / d;
}

// y_a = sum_c alpha_c int N_a + beta_c int dN_a/dz
__global__ void k_q2_cell_loads(OpDev o, const double *__restrict__ alpha, const double *__restrict__ beta,
                                double *__restrict__ y)
{
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= o.nnode) return;
    const int NX = o.NX, NY = o.NY;
    int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((int64_t)NX * NY));
    const double wint[3] = {1.0 / 6, 2.0 / 3, 1.0 / 6};   // int_0^1 N_i
    const double dend[3] = {-1.0, 0.0, 1.0};              // N_i(1) - N_i(0)
    int cx[2], lx[2], cy[2], ly[2], cz[2], lz[2];
    const int nxc = q2_cells(i, o.nx, cx, lx), nyc = q2_cells(j, o.ny, cy, ly), nzc = q2_cells(k, o.nz, cz, lz);
    double s = 0.0;
    for (int c3 = 0; c3 < nzc; c3++)
        for (int b = 0; b < nyc; b++)
            for (int a = 0; a < nxc; a++) {
                const int64_t ci = cx[a] + (int64_t)o.nx * (cy[b] + (int64_t)o.ny * cz[c3]);
                const double hx = cell_h(o, 0, cx[a]), hy = cell_h(o, 1, cy[b]), hz = cell_h(o, 2, cz[c3]);
                const double V = hx * hy * hz, A = hx * hy;
                const double wxy = wint[lx[a]] * wint[ly[b]];
                if (alpha) s += alpha[ci] * V * wxy * wint[lz[c3]];
                if (beta) s += beta[ci] * A * wxy * dend[lz[c3]];
            }
    y[n] = s;
}

}  // namespace

// ---------------------------------------------------------------- launchers
template <typename T, int FIELD, int EPI, bool MASKED, bool G>
static void launch_k2(int nwork, const OpDev *ops, const WorkItem *work, const T *x, T *y, const EpiArgs<T> &ep,
                      hipStream_t s)
{
    k_q2_apply<T, FIELD, EPI, MASKED, G><<<dim3(nwork), dim3(256), 0, s>>>(ops, work, x, y, ep);
}

template <typename T, int FIELD, bool MASKED, bool G>
static void dispatch_epi2(int epi, const OpDev *ops, const WorkItem *work, int nwork, const T *x, T *y,
                          const EpiArgs<T> &ep, hipStream_t s)
{
    switch (epi) {
    case EPI_STORE: launch_k2<T, FIELD, EPI_STORE, MASKED, G>(nwork, ops, work, x, y, ep, s); break;
    case EPI_RESID: launch_k2<T, FIELD, EPI_RESID, MASKED, G>(nwork, ops, work, x, y, ep, s); break;
    case EPI_RESID_NORM: launch_k2<T, FIELD, EPI_RESID_NORM, MASKED, G>(nwork, ops, work, x, y, ep, s); break;
    case EPI_DOT: launch_k2<T, FIELD, EPI_DOT, MASKED, G>(nwork, ops, work, x, y, ep, s); break;
    case EPI_CHEB: launch_k2<T, FIELD, EPI_CHEB, MASKED, G>(nwork, ops, work, x, y, ep, s); break;
    default: throw Error(-1, "bad epilogue");
    }
}

template <typename T, bool G>
static void launch_q2_g(int field, int epi, bool masked, const OpDev *ops, const WorkItem *work, int nwork,
                        const T *x, T *y, const EpiArgs<T> &ep, hipStream_t s)
{
    if (field == 0) {
        if (masked) dispatch_epi2<T, 0, true, G>(epi, ops, work, nwork, x, y, ep, s);
        else dispatch_epi2<T, 0, false, G>(epi, ops, work, nwork, x, y, ep, s);
    } else {
        if (masked) dispatch_epi2<T, 1, true, G>(epi, ops, work, nwork, x, y, ep, s);
        else dispatch_epi2<T, 1, false, G>(epi, ops, work, nwork, x, y, ep, s);
    }
}

// graded: some instance has a graded mesh (those kernels form the cell
// factors per layer)
template <typename T>
void launch_q2(int field, int epi, bool masked, bool graded, const OpDev *ops, const WorkItem *work, int nwork,
               const T *x, T *y, const EpiArgs<T> &ep, hipStream_t s)
{
    if (nwork <= 0) return;
    if (graded) launch_q2_g<T, true>(field, epi, masked, ops, work, nwork, x, y, ep, s);
    else launch_q2_g<T, false>(field, epi, masked, ops, work, nwork, x, y, ep, s);
    HTS_LAUNCH_CHECK();
}

template void launch_q2<double>(int, int, bool, bool, const OpDev *, const WorkItem *, int, const double *,
                                double *, const EpiArgs<double> &, hipStream_t);
template void launch_q2<float>(int, int, bool, bool, const OpDev *, const WorkItem *, int, const float *, float *,
                               const EpiArgs<float> &, hipStream_t);

void launch_q2_inv_diag(const OpDev &op, double *inv_diag, hipStream_t s)
{
    int64_t nb = (op.nnode + 255) / 256;
    k_q2_inv_diag<<<dim3((unsigned)nb), dim3(256), 0, s>>>(op, inv_diag);
    HTS_LAUNCH_CHECK();
}

void launch_q2_cell_loads(const OpDev &op, const double *alpha, const double *beta, double *y, hipStream_t s)
{
    int64_t nb = (op.nnode + 255) / 256;
    k_q2_cell_loads<<<dim3((unsigned)nb), dim3(256), 0, s>>>(op, alpha, beta, y);
    HTS_LAUNCH_CHECK();
}

}  // namespace hts
