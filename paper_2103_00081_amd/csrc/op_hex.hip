// Matrix-free Q1 operators of the pressure (Eq. 3) and heat (Eq. 4)
// equations on general hexahedra of the box topology (every node has its own
// coordinates; Section 3.3 meshes the site with hexahedra refined around the
// piles, Fig. 10b).
//
// Each cell is the trilinear (isoparametric) image of the unit cube, so its
// Jacobian varies inside the cell: the integrals are taken with the 2 x 2 x 2
// Gauss rule, as on the box, but every Gauss point forms J from the cell's
// eight vertices, its cofactor matrix C (J^-1 = C^T / det J) and det J.  With
// the reference gradients R_a of the basis and g = sum_a u_a R_a,
//   grad N_a . grad u = R_a . (C^T C g) / det^2,   dV = det dxi,
// so the stiffness contribution to node a is R_a . f with f = w s C^T C g /
// det, and mass and convection add w det (m u(xi) + c_adv q . grad u) N_a,
// q = -k (C g_P / det + rho_g e_z).  The reference derivatives of a trilinear
// field are bilinear interpolations of its four edge differences along that
// axis, which is how J, g and g_P are formed.
//
// Kernel layout as the narrow-tile box kernel: a 256-thread workgroup owns a
// 15 x 15 tile of node columns and computes the 16 x 16 cells around it,
// marching up through node planes with x (and P) planes and the node
// coordinate planes staged in 3-deep LDS rings and the cell corner sums in a
// 2-deep ring; the owner of a node adds the contributions of its eight cells
// in a fixed order (no atomics, bitwise reproducible).  Coordinates stay FP64
// in LDS; the FP32 operators form the geometry from FP64 differences to the
// cell's first vertex, rounded once.  Line sources and Dirichlet columns need
// vertical node columns and are not available on these meshes.
#include "common.h"
#include "dev_util.h"

namespace hts {

namespace {

constexpr int HB = 16;             // cell columns per tile edge
constexpr int HOWN = HB - 1;       // owned node columns per tile edge
constexpr int HCOL = (HB + 1) * (HB + 1);

// 2-point Gauss rule on [0, 1]
constexpr double HG0 = 0.21132486540518711775, HG1 = 0.78867513459481288225;

// One cell: w[a] = contributions of the cell to node a (a = ax + 2 ay + 4 az)
// of  m (v, u) + s (grad v, grad u) + cadv (v, q . grad u).
// X: vertex coordinates relative to vertex 0; P: nodal pressure (ADV only).
template <typename T, bool ADV>
__device__ __forceinline__ void hex_cell(const T (&X)[8][3], const T (&u)[8], const T (&P)[8], T m, T s,
                                         T cadvk, T rho_g, T (&w)[8])
{
    // edge differences along x (index b + 2c), y (a + 2c), z (a + 2b)
    T ex[4][3], ey[4][3], ez[4][3], ux[4], uy[4], uz[4], px[4], py[4], pz[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const int b = e & 1, c = e >> 1;
        const int nx0 = 2 * b + 4 * c, ny0 = b + 4 * c, nz0 = b + 2 * c;   // b, c: the two other indices
#pragma unroll
        for (int d = 0; d < 3; d++) {
            ex[e][d] = X[nx0 + 1][d] - X[nx0][d];
            ey[e][d] = X[ny0 + 2][d] - X[ny0][d];
            ez[e][d] = X[nz0 + 4][d] - X[nz0][d];
        }
        ux[e] = u[nx0 + 1] - u[nx0];
        uy[e] = u[ny0 + 2] - u[ny0];
        uz[e] = u[nz0 + 4] - u[nz0];
        if (ADV) {
            px[e] = P[nx0 + 1] - P[nx0];
            py[e] = P[ny0 + 2] - P[ny0];
            pz[e] = P[nz0 + 4] - P[nz0];
        }
    }
#pragma unroll
    for (int a = 0; a < 8; a++) w[a] = T(0);
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const T gx = (q & 1) ? T(HG1) : T(HG0), gy = (q & 2) ? T(HG1) : T(HG0), gz = (q & 4) ? T(HG1) : T(HG0);
        const T Nx[2] = {T(1) - gx, gx}, Ny[2] = {T(1) - gy, gy}, Nz[2] = {T(1) - gz, gz};
        // bilinear weights of the edges along each axis
        const T wx[4] = {Ny[0] * Nz[0], Ny[1] * Nz[0], Ny[0] * Nz[1], Ny[1] * Nz[1]};
        const T wy[4] = {Nx[0] * Nz[0], Nx[1] * Nz[0], Nx[0] * Nz[1], Nx[1] * Nz[1]};
        const T wz[4] = {Nx[0] * Ny[0], Nx[1] * Ny[0], Nx[0] * Ny[1], Nx[1] * Ny[1]};
        T J[3][3];   // J[i][j] = d x_i / d xi_j
#pragma unroll
        for (int i = 0; i < 3; i++) {
            J[i][0] = wx[0] * ex[0][i] + wx[1] * ex[1][i] + wx[2] * ex[2][i] + wx[3] * ex[3][i];
            J[i][1] = wy[0] * ey[0][i] + wy[1] * ey[1][i] + wy[2] * ey[2][i] + wy[3] * ey[3][i];
            J[i][2] = wz[0] * ez[0][i] + wz[1] * ez[1][i] + wz[2] * ez[2][i] + wz[3] * ez[3][i];
        }
        T C[3][3];   // cofactors: (J^-1)_{ji} = C_ij / det
        C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const T det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
        const T idet = T(1) / det;
        // reference gradient of u, det * physical gradient
        const T g[3] = {wx[0] * ux[0] + wx[1] * ux[1] + wx[2] * ux[2] + wx[3] * ux[3],
                        wy[0] * uy[0] + wy[1] * uy[1] + wy[2] * uy[2] + wy[3] * uy[3],
                        wz[0] * uz[0] + wz[1] * uz[1] + wz[2] * uz[2] + wz[3] * uz[3]};
        T cg[3];
#pragma unroll
        for (int i = 0; i < 3; i++) cg[i] = C[i][0] * g[0] + C[i][1] * g[1] + C[i][2] * g[2];
        // stiffness: f = (1/8) s C^T C g / det, contributions R_a . f
        const T sc = T(0.125) * s * idet;
        T f[3];
#pragma unroll
        for (int j = 0; j < 3; j++) f[j] = sc * (C[0][j] * cg[0] + C[1][j] * cg[1] + C[2][j] * cg[2]);
        // mass (and convection): (1/8) det (m u(xi) + cadv q . grad u)
        const T uq = Nz[0] * (Ny[0] * (Nx[0] * u[0] + Nx[1] * u[1]) + Ny[1] * (Nx[0] * u[2] + Nx[1] * u[3])) +
                     Nz[1] * (Ny[0] * (Nx[0] * u[4] + Nx[1] * u[5]) + Ny[1] * (Nx[0] * u[6] + Nx[1] * u[7]));
        T mm = m * uq * det;
        if (ADV) {
            const T gp[3] = {wx[0] * px[0] + wx[1] * px[1] + wx[2] * px[2] + wx[3] * px[3],
                             wy[0] * py[0] + wy[1] * py[1] + wy[2] * py[2] + wy[3] * py[3],
                             wz[0] * pz[0] + wz[1] * pz[1] + wz[2] * pz[2] + wz[3] * pz[3]};
            // det * (grad P + rho_g e_z) . (det grad u) / det
            const T gpx = C[0][0] * gp[0] + C[0][1] * gp[1] + C[0][2] * gp[2];
            const T gpy = C[1][0] * gp[0] + C[1][1] * gp[1] + C[1][2] * gp[2];
            const T gpz = C[2][0] * gp[0] + C[2][1] * gp[1] + C[2][2] * gp[2] + rho_g * det;
            mm -= cadvk * (gpx * cg[0] + gpy * cg[1] + gpz * cg[2]) * idet;
        }
        mm *= T(0.125);
#pragma unroll
        for (int a = 0; a < 8; a++) {
            const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
            const T sx = ax ? T(1) : T(-1), sy = ay ? T(1) : T(-1), sz = az ? T(1) : T(-1);
            w[a] += f[0] * sx * Ny[ay] * Nz[az] + f[1] * Nx[ax] * sy * Nz[az] + f[2] * Nx[ax] * Ny[ay] * sz +
                    mm * Nx[ax] * Ny[ay] * Nz[az];
        }
    }
}

template <typename T, int FIELD, int EPI, bool MASKED>
__global__ __launch_bounds__(256) void k_hex_apply(const OpDev *__restrict__ ops, const WorkItem *__restrict__ work,
                                                   const T *__restrict__ X, T *__restrict__ Y, EpiArgs<T> ep)
{
    constexpr bool HEAT = FIELD == 1;
    __shared__ T xs[3][HB + 1][HB + 2];
    __shared__ T ps[HEAT ? 3 : 1][HEAT ? HB + 1 : 1][HEAT ? HB + 2 : 1];
    __shared__ double cs[3][3][HB + 1][HB + 2];   // [slot][axis][j][i]
    __shared__ T S4[2][4][HB][HB + 1];
    __shared__ double red[4];

    const WorkItem wi = work[blockIdx.x];
    if (ep.active && !ep.active[wi.inst]) return;
    const OpDev &o = ops[wi.inst];
    const int nx = o.nx, ny = o.ny, nz = o.nz, NZ = o.NZ, m = o.dmask;
    const T *__restrict__ Xi = X + o.off;
    T *__restrict__ Yi = Y + o.off;
    const T HTS_GLOBAL *__restrict__ Pi = gptr<T>(HEAT ? o.P : nullptr);
    const T HTS_GLOBAL *__restrict__ kk = gptr<T>(o.k);
    const T HTS_GLOBAL *__restrict__ lamc = gptr<T>(o.lam);
    const T HTS_GLOBAL *__restrict__ cTc = gptr<T>(o.cT);
    const double HTS_GLOBAL *__restrict__ xyz = gptr<double>(o.xyz);
    constexpr bool CHEB = EPI == EPI_CHEB || EPI == EPI_CHEB0;
    const T *__restrict__ Bi = (EPI == EPI_RESID || EPI == EPI_RESID_NORM || CHEB) ? ep.b + o.off : nullptr;
    T *__restrict__ Di = CHEB ? ep.d + o.off : nullptr;
    const T *__restrict__ Ii = CHEB ? ep.invd + o.off : nullptr;

    const uint32_t plane32 = (uint32_t)o.NX * (uint32_t)o.NY;
    const int tid = threadIdx.x, tx = tid % HB, ty = tid / HB;
    const int cx0 = wi.tx * HOWN - 1, cy0 = wi.ty * HOWN - 1;
    const int cx = cx0 + tx, cy = cy0 + ty;
    const bool cin = cx >= 0 && cx < nx && cy >= 0 && cy < ny;
    const uint32_t cbase = cin ? (uint32_t)cx + (uint32_t)nx * (uint32_t)cy : 0u;
    const uint32_t cplane = (uint32_t)nx * (uint32_t)ny;

    // staged node columns of this thread (two of the 17 x 17)
    int li[2], lj[2];
    bool ld[2], sval[2], scol[2];
    uint32_t sbase[2];
    int sdlo[2], sdhi[2];
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const int c = tid + s * 256;
        ld[s] = c < HCOL;
        li[s] = c % (HB + 1);
        lj[s] = c / (HB + 1);
        ColInfo lc;
        if (ld[s]) lc = col_info(o, cx0 + li[s], cy0 + lj[s]);
        else { lc.valid = 0; lc.base = 0; lc.xyc = 0; lc.dlo = 1; lc.dhi = 0; }
        sval[s] = lc.valid;
        scol[s] = lc.valid && !(MASKED && lc.xyc);
        sbase[s] = lc.valid ? (uint32_t)lc.base : 0u;
        sdlo[s] = lc.dlo;
        sdhi[s] = lc.dhi;
    }
    const bool owner = tx < HOWN && ty < HOWN;
    ColInfo oc = col_info(o, cx0 + tx + 1, cy0 + ty + 1);
    const bool own_ok = owner && oc.valid;
    const uint32_t obase = own_ok ? (uint32_t)oc.base : 0u;

    T c0 = T(0), c1 = T(0), c2 = T(0);
    if (CHEB) {
        const double *Sc = ep.S + (int64_t)wi.inst * NSLOT;
        c1 = T(Sc[ep.s1]);
        c2 = T(Sc[ep.s2]);
        if (EPI == EPI_CHEB0) c0 = T(Sc[ep.s0]);
    }
    const bool adv = HEAT && o.cadv != 0.0;

    auto stage = [&](int k, int b) {
        const int kc = k < 0 ? 0 : (k >= NZ ? NZ - 1 : k);
        const uint32_t koff = (uint32_t)kc * plane32;
        const bool kin = k >= 0 && k < NZ;
        const bool kkeep = kin && !(MASKED && (((m & 16) && k == 0) || ((m & 32) && k == NZ - 1)));
#pragma unroll
        for (int s = 0; s < 2; s++) {
            if (!ld[s]) continue;
            const uint32_t gi = sbase[s] + koff;
            bool keep = kkeep && scol[s];
            if (MASKED) keep = keep && !(k >= sdlo[s] && k <= sdhi[s]);
            const T xv = EPI == EPI_CHEB0 ? c0 * *at32(Ii, gi) * *at32(Bi, gi) : *at32(Xi, gi);
            xs[b][lj[s]][li[s]] = keep ? xv : T(0);
            if (HEAT) {
                const T pv = *at32(Pi, gi);
                ps[HEAT ? b : 0][HEAT ? lj[s] : 0][HEAT ? li[s] : 0] = (kin && sval[s]) ? pv : T(0);
            }
#pragma unroll
            for (int d = 0; d < 3; d++) cs[b][d][lj[s]][li[s]] = xyz[3 * (size_t)gi + d];
        }
    };

    const int kb = wi.z0, ke = wi.z1;
    double acc = 0.0;
    T top[4] = {T(0), T(0), T(0), T(0)};
    int sx = (kb - 1 + 3) % 3;
    stage(kb - 1, sx);
    for (int L = kb - 1; L <= ke; L++) {
        const bool comp = L <= ke - 1;
        const int sx1 = sx + 1 == 3 ? 0 : sx + 1;
        if (comp) stage(L + 1, sx1);
        T cm_ = T(0), cst = T(0), ck = T(0);
        const bool lay = comp && cin && L >= 0 && L < nz;
        if (lay) {
            const uint32_t ci = cbase + (uint32_t)L * cplane;
            if (HEAT) {
                cm_ = *at32(cTc, ci);
                cst = T(o.cs) * *at32(lamc, ci);
                ck = T(o.cadv) * *at32(kk, ci);
            } else {
                cm_ = T(o.cm);
                cst = T(o.cs) * *at32(kk, ci);
            }
        }
        __syncthreads();
        // epilogue of plane L-1 (corner sums written in the previous iteration)
        if (L - 1 >= kb && own_ok && L - 1 < NZ) {
            const int P0 = L - 1, sb = P0 & 1;
            T v = S4[sb][3][ty][tx] + S4[sb][2][ty][tx + 1] + S4[sb][1][ty + 1][tx] + S4[sb][0][ty + 1][tx + 1];
            const uint32_t gi = obase + (uint32_t)P0 * plane32;
            T eb = T(0), ex = T(0), ed = T(0), ei = T(0);
            if (Bi) eb = *at32(Bi, gi);
            if (EPI == EPI_CHEB) { ed = *at32(Di, gi); ei = *at32(Ii, gi); }
            if (EPI == EPI_CHEB0) { ei = *at32(Ii, gi); ex = c0 * ei * eb; ed = ex; }
            if (EPI == EPI_CHEB || EPI == EPI_DOT || (MASKED && EPI != EPI_CHEB0)) ex = *at32(Xi, gi);
            if (MASKED && constrained(oc, P0, NZ, m)) v = ex;
            if (EPI == EPI_STORE) {
                *at32(Yi, gi) = v;
            } else if (EPI == EPI_RESID) {
                *at32(Yi, gi) = eb - v;
            } else if (EPI == EPI_RESID_NORM) {
                const T r = eb - v;
                *at32(Yi, gi) = r;
                acc += (double)r * (double)r;
            } else if (EPI == EPI_DOT) {
                *at32(Yi, gi) = v;
                acc += (double)ex * (double)v;
            } else if (CHEB) {
                const T r = eb - v;
                const T d = c1 * ed + c2 * ei * r;
                *at32(Di, gi) = d;
                *at32(Yi, gi) = ex + d;
            }
        }
        if (!comp) break;
        T bot[4] = {T(0), T(0), T(0), T(0)}, tp[4] = {T(0), T(0), T(0), T(0)};
        if (lay) {
            T u[8], P[8], Xc[8][3], w[8];
            double o0[3];
#pragma unroll
            for (int d = 0; d < 3; d++) o0[d] = cs[sx][d][ty][tx];
#pragma unroll
            for (int a = 0; a < 8; a++) {
                const int b = (a >> 2) ? sx1 : sx, jj = ty + ((a >> 1) & 1), ii = tx + (a & 1);
                u[a] = xs[b][jj][ii];
                P[a] = HEAT ? ps[HEAT ? b : 0][HEAT ? jj : 0][HEAT ? ii : 0] : T(0);
#pragma unroll
                for (int d = 0; d < 3; d++) Xc[a][d] = T(cs[b][d][jj][ii] - o0[d]);
            }
            if (adv) hex_cell<T, true>(Xc, u, P, cm_, cst, ck, T(o.rho_g), w);
            else hex_cell<T, false>(Xc, u, P, cm_, cst, T(0), T(0), w);
#pragma unroll
            for (int a = 0; a < 4; a++) { bot[a] = w[a]; tp[a] = w[a + 4]; }
        }
        if (L >= kb) {
            const int sb = L & 1;
#pragma unroll
            for (int a = 0; a < 4; a++) S4[sb][a][ty][tx] = top[a] + bot[a];
        }
#pragma unroll
        for (int a = 0; a < 4; a++) top[a] = tp[a];
        sx = sx1;
    }
    if (EPI == EPI_RESID_NORM || EPI == EPI_DOT) {
        double v = wave_sum(acc);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) ep.partial[wi.slot] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// ----------------------------------------------------------- setup kernels
// The element matrix row of local node al of cell (cx, cy, cz) in FP64:
// out[b] = int m N_al N_b + s grad N_al . grad N_b  (no convection).
__device__ void hex_row(const OpDev &o, int cx, int cy, int cz, int al, double mc, double sc, double out[8])
{
    const double *xyz = static_cast<const double *>(o.xyz);
    double X[8][3], o0[3];
    for (int a = 0; a < 8; a++) {
        const int64_t n = (int64_t)(cx + (a & 1)) + (int64_t)o.NX * ((cy + ((a >> 1) & 1)) +
                                                                     (int64_t)o.NY * (cz + (a >> 2)));
        for (int d = 0; d < 3; d++) X[a][d] = xyz[3 * n + d];
    }
    for (int d = 0; d < 3; d++) o0[d] = X[0][d];
    for (int a = 0; a < 8; a++)
        for (int d = 0; d < 3; d++) X[a][d] -= o0[d];
    for (int b = 0; b < 8; b++) out[b] = 0.0;
    for (int q = 0; q < 8; q++) {
        const double g3[3] = {(q & 1) ? HG1 : HG0, (q & 2) ? HG1 : HG0, (q & 4) ? HG1 : HG0};
        double N[8], R[8][3];
        for (int a = 0; a < 8; a++) {
            double v[3], dv[3];
            for (int d = 0; d < 3; d++) {
                const int ad = (a >> d) & 1;
                v[d] = ad ? g3[d] : 1.0 - g3[d];
                dv[d] = ad ? 1.0 : -1.0;
            }
            N[a] = v[0] * v[1] * v[2];
            R[a][0] = dv[0] * v[1] * v[2];
            R[a][1] = v[0] * dv[1] * v[2];
            R[a][2] = v[0] * v[1] * dv[2];
        }
        double J[3][3] = {{0.0}};
        for (int a = 0; a < 8; a++)
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) J[i][j] += X[a][i] * R[a][j];
        double C[3][3];
        C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
        double Ga[3];
        for (int i = 0; i < 3; i++) Ga[i] = C[i][0] * R[al][0] + C[i][1] * R[al][1] + C[i][2] * R[al][2];
        for (int b = 0; b < 8; b++) {
            double gg = 0.0;
            for (int i = 0; i < 3; i++) gg += Ga[i] * (C[i][0] * R[b][0] + C[i][1] * R[b][1] + C[i][2] * R[b][2]);
            out[b] += 0.125 * (mc * N[al] * N[b] * det + sc * gg / det);
        }
    }
}

// coefficients of cell c: pressure cm, cs k; heat c_T, cs lambda (FP64 arrays)
__device__ __forceinline__ void hex_coefs(const OpDev &o, int64_t c, double &mc, double &sc)
{
    if (o.field == 0) {
        mc = o.cm;
        sc = o.cs * static_cast<const double *>(o.k)[c];
    } else {
        mc = static_cast<const double *>(o.cT)[c];
        sc = o.cs * static_cast<const double *>(o.lam)[c];
    }
}

__global__ void k_hex_inv_diag(OpDev o, double *__restrict__ out)
{
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= o.nnode) return;
    const int NX = o.NX, NY = o.NY;
    const int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((int64_t)NX * NY));
    ColInfo c = col_info(o, i, j);
    if (constrained(c, k, o.NZ, o.dmask)) { out[n] = 1.0; return; }
    double d = 0.0;
    for (int dz = -1; dz <= 0; dz++)
        for (int dy = -1; dy <= 0; dy++)
            for (int dx = -1; dx <= 0; dx++) {
                const int cx = i + dx, cy = j + dy, cz = k + dz;
                if (cx < 0 || cx >= o.nx || cy < 0 || cy >= o.ny || cz < 0 || cz >= o.nz) continue;
                const int64_t ci = cx + (int64_t)o.nx * (cy + (int64_t)o.ny * cz);
                double mc, sc, row[8];
                hex_coefs(o, ci, mc, sc);
                const int al = (-dx) + 2 * (-dy) + 4 * (-dz);
                hex_row(o, cx, cy, cz, al, mc, sc, row);
                d += row[al];
            }
    out[n] = 1.0 / d;
}

// 27-point stencil of the symmetric part (the multigrid's fine level):
// S[e * nnode + n], e = (di + 1) + 3 (dj + 1) + 9 (dk + 1); constrained rows
// and columns eliminated (identity rows)
__global__ void k_hex_stencil(OpDev o, double *__restrict__ S)
{
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= o.nnode) return;
    const int NX = o.NX, NY = o.NY, NZ = o.NZ;
    const int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((int64_t)NX * NY));
    double st[27];
    for (int e = 0; e < 27; e++) st[e] = 0.0;
    ColInfo c = col_info(o, i, j);
    if (constrained(c, k, NZ, o.dmask)) {
        st[13] = 1.0;
    } else {
        for (int dz = -1; dz <= 0; dz++)
            for (int dy = -1; dy <= 0; dy++)
                for (int dx = -1; dx <= 0; dx++) {
                    const int cx = i + dx, cy = j + dy, cz = k + dz;
                    if (cx < 0 || cx >= o.nx || cy < 0 || cy >= o.ny || cz < 0 || cz >= o.nz) continue;
                    const int64_t ci = cx + (int64_t)o.nx * (cy + (int64_t)o.ny * cz);
                    double mc, sc, row[8];
                    hex_coefs(o, ci, mc, sc);
                    hex_row(o, cx, cy, cz, (-dx) + 2 * (-dy) + 4 * (-dz), mc, sc, row);
                    for (int b = 0; b < 8; b++) {
                        const int gi = cx + (b & 1), gj = cy + ((b >> 1) & 1), gk = cz + (b >> 2);
                        ColInfo cb = col_info(o, gi, gj);
                        if (constrained(cb, gk, NZ, o.dmask)) continue;
                        st[(gi - i + 1) + 3 * (gj - j + 1) + 9 * (gk - k + 1)] += row[b];
                    }
                }
    }
    for (int e = 0; e < 27; e++) S[(int64_t)e * o.nnode + n] = st[e];
}

// y_a = sum_c alpha_c int N_a dV + beta_c int dN_a/dz dV
__global__ void k_hex_cell_loads(OpDev o, const double *__restrict__ alpha, const double *__restrict__ beta,
                                 double *__restrict__ y)
{
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= o.nnode) return;
    const int NX = o.NX, NY = o.NY;
    const int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((int64_t)NX * NY));
    const double *xyz = static_cast<const double *>(o.xyz);
    double s = 0.0;
    for (int dz = -1; dz <= 0; dz++)
        for (int dy = -1; dy <= 0; dy++)
            for (int dx = -1; dx <= 0; dx++) {
                const int cx = i + dx, cy = j + dy, cz = k + dz;
                if (cx < 0 || cx >= o.nx || cy < 0 || cy >= o.ny || cz < 0 || cz >= o.nz) continue;
                const int64_t ci = cx + (int64_t)o.nx * (cy + (int64_t)o.ny * cz);
                const double al = alpha ? alpha[ci] : 0.0, be = beta ? beta[ci] : 0.0;
                if (al == 0.0 && be == 0.0) continue;
                const int a = (-dx) + 2 * (-dy) + 4 * (-dz);
                double X[8][3];
                for (int b = 0; b < 8; b++) {
                    const int64_t nb = (int64_t)(cx + (b & 1)) +
                                       (int64_t)NX * ((cy + ((b >> 1) & 1)) + (int64_t)NY * (cz + (b >> 2)));
                    for (int d = 0; d < 3; d++) X[b][d] = xyz[3 * nb + d] - xyz[3 * (nb - (b & 1) - NX * ((b >> 1) & 1) - (int64_t)NX * NY * (b >> 2)) + d];
                }
                for (int q = 0; q < 8; q++) {
                    const double g3[3] = {(q & 1) ? HG1 : HG0, (q & 2) ? HG1 : HG0, (q & 4) ? HG1 : HG0};
                    double R[8][3], Na = 1.0;
                    for (int b = 0; b < 8; b++) {
                        double v[3], dv[3];
                        for (int d = 0; d < 3; d++) {
                            const int bd = (b >> d) & 1;
                            v[d] = bd ? g3[d] : 1.0 - g3[d];
                            dv[d] = bd ? 1.0 : -1.0;
                        }
                        if (b == a) Na = v[0] * v[1] * v[2];
                        R[b][0] = dv[0] * v[1] * v[2];
                        R[b][1] = v[0] * dv[1] * v[2];
                        R[b][2] = v[0] * v[1] * dv[2];
                    }
                    double J[3][3] = {{0.0}};
                    for (int b = 0; b < 8; b++)
                        for (int ii = 0; ii < 3; ii++)
                            for (int jj = 0; jj < 3; jj++) J[ii][jj] += X[b][ii] * R[b][jj];
                    // det and the z row of the cofactors (det * d N / dz = C_2j R_j)
                    const double C20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
                    const double C21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
                    const double C22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
                    const double det = J[2][0] * C20 + J[2][1] * C21 + J[2][2] * C22;
                    s += 0.125 * (al * Na * det + be * (C20 * R[a][0] + C21 * R[a][1] + C22 * R[a][2]));
                }
            }
    y[n] = s;
}

}  // namespace

// ---------------------------------------------------------------- launchers
template <typename T, int FIELD, bool MASKED>
static void dispatch_hex(int epi, const OpDev *ops, const WorkItem *work, int nwork, const T *x, T *y,
                         const EpiArgs<T> &ep, hipStream_t s)
{
    const dim3 g(nwork), b(256);
    switch (epi) {
    case EPI_STORE: k_hex_apply<T, FIELD, EPI_STORE, MASKED><<<g, b, 0, s>>>(ops, work, x, y, ep); break;
    case EPI_RESID: k_hex_apply<T, FIELD, EPI_RESID, MASKED><<<g, b, 0, s>>>(ops, work, x, y, ep); break;
    case EPI_RESID_NORM: k_hex_apply<T, FIELD, EPI_RESID_NORM, MASKED><<<g, b, 0, s>>>(ops, work, x, y, ep); break;
    case EPI_DOT: k_hex_apply<T, FIELD, EPI_DOT, MASKED><<<g, b, 0, s>>>(ops, work, x, y, ep); break;
    case EPI_CHEB: k_hex_apply<T, FIELD, EPI_CHEB, MASKED><<<g, b, 0, s>>>(ops, work, x, y, ep); break;
    case EPI_CHEB0:
        if (!MASKED) throw Error(-1, "EPI_CHEB0 is for masked operators");
        k_hex_apply<T, FIELD, EPI_CHEB0, true><<<g, b, 0, s>>>(ops, work, x, y, ep);
        break;
    default: throw Error(-1, "bad epilogue");
    }
}

template <typename T>
void launch_hex(int field, int epi, bool masked, const OpDev *ops, const WorkItem *work, int nwork, const T *x,
                T *y, const EpiArgs<T> &ep, hipStream_t s)
{
    if (nwork <= 0) return;
    if (field == 0) {
        if (masked) dispatch_hex<T, 0, true>(epi, ops, work, nwork, x, y, ep, s);
        else dispatch_hex<T, 0, false>(epi, ops, work, nwork, x, y, ep, s);
    } else {
        if (masked) dispatch_hex<T, 1, true>(epi, ops, work, nwork, x, y, ep, s);
        else dispatch_hex<T, 1, false>(epi, ops, work, nwork, x, y, ep, s);
    }
    HTS_LAUNCH_CHECK();
}
template void launch_hex<double>(int, int, bool, const OpDev *, const WorkItem *, int, const double *, double *,
                                 const EpiArgs<double> &, hipStream_t);
template void launch_hex<float>(int, int, bool, const OpDev *, const WorkItem *, int, const float *, float *,
                                const EpiArgs<float> &, hipStream_t);

void launch_hex_inv_diag(const OpDev &op, double *inv_diag, hipStream_t s)
{
    k_hex_inv_diag<<<dim3((unsigned)((op.nnode + 127) / 128)), dim3(128), 0, s>>>(op, inv_diag);
    HTS_LAUNCH_CHECK();
}

void launch_hex_stencil(const OpDev &op, double *S, hipStream_t s)
{
    k_hex_stencil<<<dim3((unsigned)((op.nnode + 127) / 128)), dim3(128), 0, s>>>(op, S);
    HTS_LAUNCH_CHECK();
}

void launch_hex_cell_loads(const OpDev &op, const double *alpha, const double *beta, double *y, hipStream_t s)
{
    k_hex_cell_loads<<<dim3((unsigned)((op.nnode + 127) / 128)), dim3(128), 0, s>>>(op, alpha, beta, y);
    HTS_LAUNCH_CHECK();
}

}  // namespace hts
