// Matrix-free Q1 operators of the pressure (Eq. 3) and heat (Eq. 4)
// equations on a uniform box, sum-factorised per cell.
//
// Kernel layout: a 256-thread workgroup (16 x 16 threads) owns a 31 x 15
// tile of node columns and marches upward through a range of node planes.
// Each thread handles two neighbouring cell columns along x of the 32 x 16
// cells that touch the tile (one-cell halo on the low x/y side).  Per cell
// layer the new node plane is staged in LDS; each thread keeps its own 3 x 2
// node values of the previous plane in registers, evaluates both cells by
// Kronecker sum factorisation (1D mass h/6 [2 1; 1 2] and stiffness
// 1/h [1 -1; -1 1] in each direction; the y-z factors of the face the two
// cells share are formed once; 2-point Gauss for the convection term), sums
// the contributions to its 3 x 2 plane corners and passes the four that
// other threads own through LDS.  A thread owns the node between its two
// cells and the node to the right of its second cell; the owner of a node
// adds the contributions in a fixed order.  Every node value is produced by
// exactly one thread: no atomics, bitwise reproducible.
#include <type_traits>

#include "common.h"
#include "dev_util.h"

namespace hts {

namespace {

constexpr int TCX = 32;                       // cell columns per tile along x
constexpr int TCY = 16;                       // cell columns per tile along y
constexpr int OWNX = TCX - 1, OWNY = TCY - 1; // owned node columns per tile
constexpr int SXN = TCX + 1, SYN = TCY + 1;   // staged node columns per plane
constexpr int SXP = SXN + 1;                  // LDS row pitch (even: 16-byte pair reads)
constexpr int NSTAGE = SXN * SYN;             // 561 staged values per plane

// The 1D factors are applied unscaled, [2 1; 1 2] for the mass matrix
// (h/6 times it) and [1 -1; -1 1] for the stiffness matrix (1/h times it);
// the 1/6 factors and the cell sizes go into the per-cell coefficients.
template <typename T>
__device__ __forceinline__ void m1p(T &a, T &b)
{
    const T na = T(2) * a + b;
    const T nb = T(2) * b + a;
    a = na;
    b = nb;
}

template <typename T>
__device__ __forceinline__ void k1p(T &a, T &b)
{
    T d = a - b;
    a = d;
    b = -d;
}


#define PZ(F, v) F(v[0], v[4]); F(v[1], v[5]); F(v[2], v[6]); F(v[3], v[7]);
#define PY(F, v) F(v[0], v[2]); F(v[1], v[3]); F(v[4], v[6]); F(v[5], v[7]);
#define PX(F, v) F(v[0], v[1]); F(v[2], v[3]); F(v[4], v[5]); F(v[6], v[7]);

// w = m (M x M x M) u + (sx K x M x M + sy M x K x M + sz M x M x K) u with
// the unscaled 1D factors; for mass coefficient c and stiffness coefficient
// s of a cell: m = c V / 216, sx = s (hy hz / hx) / 36, and so on.
template <typename T>
__device__ __forceinline__ void cell_mass_stiff(const T u[8], T m, T sx, T sy, T sz, T w[8])
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
    // f = (m c + 6 sy d + 6 sz e) / 6 is what the x mass factor takes
    T f[8], g[8];
#pragma unroll
    for (int i = 0; i < 8; i++) {
        f[i] = m * c[i] + sy * d[i] + sz * e[i];
        g[i] = c[i];
    }
    PX(m1p, f);
    PX(k1p, g);
#pragma unroll
    for (int i = 0; i < 8; i++) w[i] = f[i] + sx * g[i];
}

// y-z factors of one x-face of a cell from its node values v{y}{z}, with the
// unscaled 1D factors: c = (Mz My) v (index y + 2 z), the part with the y
// stiffness (Mz Ky) v in its two magnitudes d[z] (sign + at y = 0, - at
// y = 1) and the part with the z stiffness (Kz My) v in its two magnitudes
// e[y] (sign + at z = 0, - at z = 1).  Two cells that share the face share
// these.
template <typename T>
struct FaceYZ {
    T c[4];
    T d[2];
    T e[2];
};

template <typename T>
__device__ __forceinline__ FaceYZ<T> face_yz(T v00, T v10, T v01, T v11)
{
    FaceYZ<T> f;
    const T a00 = T(2) * v00 + v01, a01 = v00 + T(2) * v01;   // mass along z, y = 0
    const T a10 = T(2) * v10 + v11, a11 = v10 + T(2) * v11;   // y = 1
    const T b0 = v00 - v01, b1 = v10 - v11;                   // stiffness along z, z = 0 row
    f.c[0] = T(2) * a00 + a10;
    f.c[1] = a00 + T(2) * a10;
    f.c[2] = T(2) * a01 + a11;
    f.c[3] = a01 + T(2) * a11;
    f.d[0] = a00 - a10;
    f.d[1] = a01 - a11;
    f.e[0] = T(2) * b0 + b1;
    f.e[1] = b0 + T(2) * b1;
    return f;
}

// w = m (M x M x M) u + (sx K x M x M + sy M x K x M + sz M x M x K) u of the
// cell whose x = 0 and x = 1 faces are F0 and F1 (corner index x + 2y + 4z);
// for mass coefficient c and stiffness coefficient s of a cell: m = c V / 216,
// sx = s (hy hz / hx) / 36, and so on.
template <typename T>
__device__ __forceinline__ void cell_from_faces(const FaceYZ<T> &F0, const FaceYZ<T> &F1, T m, T sx, T sy, T sz,
                                                T w[8])
{
#pragma unroll
    for (int z = 0; z < 2; z++)
#pragma unroll
        for (int y = 0; y < 2; y++) {
            const int q = y + 2 * z;
            const T sd = y == 0 ? sy : -sy, se = z == 0 ? sz : -sz;
            const T f0 = m * F0.c[q] + (sd * F0.d[z] + se * F0.e[y]);
            const T f1 = m * F1.c[q] + (sd * F1.d[z] + se * F1.e[y]);
            const T g = sx * (F0.c[q] - F1.c[q]);
            w[2 * y + 4 * z] = (T(2) * f0 + f1) + g;
            w[1 + 2 * y + 4 * z] = (f0 + T(2) * f1) - g;
        }
}

template <typename T, int EPI, bool MASKED, bool GRADED>
__global__ __launch_bounds__(256) void k_q1_pressure(const OpDev *__restrict__ ops,
                                                     const WorkItem *__restrict__ work,
                                                     const T *__restrict__ X, T *__restrict__ Y,
                                                     EpiArgs<T> ep)
{
    // Software pipeline over node planes, one barrier per plane: x planes in
    // an LDS ring of 2 (plane p in slot p & 1; each thread keeps its own
    // values of the lower plane in registers), the four exchanged
    // plane-corner sums of each thread in a ring of 2; the global loads of
    // plane L+2, of the coefficients of layer L+1 and of the epilogue
    // operands of plane L are issued one iteration before they are used.
    __shared__ __align__(16) T xs[2][SYN][SXP];
    __shared__ T ex[2][4][TCY][17];
    __shared__ double red[4];

    const WorkItem wi = work[blockIdx.x];
    if (ep.active && !ep.active[wi.inst]) return;
    const OpDev &o = ops[wi.inst];
    const int nx = o.nx, ny = o.ny, nz = o.nz, NZ = o.NZ, m = o.dmask;
    const T *__restrict__ Xi = X + o.off;
    T *__restrict__ Yi = Y + o.off;
    const T HTS_GLOBAL *__restrict__ kk = gptr<T>(o.k);
    constexpr bool CHEB = EPI == EPI_CHEB || EPI == EPI_CHEB0;
    const T *__restrict__ Bi = (EPI == EPI_RESID || EPI == EPI_RESID_NORM || CHEB) ? ep.b + o.off : nullptr;
    T *__restrict__ Di = CHEB ? ep.d + o.off : nullptr;
    const T *__restrict__ Ii = CHEB ? ep.invd + o.off : nullptr;

    // Node and cell indices are instance-local, non-negative and below 2^31:
    // unsigned 32-bit offsets (the loads take a uniform base and a 32-bit
    // offset; the vectors are offset to the instance already).
    const uint32_t plane32 = (uint32_t)(o.NX * o.NY);
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int lx = 2 * tx;                        // local x of the thread's first cell
    const int cx0 = wi.tx * OWNX - 1, cy0 = wi.ty * OWNY - 1;
    const int cxa = cx0 + lx, cy = cy0 + ty;      // global indices of cell 0 (cell 1 is cxa + 1)
    const bool cyin = cy >= 0 && cy < ny;
    const bool cin0 = cyin && cxa >= 0 && cxa < nx;
    const bool cin1 = cyin && cxa + 1 >= 0 && cxa + 1 < nx;
    const uint32_t cbase0 = cin0 ? (uint32_t)(cxa + nx * cy) : 0u, cbase1 = cin1 ? (uint32_t)(cxa + 1 + nx * cy) : 0u;
    const uint32_t cplane = (uint32_t)(nx * ny);

    // staged node columns of this thread (three slots, the third only for
    // the first NSTAGE - 512 threads): base index (0 outside the mesh, so the
    // loads stay in range; the value is then discarded), kept (in the mesh,
    // not on a constraining x/y face), constrained z-range
    int lj[3], li[3];
    bool scol[3];
    uint32_t sbase[3];
    int sdlo[3], sdhi[3];
    const bool ld2 = tid < NSTAGE - 512;
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const int c = tid + q * 256;
        li[q] = c % SXN;
        lj[q] = c / SXN;
        ColInfo lc;
        if (q < 2 || ld2) lc = col_info(o, cx0 + li[q], cy0 + lj[q]);
        else { lc.valid = 0; lc.base = 0; lc.xyc = 0; lc.dlo = 1; lc.dhi = 0; li[q] = 0; lj[q] = 0; }
        scol[q] = lc.valid && !(MASKED && lc.xyc);
        sbase[q] = lc.valid ? (uint32_t)lc.base : 0u;
        sdlo[q] = lc.dlo;
        sdhi[q] = lc.dhi;
    }
    // owned nodes: A between the thread's two cells, B right of its second
    // cell (not for the last thread of a row), both on the upper cell row
    const bool ownrow = ty < OWNY;
    const ColInfo ocA = col_info(o, cx0 + lx + 1, cy0 + ty + 1);
    const ColInfo ocB = col_info(o, cx0 + lx + 2, cy0 + ty + 1);
    const bool okA = ownrow && ocA.valid, okB = ownrow && tx < 15 && ocB.valid;

    // per-cell coefficient factors of the unscaled 1D products (formed in
    // double on the host, rounded once here)
    const T fm = T(o.q1m), fx = T(o.q1x), fy = T(o.q1y), fz = T(o.q1z);
    const T cm = T(o.cm);
    // graded meshes: every factor is a per-column part (from the cell's hx,
    // hy, formed once in double and rounded) times hz or 1 / hz of the layer
    const bool graded = GRADED && o.hzs != nullptr;
    T gm[2] = {T(0), T(0)}, gx[2] = {T(0), T(0)}, gy[2] = {T(0), T(0)}, gz[2] = {T(0), T(0)};
    if (graded) {
        const int iy = cy < 0 ? 0 : (cy >= ny ? ny - 1 : cy);
        const double ghy = o.hys[iy];
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const int c = cxa + q, ix = c < 0 ? 0 : (c >= nx ? nx - 1 : c);
            const double ghx = o.hxs[ix], hxy = ghx * ghy;
            gm[q] = T(hxy / 216.0);                           // x hz
            gx[q] = T(o.cs * (ghy / ghx) / 36.0);             // x hz
            gy[q] = T(o.cs * (ghx / ghy) / 36.0);             // x hz
            gz[q] = T(o.cs * hxy / 36.0);                     // x 1/hz
        }
    }
    T c0 = T(0), c1 = T(0), c2 = T(0);
    if (CHEB) {
        const double *Sc = ep.S + (int64_t)wi.inst * NSLOT;
        c1 = T(Sc[ep.s1]);
        c2 = T(Sc[ep.s2]);
        if (EPI == EPI_CHEB0) c0 = T(Sc[ep.s0]);
    }

    // Plane / coefficient / epilogue loads are unconditional (clamped to a
    // valid address) and the keep-or-zero decision is applied when the value
    // is consumed, so that no branch or select forces an early wait on a
    // load.  Keep decisions are all-ones / zero bit masks in vector
    // registers (bool arrays would take a 64-bit scalar mask each).
    using UT = typename std::conditional<sizeof(T) == 8, uint64_t, uint32_t>::type;
    T pfx[3];
    UT pkeep[3];
    auto fetch_plane = [&](int k) {
        const int kc = k < 0 ? 0 : (k >= NZ ? NZ - 1 : k);
        const uint32_t koff = (uint32_t)kc * plane32;
        // the part of the keep decision that is the same for every column
        const bool kin = k >= 0 && k < NZ;
        const bool kkeep = kin && !(MASKED && (((m & 16) && k == 0) || ((m & 32) && k == NZ - 1)));
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const uint32_t gi = sbase[q] + koff;
            // EPI_CHEB0 operand: x0 = c0 D^-1 b, in the order of the
            // separate first Chebyshev kernel
            if (EPI == EPI_CHEB0) pfx[q] = c0 * *at32(Ii, gi) * *at32(Bi, gi);
            else pfx[q] = *at32(Xi, gi);
            bool keep = kkeep && scol[q];
            if (MASKED) keep = keep && !(k >= sdlo[q] && k <= sdhi[q]);
            pkeep[q] = keep ? ~UT(0) : UT(0);
        }
    };
    auto store_plane = [&](int bx) {
#pragma unroll
        for (int q = 0; q < 3; q++) {
            if (q == 2 && !ld2) continue;
            xs[bx][lj[q]][li[q]] = __builtin_bit_cast(T, __builtin_bit_cast(UT, pfx[q]) & pkeep[q]);
        }
    };
    // the thread's 3 x 2 node values of a staged plane: [y * 3 + c]
    auto read_plane = [&](int bx, T *u) {
#pragma unroll
        for (int y = 0; y < 2; y++)
#pragma unroll
            for (int c = 0; c < 3; c++) u[3 * y + c] = xs[bx][ty + y][lx + c];
    };
    T cfk[2] = {T(0), T(0)};
    double cfh = 0.0, cfih = 0.0;     // graded: hz and 1/hz of the layer
    auto fetch_coef = [&](int L) {
        const int Lc = L < 0 ? 0 : (L >= nz ? nz - 1 : L);
        const uint32_t lo = (uint32_t)Lc * cplane;
        cfk[0] = *at32(kk, cbase0 + lo);
        cfk[1] = *at32(kk, cbase1 + lo);
        if (graded) { cfh = o.hzs[Lc]; cfih = o.ihzs[Lc]; }
    };
    // epilogue operands of the two owned nodes
    const uint32_t obA = okA ? (uint32_t)ocA.base : 0u, obB = okB ? (uint32_t)ocB.base : 0u;
    T eb[2] = {T(0), T(0)}, ed[2] = {T(0), T(0)}, ei[2] = {T(0), T(0)}, exv[2] = {T(0), T(0)};
    auto fetch_epi = [&](int L) {
        const int Lc = L < NZ ? L : NZ - 1;
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const uint32_t gi = (q ? obB : obA) + (uint32_t)Lc * plane32;
            if (Bi) eb[q] = *at32(Bi, gi);
            if (EPI == EPI_CHEB) { ed[q] = *at32(Di, gi); ei[q] = *at32(Ii, gi); }
            if (EPI == EPI_CHEB0) ei[q] = *at32(Ii, gi);
            if (EPI == EPI_CHEB || EPI == EPI_DOT || (MASKED && EPI != EPI_CHEB0)) exv[q] = *at32(Xi, gi);
        }
    };

    const int kb = wi.z0, ke = wi.z1;
    double acc = 0.0;
    // carried between layers: the thread's values of the lower plane, the
    // top-corner sums of the previous layer per (y, c), and the own sums of
    // the last plane at the owned nodes A and B (for its epilogue)
    T cu[6];
    T tv[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    T hA = T(0), hB = T(0);

    // epilogue of one owned node: constraint, the selected result
    auto epilogue = [&](int q, T v, const ColInfo &oc, uint32_t ob, int P0) {
        const uint32_t gi = ob + (uint32_t)P0 * plane32;
        T xq = exv[q], dq = ed[q];
        if (EPI == EPI_CHEB0) {
            xq = c0 * ei[q] * eb[q];
            dq = xq;
        }
        if (MASKED && constrained(oc, P0, NZ, m)) v = xq;
        if (EPI == EPI_STORE) {
            *at32(Yi, gi) = v;
        } else if (EPI == EPI_RESID) {
            *at32(Yi, gi) = eb[q] - v;
        } else if (EPI == EPI_RESID_NORM) {
            const T r = eb[q] - v;
            *at32(Yi, gi) = r;
            acc += (double)r * (double)r;
        } else if (EPI == EPI_DOT) {
            *at32(Yi, gi) = v;
            acc += (double)xq * (double)v;
        } else if (CHEB) {
            const T r = eb[q] - v;
            const T d = c1 * dq + c2 * ei[q] * r;
            *at32(Di, gi) = d;
            *at32(Yi, gi) = xq + d;
        }
    };

    int sx = (kb - 1) & 1;
    fetch_plane(kb - 1);
    store_plane(sx);
    fetch_plane(kb);
    fetch_coef(kb - 1);
    __syncthreads();
    read_plane(sx, cu);

    for (int L = kb - 1; L <= ke; L++) {
        const bool comp = L <= ke - 1;
        const int sx1 = sx ^ 1;
        if (comp) store_plane(sx1);
        // a cell outside the mesh contributes nothing: its coefficients are
        // zero (its node values are finite); the selects sit where the loaded
        // values are consumed
        const bool lin = L >= 0 && L < nz, on0 = lin && cin0, on1 = lin && cin1;
        const T ck0 = on0 ? cfk[0] : T(0), ck1 = on1 ? cfk[1] : T(0);
        const T cm0 = on0 ? cm : T(0), cm1 = on1 ? cm : T(0);
        const double lhz = cfh, lihz = cfih;
        if (L + 1 <= ke - 1) {
            fetch_plane(L + 2);
            fetch_coef(L + 1);
        }
        __syncthreads();
        // epilogue of plane L-1 (corner sums written in the previous iteration)
        if (L - 1 >= kb && L - 1 < NZ) {
            const int P0 = L - 1, sb = P0 & 1;
            if (okA) epilogue(0, hA + ex[sb][1][ty + 1][tx], ocA, obA, P0);
            if (okB) {
                const T v = (hB + ex[sb][3][ty][tx + 1]) + (ex[sb][2][ty + 1][tx] + ex[sb][0][ty + 1][tx + 1]);
                epilogue(1, v, ocB, obB, P0);
            }
        }
        if (!comp) break;
        if (L >= kb) fetch_epi(L);
        // the new upper plane L+1
        T nu[6];
        read_plane(sx1, nu);
        // cell layer L between planes L and L+1: cell 0, then cell 1 (the
        // shared face is formed once); each cell's corner values are folded
        // into the plane sums at once, which keeps few values live.  sv[]:
        // plane L sums per (y, c), tt[]: top corners of layer L per (y, c).
        T sv[6], tt[6];
        {
            FaceYZ<T> Fa = face_yz(cu[0], cu[3], nu[0], nu[3]);
            FaceYZ<T> Fb = face_yz(cu[1], cu[4], nu[1], nu[4]);
#pragma unroll
            for (int q = 0; q < 2; q++) {
                if (q == 1) {
                    Fa = Fb;
                    Fb = face_yz(cu[2], cu[5], nu[2], nu[5]);
                }
                T lfm = fm, lfx = fx, lfy = fy, lfz = fz;
                if (graded) {
                    const T hz = T(lhz), ihz = T(lihz);
                    lfm = gm[q] * hz;
                    lfx = gx[q] * hz;
                    lfy = gy[q] * hz;
                    lfz = gz[q] * ihz;
                }
                const T ck = q ? ck1 : ck0;
                T w[8];
                cell_from_faces(Fa, Fb, (q ? cm1 : cm0) * lfm, ck * lfx, ck * lfy, ck * lfz, w);
                if (q == 0) {
                    sv[0] = tv[0] + w[0];
                    sv[1] = w[1];
                    sv[3] = tv[3] + w[2];
                    sv[4] = w[3];
                    tt[0] = w[4];
                    tt[1] = w[5];
                    tt[3] = w[6];
                    tt[4] = w[7];
                } else {
                    sv[1] = tv[1] + (sv[1] + w[0]);
                    sv[2] = tv[2] + w[1];
                    sv[4] = tv[4] + (sv[4] + w[2]);
                    sv[5] = tv[5] + w[3];
                    tt[1] = tt[1] + w[4];
                    tt[2] = w[5];
                    tt[4] = tt[4] + w[6];
                    tt[5] = w[7];
                }
            }
        }
        // plane L: pass the sums other threads own, keep the own ones
        if (L >= kb) {
            const int sb = L & 1;
            ex[sb][0][ty][tx] = sv[0];
            ex[sb][1][ty][tx] = sv[1];
            ex[sb][2][ty][tx] = sv[2];
            ex[sb][3][ty][tx] = sv[3];
            hA = sv[4];
            hB = sv[5];
        }
#pragma unroll
        for (int a = 0; a < 6; a++) {
            tv[a] = tt[a];
            cu[a] = nu[a];
        }
        sx = sx1;
    }
    if (EPI == EPI_RESID_NORM || EPI == EPI_DOT) {
        double v = wave_sum(acc);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) ep.partial[wi.slot] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// Narrow tiles (heat operator): a 256-thread workgroup owns a 15 x 15 tile
// of node columns; each thread handles one cell column of the 16 x 16 cells
// that touch it (one-cell halo on the low x/y side), evaluates its cell's 8
// outputs and writes its four plane-corner contributions to LDS; the owner
// of a node adds the four cell contributions in a fixed order.  Fewer
// registers per thread than the wide tiles, which the convection term needs.
constexpr int NB = 16;          // cell columns per tile edge
constexpr int NOWN = NB - 1;    // owned node columns per tile edge
constexpr int NNCOL = (NB + 1) * (NB + 1);

// Heat cell operator in Haar coordinates.  Along one axis the pair of node
// values (v0, v1) becomes (s, d) = (v0 + v1, v0 - v1); there the unscaled 1D
// mass [2 1; 1 2] and stiffness [1 -1; -1 1] are diagonal, (3, 1) and (0, 2),
// and so is the interpolation to the two Gauss points, (1, 1/sqrt 3).  Mass
// and conduction become one diagonal scaling of the 8 Haar coefficients, and
// the convection term of an axis, a Gauss-point product of two bilinear
// fields on the cell's cross-section, becomes the product rule
//   out_s = (S s + D d / 3) / 2,  out_d = (S d + D s) / 6
// per cross-section axis (S, D: the flux field, s, d: the temperature
// differences), whose result is constant along the axis.  The same quadrature
// sums as the nodal form, about two thirds of its operations.
template <typename T>
__device__ __forceinline__ void haar_pair(T &a, T &b)
{
    const T s = a + b, d = a - b;
    a = s;
    b = d;
}

// 3D transform in place, index x + 2y + 4z (its own inverse up to 1/8)
template <typename T>
__device__ __forceinline__ void haar3(T v[8])
{
    haar_pair(v[0], v[1]); haar_pair(v[2], v[3]); haar_pair(v[4], v[5]); haar_pair(v[6], v[7]);
    haar_pair(v[0], v[2]); haar_pair(v[1], v[3]); haar_pair(v[4], v[6]); haar_pair(v[5], v[7]);
    haar_pair(v[0], v[4]); haar_pair(v[1], v[5]); haar_pair(v[2], v[6]); haar_pair(v[3], v[7]);
}

// 2D transform in place, index i + 2j: 0 ss, 1 ds, 2 sd, 3 dd
template <typename T>
__device__ __forceinline__ void haar2(T v[4])
{
    haar_pair(v[0], v[1]); haar_pair(v[2], v[3]); haar_pair(v[0], v[2]); haar_pair(v[1], v[3]);
}

// o += the back-projected Gauss-point product of A and v (2D Haar
// coordinates); A carries the weights 1/4, 1/12, 1/12, 1/36 of its terms
template <typename T>
__device__ __forceinline__ void haar_prod2(const T A[4], const T v[4], T &o0, T &o1, T &o2, T &o3)
{
    const T third = T(1) / T(3);
    const T A03 = A[0] * third, A13 = A[1] * third, A23 = A[2] * third, A09 = A03 * third;
    o0 += A[0] * v[0] + A[1] * v[1] + A[2] * v[2] + A[3] * v[3];
    o1 += A03 * v[1] + A[1] * v[0] + A23 * v[3] + A[3] * v[2];
    o2 += A03 * v[2] + A[2] * v[0] + A13 * v[3] + A[3] * v[1];
    o3 += A09 * v[3] + A13 * v[2] + A23 * v[1] + A[3] * v[0];
}

// w = (m M x M x M + sx K x M x M + sy M x K x M + sz M x M x K) u plus
// sum_q N_a(q) (q_h . grad u)(q) dt c_w V / 8 at the 2 x 2 x 2 Gauss points,
// q_h = -k (grad P + rho_g e_z), in Haar coordinates.  ax_, ay_, az_:
// -k dt c_w V / (8 h_d^2), per cell; pz0 = rho_g hz.
template <typename T>
__device__ __forceinline__ void cell_heat_haar(const T u[8], const T P[8], T m, T sx, T sy, T sz, T ax_, T ay_,
                                               T az_, T pz0, T w[8])
{
    T U[8];
#pragma unroll
    for (int i = 0; i < 8; i++) U[i] = u[i];
    haar3(U);
    // eigenvalues m mu mu mu + sx kappa mu mu + ..., mu = (3, 1), kappa =
    // (0, 2), times the 1/8 of the inverse transform
    const T a = T(0.375) * m, b = T(0.75) * sx, c = T(0.75) * sy, d = T(0.75) * sz;
    T W[8];
    W[0] = (T(9) * a) * U[0];
    W[1] = (T(3) * (a + b)) * U[1];
    W[2] = (T(3) * (a + c)) * U[2];
    W[4] = (T(3) * (a + d)) * U[4];
    W[3] = (a + b + c) * U[3];
    W[5] = (a + b + d) * U[5];
    W[6] = (a + c + d) * U[6];
    W[7] = ((a + b + c + d) * (T(1) / T(3))) * U[7];
    // per axis: the P differences along it (direct, then 2D Haar over the
    // cross-section), weighted by the axis factor times -1/4 (the 1/8 of the
    // inverse, the 2 of the broadcast along the axis, and the sign of the d
    // coefficients of U) and the per-term weights
    T px[4], py[4], pz[4];
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
        for (int t = 0; t < 2; t++) {
            px[s + 2 * t] = P[1 + 2 * s + 4 * t] - P[2 * s + 4 * t];
            py[s + 2 * t] = P[s + 2 + 4 * t] - P[s + 4 * t];
            pz[s + 2 * t] = P[s + 2 * t + 4] - P[s + 2 * t];
        }
    haar2(px);
    haar2(py);
    haar2(pz);
    pz[0] += T(4) * pz0;
    const T q4 = T(-1) / T(16), q12 = T(-1) / T(48), q36 = T(-1) / T(144);
    T A[4], v[4];
    A[0] = (ax_ * q4) * px[0]; A[1] = (ax_ * q12) * px[1]; A[2] = (ax_ * q12) * px[2]; A[3] = (ax_ * q36) * px[3];
    v[0] = U[1]; v[1] = U[3]; v[2] = U[5]; v[3] = U[7];
    haar_prod2(A, v, W[0], W[2], W[4], W[6]);
    A[0] = (ay_ * q4) * py[0]; A[1] = (ay_ * q12) * py[1]; A[2] = (ay_ * q12) * py[2]; A[3] = (ay_ * q36) * py[3];
    v[0] = U[2]; v[1] = U[3]; v[2] = U[6]; v[3] = U[7];
    haar_prod2(A, v, W[0], W[1], W[4], W[5]);
    A[0] = (az_ * q4) * pz[0]; A[1] = (az_ * q12) * pz[1]; A[2] = (az_ * q12) * pz[2]; A[3] = (az_ * q36) * pz[3];
    v[0] = U[4]; v[1] = U[5]; v[2] = U[6]; v[3] = U[7];
    haar_prod2(A, v, W[0], W[1], W[2], W[3]);
    haar3(W);
#pragma unroll
    for (int i = 0; i < 8; i++) w[i] = W[i];
}

template <typename T, int EPI, bool MASKED, bool GRADED>
__global__ __launch_bounds__(256) void k_q1_heat(const OpDev *__restrict__ ops,
                                                  const WorkItem *__restrict__ work,
                                                  const T *__restrict__ X, T *__restrict__ Y,
                                                  EpiArgs<T> ep)
{
    // Software pipeline over node planes, one barrier per plane:
    //   x planes live in a 3-deep LDS ring (plane p in slot p % 3), the four
    //   corner sums of each cell layer in a 2-deep ring; the global loads of
    //   plane L+2, of the coefficients of layer L+1 and of the epilogue
    //   operands of plane L are issued one iteration before they are used.
    // heat: a 5-deep x ring, so that the epilogue of plane P can read planes
    // P-1 .. P+1 of the injection-line rows while the next plane is stored
    constexpr int XR = 5;
    __shared__ T xs[XR][NB + 1][NB + 2];
    __shared__ T ps[3][NB + 1][NB + 2];
    __shared__ T S4[2][4][NB][NB + 1];
    __shared__ double red[4];

    const WorkItem wi = work[blockIdx.x];
    if (ep.active && !ep.active[wi.inst]) return;
    const OpDev &o = ops[wi.inst];
    const int nx = o.nx, ny = o.ny, nz = o.nz, NZ = o.NZ, m = o.dmask;
    const T *__restrict__ Xi = X + o.off;
    T *__restrict__ Yi = Y + o.off;
    const T HTS_GLOBAL *__restrict__ Pi = gptr<T>(o.P);
    const T HTS_GLOBAL *__restrict__ kk = gptr<T>(o.k);
    const T HTS_GLOBAL *__restrict__ lamc = gptr<T>(o.lam);
    const T HTS_GLOBAL *__restrict__ cTc = gptr<T>(o.cT);
    constexpr bool CHEB = EPI == EPI_CHEB || EPI == EPI_CHEB0;
    const T *__restrict__ Bi = (EPI == EPI_RESID || EPI == EPI_RESID_NORM || CHEB) ? ep.b + o.off : nullptr;
    T *__restrict__ Di = CHEB ? ep.d + o.off : nullptr;
    const T *__restrict__ Ii = CHEB ? ep.invd + o.off : nullptr;

    // Node and cell indices are instance-local and below 2^31: 32-bit index
    // arithmetic (the vectors are offset to the instance already).
    const int32_t plane32 = o.NX * o.NY;
    const int tid = threadIdx.x, tx = tid % NB, ty = tid / NB;
    const int cx0 = wi.tx * NOWN - 1, cy0 = wi.ty * NOWN - 1;
    const int cx = cx0 + tx, cy = cy0 + ty;
    const bool cin = cx >= 0 && cx < nx && cy >= 0 && cy < ny;
    const int32_t cbase = cin ? cx + nx * cy : 0;
    const int32_t cplane = nx * ny;

    // staged node columns of this thread: base index (0 outside the mesh, so
    // that the loads stay in range; the value is then discarded), whether the
    // column is in the mesh, whether its values are kept (not on a
    // constraining x/y face), and its constrained z-range
    int lj[2], li[2];
    bool ld[2], sval[2], scol[2];
    int32_t sbase[2];
    int sdlo[2], sdhi[2];
#pragma unroll
    for (int s = 0; s < 2; s++) {
        int c = tid + s * 256;
        ld[s] = c < NNCOL;
        li[s] = c % (NB + 1);
        lj[s] = c / (NB + 1);
        ColInfo lc;
        if (ld[s]) lc = col_info(o, cx0 + li[s], cy0 + lj[s]);
        else { lc.valid = 0; lc.base = 0; lc.xyc = 0; lc.dlo = 1; lc.dhi = 0; }
        sval[s] = lc.valid;
        scol[s] = lc.valid && !(MASKED && lc.xyc);
        sbase[s] = lc.valid ? (int32_t)lc.base : 0;
        sdlo[s] = lc.dlo;
        sdhi[s] = lc.dhi;
    }
    const bool owner = tx < NOWN && ty < NOWN;
    const int oi = cx0 + tx + 1, oj = cy0 + ty + 1;
    ColInfo oc = col_info(o, oi, oj);
    const bool own_ok = owner && oc.valid;
    int lr = -1;
    LineCol lh{-1, 0, -1, 0};
    if (o.lfcol && own_ok) {
        const LineCol HTS_GLOBAL *hp = gptr<LineCol>(o.lfcol) + oc.base;
        lh.first = hp->first;
        lh.kmin = hp->kmin;
        lh.kmax = hp->kmax;
    }
    if (!o.lfcol && o.lcol && own_ok) lr = gptr<int32_t>(o.lcol)[oc.base];

    // per-cell coefficient factors of the unscaled 1D products (formed in
    // double on the host, rounded once here)
    const T fm = T(o.q1m), fx = T(o.q1x), fy = T(o.q1y), fz = T(o.q1z);
    const T vx = T(o.q1vx), vy = T(o.q1vy), vz = T(o.q1vz);
    const T pz0 = T(o.rho_g * o.hz);   // rho_g is 0 where the pressure is piezometric
    const bool adv = o.cadv != 0.0;
    // graded meshes: every factor is a per-column part (from this thread's
    // hx, hy, formed once in double and rounded) times hz or 1 / hz of the
    // layer (tables, one value per layer)
    const bool graded = GRADED && o.hzs != nullptr;
    T gm = T(0), gx = T(0), gy = T(0), gz = T(0), gvx = T(0), gvy = T(0), gvz = T(0);
    if (graded) {
        const int ix = cx < 0 ? 0 : (cx >= nx ? nx - 1 : cx), iy = cy < 0 ? 0 : (cy >= ny ? ny - 1 : cy);
        const double ghx = o.hxs[ix], ghy = o.hys[iy], hxy = ghx * ghy;
        gm = T(hxy / 216.0);                           // x hz
        gx = T(o.cs * (ghy / ghx) / 36.0);             // x hz
        gy = T(o.cs * (ghx / ghy) / 36.0);             // x hz
        gz = T(o.cs * hxy / 36.0);                     // x 1/hz
        gvx = T(-o.cadv * 0.125 * ghy / ghx);          // x hz
        gvy = T(-o.cadv * 0.125 * ghx / ghy);          // x hz
        gvz = T(-o.cadv * 0.125 * hxy);                // x 1/hz
    }
    T c0 = T(0), c1 = T(0), c2 = T(0);
    if (CHEB) {
        const double *Sc = ep.S + (int64_t)wi.inst * NSLOT;
        c1 = T(Sc[ep.s1]);
        c2 = T(Sc[ep.s2]);
        if (EPI == EPI_CHEB0) c0 = T(Sc[ep.s0]);
    }

    // Plane / coefficient / epilogue loads are unconditional (clamped to a
    // valid address) and the keep-or-zero decision is a select applied when
    // the value is consumed, so no branch forces an early wait on a load.
    T pfx[2], pfp[2];
    bool pkeep[2] = {false, false}, pin[2] = {false, false};
    auto fetch_plane = [&](int k) {
        const int kc = k < 0 ? 0 : (k >= NZ ? NZ - 1 : k);
        const int32_t koff = kc * plane32;
        // the part of the keep decision that is the same for every column
        const bool kin = k >= 0 && k < NZ;
        const bool kkeep = kin && !(MASKED && (((m & 16) && k == 0) || ((m & 32) && k == NZ - 1)));
#pragma unroll
        for (int s = 0; s < 2; s++) {
            const int32_t gi = sbase[s] + koff;
            // EPI_CHEB0 operand: x0 = c0 D^-1 b, in the order of the
            // separate first Chebyshev kernel
            if (EPI == EPI_CHEB0) pfx[s] = c0 * Ii[gi] * Bi[gi];
            else pfx[s] = Xi[gi];
            pfp[s] = Pi[gi];
            bool keep = kkeep && scol[s];
            if (MASKED) keep = keep && !(k >= sdlo[s] && k <= sdhi[s]);
            pkeep[s] = keep;
            pin[s] = kin && sval[s];
        }
    };
    // ring slots: x planes in a ring of XR, pressure planes in a ring of 3
    auto store_plane = [&](int bx, int b) {
#pragma unroll
        for (int s = 0; s < 2; s++) {
            if (!ld[s]) continue;
            xs[bx][lj[s]][li[s]] = pkeep[s] ? pfx[s] : T(0);
            ps[b][lj[s]][li[s]] = pin[s] ? pfp[s] : T(0);
        }
    };
    T cfk = T(0), cfl = T(0), cfc = T(0);
    double cfh = 0.0, cfih = 0.0;     // graded: hz and 1/hz of the layer
    auto fetch_coef = [&](int L) {
        const int Lc = L < 0 ? 0 : (L >= nz ? nz - 1 : L);
        const int32_t ci = cbase + Lc * cplane;
        cfk = kk[ci];
        { cfl = lamc[ci]; cfc = cTc[ci]; }
        if (graded) { cfh = o.hzs[Lc]; cfih = o.ihzs[Lc]; }
    };
    // epilogue operands of one owned node
    const int32_t obase = own_ok ? (int32_t)oc.base : 0;
    T eb = T(0), ed = T(0), ei = T(0), ex = T(0);
    auto fetch_epi = [&](int L) {
        const int Lc = L < NZ ? L : NZ - 1;
        const int32_t gi = obase + Lc * plane32;
        if (Bi) eb = Bi[gi];
        if (EPI == EPI_CHEB) { ed = Di[gi]; ei = Ii[gi]; }
        if (EPI == EPI_CHEB0) ei = Ii[gi];
        if (EPI == EPI_CHEB || EPI == EPI_DOT || (MASKED && EPI != EPI_CHEB0)) ex = Xi[gi];
    };

    const int kb = wi.z0, ke = wi.z1;
    double acc = 0.0;
    T top[4] = {T(0), T(0), T(0), T(0)};

    // slots of plane L in the two rings, advanced by one per iteration
    int sx = (kb - 1 + XR) % XR, sp = (kb - 1 + 3) % 3;
    fetch_plane(kb - 1);
    store_plane(sx, sp);
    fetch_plane(kb);
    fetch_coef(kb - 1);

    for (int L = kb - 1; L <= ke; L++) {
        const bool comp = L <= ke - 1;
        const int sx1 = sx + 1 == XR ? 0 : sx + 1, sp1 = sp + 1 == 3 ? 0 : sp + 1;
        if (comp) store_plane(sx1, sp1);
        const T ck = cfk, cl = cfl, cc = cfc;
        const double lhz = cfh, lihz = cfih;
        if (L + 1 <= ke - 1) {
            fetch_plane(L + 2);
            fetch_coef(L + 1);
        }
        __syncthreads();
        // epilogue of plane L-1 (corner sums written in the previous iteration)
        if (L - 1 >= kb && own_ok && L - 1 < NZ) {
            const int P0 = L - 1, sb = P0 & 1;
            T v = S4[sb][3][ty][tx] + S4[sb][2][ty][tx + 1] + S4[sb][1][ty + 1][tx] + S4[sb][0][ty + 1][tx + 1];
            const int32_t gi = obase + P0 * plane32;
            if (lh.first >= 0 && P0 >= lh.kmin && P0 <= lh.kmax) {
                // injection-line row: operand values from the staged planes
                const LineFlat HTS_GLOBAL &R = gptr<LineFlat>(o.lflat)[lh.first + (P0 - lh.kmin)];
                const double HTS_GLOBAL *lco = gptr<double>(o.lcoef);
                const int ne = R.n;
                if (ne > 0 && !(MASKED && R.row_constrained)) {
                    T la = T(0);
                    for (int e = 0; e < ne; e++) {
                        const int of = R.off[e];
                        const int dx = (of & 3) - 1, dy = ((of >> 2) & 3) - 1, dk = ((of >> 4) & 3) - 1;
                        // plane P0 + dk = L - 1 + dk sits in slot sx - 1 + dk (mod XR)
                        const T xc = xs[(sx + XR - 1 + dk) % XR][ty + 1 + dy][tx + 1 + dx];
                        la += T(lco[R.src[e]] * R.w[e]) * xc;
                    }
                    v += la;
                }
            }
            if (lr >= 0) {
                const LineRow HTS_GLOBAL *rows = gptr<LineRow>(o.lrows);
                const LineEnt HTS_GLOBAL *ents = gptr<LineEnt>(o.lents);
                const double HTS_GLOBAL *lco = gptr<double>(o.lcoef);
                while (rows[lr].col == (int)oc.base && rows[lr].k < P0) lr++;
                const int rcol = rows[lr].col, rk = rows[lr].k;
                if (rcol == (int)oc.base && rk == P0 && !(MASKED && rows[lr].row_constrained)) {
                    T la = T(0);
                    for (int e = rows[lr].beg; e < rows[lr].end; e++) {
                        if (MASKED && ents[e].col_constrained) continue;
                        const int64_t col = ents[e].col;
                        const T xc = EPI == EPI_CHEB0 ? c0 * Ii[col] * Bi[col] : Xi[col];
                        la += T(lco[ents[e].src] * ents[e].w) * xc;
                    }
                    v += la;
                }
            }
            if (EPI == EPI_CHEB0) {
                ex = c0 * ei * eb;
                ed = ex;
            }
            if (MASKED && constrained(oc, P0, NZ, m)) v = ex;
            if (EPI == EPI_STORE) {
                Yi[gi] = v;
            } else if (EPI == EPI_RESID) {
                Yi[gi] = eb - v;
            } else if (EPI == EPI_RESID_NORM) {
                const T r = eb - v;
                Yi[gi] = r;
                acc += (double)r * (double)r;
            } else if (EPI == EPI_DOT) {
                Yi[gi] = v;
                acc += (double)ex * (double)v;
            } else if (CHEB) {
                const T r = eb - v;
                const T d = c1 * ed + c2 * ei * r;
                Di[gi] = d;
                Yi[gi] = ex + d;
            }
        }
        if (!comp) break;
        if (L >= kb) fetch_epi(L);
        // cell layer L between planes L and L+1
        const bool lay = cin && L >= 0 && L < nz;
        T bot[4] = {T(0), T(0), T(0), T(0)}, tp[4] = {T(0), T(0), T(0), T(0)};
        if (lay) {
            const int b0 = sp, b1 = sp1;
            const int x0 = sx, x1 = sx1;
            T u[8], w[8];
#pragma unroll
            for (int a = 0; a < 4; a++) {
                u[a] = xs[x0][ty + (a >> 1)][tx + (a & 1)];
                u[a + 4] = xs[x1][ty + (a >> 1)][tx + (a & 1)];
            }
            T lfm = fm, lfx = fx, lfy = fy, lfz = fz, lvx = vx, lvy = vy, lvz = vz, lpz0 = pz0;
            if (graded) {
                const T hz = T(lhz), ihz = T(lihz);
                lfm = gm * hz;
                lfx = gx * hz;
                lfy = gy * hz;
                lfz = gz * ihz;
                lvx = gvx * hz;
                lvy = gvy * hz;
                lvz = gvz * ihz;
                lpz0 = T(o.rho_g) * hz;
            }
            if (adv) {
                T pp[8];
#pragma unroll
                for (int a = 0; a < 4; a++) {
                    pp[a] = ps[b0][ty + (a >> 1)][tx + (a & 1)];
                    pp[a + 4] = ps[b1][ty + (a >> 1)][tx + (a & 1)];
                }
                cell_heat_haar(u, pp, cc * lfm, cl * lfx, cl * lfy, cl * lfz, ck * lvx, ck * lvy, ck * lvz, lpz0, w);
            } else {   // no convection in the mass-only heat operator
                cell_mass_stiff(u, cc * lfm, cl * lfx, cl * lfy, cl * lfz, w);
            }
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
        sp = sp1;
    }
    if (EPI == EPI_RESID_NORM || EPI == EPI_DOT) {
        double v = wave_sum(acc);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) ep.partial[wi.slot] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// ----------------------------------------------------------- setup kernels
// size of cell c along axis d (graded meshes: from the per-axis tables)
__device__ __forceinline__ static double cell_h(const OpDev &o, int d, int c)
{
    if (d == 0) return o.hxs ? o.hxs[c] : o.hx;
    if (d == 1) return o.hys ? o.hys[c] : o.hy;
    return o.hzs ? o.hzs[c] : o.hz;
}

__global__ void k_q1_inv_diag(OpDev o, double *__restrict__ out)
{
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= o.nnode) return;
    const int NX = o.NX, NY = o.NY;
    int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((int64_t)NX * NY));
    ColInfo c = col_info(o, i, j);
    if (constrained(c, k, o.NZ, o.dmask)) { out[n] = 1.0; return; }
    double d = 0.0;
    for (int dz = -1; dz <= 0; dz++)
        for (int dy = -1; dy <= 0; dy++)
            for (int dx = -1; dx <= 0; dx++) {
                int a = i + dx, b = j + dy, cc = k + dz;
                if (a < 0 || a >= o.nx || b < 0 || b >= o.ny || cc < 0 || cc >= o.nz) continue;
                const double hx = cell_h(o, 0, a), hy = cell_h(o, 1, b), hz = cell_h(o, 2, cc);
                const double V = hx * hy * hz;
                const double kd = (hy * hz / hx + hx * hz / hy + hx * hy / hz) / 9.0;
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
        for (int dz = -1; dz <= 0; dz++)
            for (int dy = -1; dy <= 0; dy++)
                for (int dx = -1; dx <= 0; dx++) {
                    int cx = i + dx, cy = j + dy, cz = k + dz;
                    if (cx < 0 || cx >= o.nx || cy < 0 || cy >= o.ny || cz < 0 || cz >= o.nz) continue;
                    const double h[3] = {cell_h(o, 0, cx), cell_h(o, 1, cy), cell_h(o, 2, cz)};
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
    double s = 0.0;
    for (int dz = -1; dz <= 0; dz++)
        for (int dy = -1; dy <= 0; dy++)
            for (int dx = -1; dx <= 0; dx++) {
                int cx = i + dx, cy = j + dy, cz = k + dz;
                if (cx < 0 || cx >= o.nx || cy < 0 || cy >= o.ny || cz < 0 || cz >= o.nz) continue;
                const double hx = cell_h(o, 0, cx), hy = cell_h(o, 1, cy), hz = cell_h(o, 2, cz);
                const double V8 = hx * hy * hz / 8.0, A4 = hx * hy / 4.0;
                int64_t ci = cx + (int64_t)o.nx * (cy + (int64_t)o.ny * cz);
                if (alpha) s += alpha[ci] * V8;
                // node is the top corner (az = 1) when the cell lies below it
                if (beta) s += beta[ci] * A4 * (dz == -1 ? 1.0 : -1.0);
            }
    y[n] = s;
}

}  // namespace

// ---------------------------------------------------------------- launchers
// pressure: wide tiles; heat: narrow tiles
template <typename T, int FIELD, int EPI, bool MASKED, bool G>
static void launch_k(int nwork, const OpDev *ops, const WorkItem *work, const T *x, T *y, const EpiArgs<T> &ep,
                     hipStream_t s)
{
    if constexpr (FIELD == 0)
        k_q1_pressure<T, EPI, MASKED, G><<<dim3(nwork), dim3(256), 0, s>>>(ops, work, x, y, ep);
    else
        k_q1_heat<T, EPI, MASKED, G><<<dim3(nwork), dim3(256), 0, s>>>(ops, work, x, y, ep);
}

template <typename T, int FIELD, bool MASKED, bool G>
static void dispatch_epi(int epi, const OpDev *ops, const WorkItem *work, int nwork, const T *x, T *y,
                         const EpiArgs<T> &ep, hipStream_t s)
{
    switch (epi) {
    case EPI_STORE: launch_k<T, FIELD, EPI_STORE, MASKED, G>(nwork, ops, work, x, y, ep, s); break;
    case EPI_RESID: launch_k<T, FIELD, EPI_RESID, MASKED, G>(nwork, ops, work, x, y, ep, s); break;
    case EPI_RESID_NORM: launch_k<T, FIELD, EPI_RESID_NORM, MASKED, G>(nwork, ops, work, x, y, ep, s); break;
    case EPI_DOT: launch_k<T, FIELD, EPI_DOT, MASKED, G>(nwork, ops, work, x, y, ep, s); break;
    case EPI_CHEB: launch_k<T, FIELD, EPI_CHEB, MASKED, G>(nwork, ops, work, x, y, ep, s); break;
    case EPI_CHEB0:
        if (!MASKED) throw Error(-1, "EPI_CHEB0 is for masked operators");
        launch_k<T, FIELD, EPI_CHEB0, true, G>(nwork, ops, work, x, y, ep, s);
        break;
    default: throw Error(-1, "bad epilogue");
    }
}

template <typename T, bool G>
static void launch_q1_g(int field, int epi, bool masked, const OpDev *ops, const WorkItem *work, int nwork,
                        const T *x, T *y, const EpiArgs<T> &ep, hipStream_t s)
{
    if (field == 0) {
        if (masked) dispatch_epi<T, 0, true, G>(epi, ops, work, nwork, x, y, ep, s);
        else dispatch_epi<T, 0, false, G>(epi, ops, work, nwork, x, y, ep, s);
    } else {
        if (masked) dispatch_epi<T, 1, true, G>(epi, ops, work, nwork, x, y, ep, s);
        else dispatch_epi<T, 1, false, G>(epi, ops, work, nwork, x, y, ep, s);
    }
}

// graded: some instance has a graded mesh; those kernels form the per-cell
// factors per layer, the uniform ones keep them in registers
template <typename T>
void launch_q1(int field, int epi, bool masked, bool graded, const OpDev *ops, const WorkItem *work, int nwork,
               const T *x, T *y, const EpiArgs<T> &ep, hipStream_t s)
{
    if (nwork <= 0) return;
    if (graded) launch_q1_g<T, true>(field, epi, masked, ops, work, nwork, x, y, ep, s);
    else launch_q1_g<T, false>(field, epi, masked, ops, work, nwork, x, y, ep, s);
    HTS_LAUNCH_CHECK();
}

template void launch_q1<double>(int, int, bool, bool, const OpDev *, const WorkItem *, int, const double *,
                                double *, const EpiArgs<double> &, hipStream_t);
template void launch_q1<float>(int, int, bool, bool, const OpDev *, const WorkItem *, int, const float *,
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
