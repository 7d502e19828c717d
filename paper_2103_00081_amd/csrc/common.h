// Internal declarations shared by the HIP translation units of libhts.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <stdexcept>
#include <string>

namespace hts {

// ----------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HTS_HIP(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            throw ::hts::Error(-4, std::string(#call) + ": " + hipGetErrorString(e_));      \
    } while (0)

#define HTS_LAUNCH_CHECK() HTS_HIP(hipGetLastError())

// ------------------------------------------------------- device structures
// Packed z-range of constrained nodes in one node column: lo | hi << 16;
// lo > hi means none.
constexpr int32_t DCOL_NONE = 0x0000FFFF;

// One node of the injection-line mass operator (heat): the row of node
// (column, k) holds entries [beg, end).
struct LineRow {
    int32_t col;               // node column i + NX*j (-1 terminates the list)
    int32_t k;                 // node plane
    int32_t beg, end;          // entries [beg, end)
    int32_t row_constrained;
    int32_t pad[3];
};
struct LineEnt {
    int32_t col;               // instance-local node index
    int32_t src;               // line source index (coefficient slot)
    int32_t col_constrained;
    int32_t pad;
    double w;                  // int N_a N_b dz / L along the line
};

// The same operator for Q1 meshes, laid out for the owner of a node: per node
// column the rows of planes kmin .. kmax are dense from index first (first < 0:
// no line rows); each row lists its entries by offset from the row's node
// (-1..1 per axis), so the kernel reads the operand from its staged planes.
constexpr int LINE_MAXE = 16;
struct LineCol {
    int32_t first, kmin, kmax, pad;
};
struct LineFlat {
    int32_t n;                 // entries (0: no row on this plane)
    int32_t row_constrained;
    uint8_t off[LINE_MAXE];    // (dx + 1) | (dy + 1) << 2 | (dk + 1) << 4
    int32_t src[LINE_MAXE];    // line source index (coefficient slot)
    double w[LINE_MAXE];
};

// Per-instance operator descriptor consumed by the apply kernels.
struct OpDev {
    int32_t nx, ny, nz;        // cells
    int32_t NX, NY, NZ;        // nodes
    int32_t p;                 // degree
    int32_t dmask;             // Dirichlet faces: bit f for face f
    double hx, hy, hz;         // cell sizes (uniform meshes)
    // graded (rectilinear) meshes: cell sizes along each axis and node z
    // coordinates; null on uniform meshes
    const double *hxs, *hys, *hzs;
    const double *ihzs;        // 1 / hz per cell layer
    const double *zn;
    double cm;                 // pressure: mass coefficient (1 transient, 0 steady)
    double cs;                 // stiffness scale: pressure dt*B (or 1), heat dt
    double cadv;               // heat: dt * c_w
    double rho_g;              // rho_w * g
    // Q1 cell factors of the unscaled 1D products on a uniform mesh, formed
    // on the host: mass V / 216, stiffness cs (hy hz / hx) / 36 (and the
    // y, z analogues), convection -cadv V / (8 h_d^2)
    double q1m, q1x, q1y, q1z, q1vx, q1vy, q1vz;
    const void *k;             // [ncell] k_c              (T)
    const void *lam;           // [ncell] lambda_c         (T, heat)
    const void *cT;            // [ncell] c_T,c            (T, heat)
    const void *P;             // [nnode] pressure for q_h (T, heat)
    const int32_t *dcol;       // [NX*NY] packed constrained z-range, or null
    const int32_t *lcol;       // [NX*NY] first LineRow of the column or -1; null = none
    const LineRow *lrows;
    const LineEnt *lents;
    const LineCol *lfcol;      // [NX*NY] (Q1) dense per-column rows, or null
    const LineFlat *lflat;
    const double *lcoef;       // per line source: dt c_w max(Q,0)/L at t^{n+1}
    const double *xyz;         // general hexahedra: node coordinates [nnode][3]; null on box meshes
    int64_t off;               // offset of the instance in batch node vectors
    int64_t nnode;
    int32_t field;
    int32_t pad;
};

// One block of work of the z-marching operator kernels: node-column tile
// (tx, ty) of instance inst, owning node planes [z0, z1).
struct WorkItem {
    int32_t inst, tx, ty, z0, z1;
    int32_t slot;              // natural index: where the block's partial sum goes
    int32_t pad1, pad2;
};

// Contiguous range [beg, end) of a batch vector belonging to one instance.
struct Chunk {
    int32_t inst, pad;
    int64_t beg, end;
};

// Per-instance scalar slots of the Krylov solvers.
enum Slot {
    S_BB = 0, S_RR, S_RZ, S_PQ, S_ALPHA, S_BETA, S_TOL2, S_ITER, S_STATUS, S_RR0,
    S_C1, S_C2, S_SCALE, S_TNEW, S_XTRA2, S_TMP0, S_TMP1, S_TMP2, S_TMP3,
    // outer (FP64) system of a field solve
    S_OBB = 19, S_OTOL2, S_ORR, S_ONORM, S_OINV, S_OSTATUS, S_FSCALE,
    S_CYC = 26,                // 1 if the instance takes part in the current FGMRES cycle
    S_XTRA = 27,               // initial guess X^n + S_XTRA (X^n - X^{n-1}) + S_XTRA2 (X^{n-1} - X^{n-2})
    S_CHEB = 28,               // Chebyshev coefficients: 2 per step, up to 16 steps
    // learned preconditioner in an inner solve: last ||r||^2 it was applied
    // to (-1: none yet), consecutive weak iterations, fallback flag, fallbacks
    S_NN_PREV = 60, S_NN_FAIL, S_NN_FB, S_NN_NFB,
    NSLOT = 64
};

// Epilogue of an operator application (what is written at each owned node).
enum Epi {
    EPI_STORE = 0,             // y = A x
    EPI_RESID = 1,             // y = b - A x
    EPI_RESID_NORM = 2,        // y = b - A x, partial += y^2
    EPI_DOT = 3,               // y = A x, partial += x . y
    EPI_CHEB = 4,              // r = b - A x; d = c1 d + c2 D^-1 r; y = x + d
    EPI_CHEB0 = 5              // the first two Chebyshev steps from x = 0: the
                               // operand is x0 = c0 D^-1 b (x ignored), d = x0,
                               // then as EPI_CHEB (Q1 and stencil levels)
};

template <typename T>
struct EpiArgs {
    const T *b;
    T *d;
    const T *invd;
    const double *S;           // per-instance scalar slots
    int32_t s1, s2;            // slots of the Chebyshev coefficients
    int32_t s0, pad;           // slot of c0 (EPI_CHEB0)
    double *partial;           // per work item partial sums
    const int32_t *active;     // per-instance flags (null = all active)
};

struct LevelGeo {              // one instance on one multigrid level
    int32_t NX, NY, NZ, pad;
    int64_t off;               // offset in the level's batch vectors
    int64_t n;
    const double *S64;         // assembled 27-point stencil [27][n] (levels >= 1)
    const float *S32;
    const int32_t *fmap[3];    // not used on device (host bookkeeping)
};

// ------------------------------------------------------------ launchers
// Operator kernels (op_q1.hip / op_q2.hip / op_hex.hip); degree 3 selects the
// Q1 kernels of general hexahedra (node coordinates in OpDev::xyz)
constexpr int DEGREE_HEX = 3;
template <typename T>
void launch_apply(int degree, int field, int epi, bool masked, bool graded, const OpDev *ops, const WorkItem *work,
                  int nwork, const T *x, T *y, const EpiArgs<T> &ep, hipStream_t s);
// Setup kernels, one instance per launch (op is passed by value).
// Inverse of the diagonal of the symmetric part of the operator (constrained
// rows: 1).  Pressure: M + s K_k.  Heat: M_cT + dt K_lambda.
void launch_inv_diag(const OpDev &op, double *inv_diag, hipStream_t s);
// 27-point assembled stencil [27][nnode] of the (Dirichlet-eliminated)
// symmetric part of a Q1 operator; offset e = (dx+1) + 3(dy+1) + 9(dz+1).
void launch_q1_stencil(const OpDev &op, double *S, hipStream_t s);
// the same for a Q1 operator of box or general hexahedral geometry
void launch_fine_stencil(const OpDev &op, double *S, hipStream_t s);
// y_a = sum_c alpha_c int N_a + beta_c int dN_a/dz   (static load vectors)
void launch_cell_loads(const OpDev &op, const double *alpha, const double *beta, double *y,
                       hipStream_t s);

}  // namespace hts
