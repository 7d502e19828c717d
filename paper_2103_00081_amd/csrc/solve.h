// Batches of instances and the solvers that run over them (solve.hip).
#pragma once
#include <functional>
#include <map>
#include <tuple>
#include <memory>
#include <vector>

#include "internal.h"
#include "tmass.h"

namespace hts {


template <typename T>
void launch_apply(int degree, int field, int epi, bool masked, bool graded, const OpDev *ops, const WorkItem *work,
                  int nwork, const T *x, T *y, const EpiArgs<T> &ep, hipStream_t s);
void launch_inv_diag(const OpDev &op, double *inv_diag, hipStream_t s);
void launch_q1_stencil(const OpDev &op, double *S, hipStream_t s);
void launch_fine_stencil(const OpDev &op, double *S, hipStream_t s);

// Per-instance operator descriptors of one operator variant (FP64 and FP32).
struct Tables {
    int field = 0;
    std::vector<OpDev> h64, h32;
    DBuf<OpDev> d64, d32;
};

// One multigrid level of a batch (level 0 is the matrix-free fine level).
struct Level {
    int64_t ntot = 0;
    std::vector<int> dims;                 // NX, NY, NZ per instance
    std::vector<int64_t> off, soff;        // instance offsets (vectors, stencils)
    std::vector<LevelDev> h64;
    DBuf<LevelDev> g64, g32;
    std::vector<int> present, cont;        // instance on this level / continues to a coarser one
    std::vector<Chunk> hch, hch_all;
    DBuf<Chunk> ch, ch_all;
    const Chunk *ch_ext = nullptr;         // chunks of continuing instances (level 0: the batch's)
    const Chunk *ch_all_ext = nullptr;     // chunks of every present instance
    int nch = 0, nch_all = 0;
    std::vector<DBuf<double>> Ainv;        // dense inverses of instances ending here
    DBuf<CoarseDev> cd;
    int ncd = 0;
    int64_t crows = 0;
    DBuf<int32_t> segp;
    RedCtx red{};
    DBuf<double> S64;
    DBuf<float> S32;
    DBuf<double> invd64, x64, xb64, b64, d64, t64;
    DBuf<float> invd32, x32, xb32, b32, d32, t32;
    DBuf<double> cheb;                     // [ninst][NSLOT] Chebyshev coefficients
    std::vector<DBuf<int32_t>> qdcol;      // Q1 vertex Dirichlet columns under a Q2 fine level
};

struct Hier {
    int field = 0;
    int deg = 2;                  // Chebyshev steps launched
    int deg_req = 2;              // the degree asked for (the cache key)
    bool multigrid = true;
    double ratio = 15.0;          // Chebyshev interval [lmax/ratio, 1.1 lmax] on the fine level
    double ratio_coarse = 15.0;   // and on coarse levels
    double dt = -1.0;
    Tables ops;                            // fine-level operator
    std::vector<Level> lev;
    std::vector<double> lmax;
    // separable mass preconditioner (heat, Q1)
    bool tensor = false;
    DBuf<TMassInst> tm64, tm32;
    std::vector<DBuf<double>> tfac;
    DBuf<double> ts64;
    DBuf<float> ts32;
    DBuf<int64_t> tl[3];                   // first block of each instance per axis
    int64_t tn[3] = {0, 0, 0};             // blocks per axis
    int tlb[3] = {1, 1, 1}, tlds64[3] = {0, 0, 0}, tlds32[3] = {0, 0, 0};
};

struct FieldStats {
    std::vector<int> status, iters, outer, fallbacks;
    std::vector<double> relres;
    double ms = 0.0;
};

struct Batch {
    std::vector<hts_mesh *> m;
    int n = 0, p = 1, device = 0;
    hipStream_t s = nullptr;
    Alloc *al = nullptr;
    std::vector<int64_t> off;
    int64_t ntot = 0, ctot = 0;
    bool graded = false;       // some instance has a graded mesh
    bool general = false;      // the instances are general hexahedral meshes

    std::vector<Chunk> hch;
    DBuf<Chunk> ch;
    int nch = 0;
    DBuf<int32_t> chp;
    RedCtx rch{};
    // fine-level work lists per field and precision (index [field][prec],
    // prec 0 FP64, 1 FP32: the z-chunk depth is tuned per field and
    // precision)
    std::vector<WorkItem> hwork[2][2];
    DBuf<WorkItem> work[2][2];
    int nwork[2][2] = {{0, 0}, {0, 0}};
    DBuf<int32_t> wkp[2][2];
    RedCtx rwk[2][2]{};
    int zc_force[2][2] = {{0, 0}, {0, 0}};

    DBuf<double> S;
    DBuf<int32_t> active;
    // learned preconditioner: which instances take the network or the
    // multigrid fallback in the current application, and the solve's flags
    DBuf<int32_t> nn_use, nn_mg, act_save;
    double *hS = nullptr;
    int32_t *hact = nullptr;      // flags as last exported (coherent pinned)
    double *hexpS = nullptr;      // slots as last exported (coherent pinned)
    uint32_t *hseq = nullptr;     // sequence number of the last export (coherent pinned)
    uint32_t exp_seq = 0;
    // set by cg / fgmres on return: no work was queued after their last
    // export, so hexpS still holds the current slots
    bool exported_last = false;
    DBuf<double> partial, redout, redout2, redout3;

    DBuf<double> Pn, Tn, P1, T1, g, b, x, r, z, pp, q, rold, y, ld0, ld1, inner_b, inner_x;
    DBuf<double> Pp, Tp, Ppp, Tpp;   // previous time levels n-1, n-2 (valid where hist_dt, hist_dt2 > 0)
    // one instance: Pn, Tn, Pp, Tp are the mesh's own state buffers (no
    // gather or scatter copies)
    bool alias_state = false;
    DBuf<float> P32, b32, x32, r32, z32, p32, q32, rold32, y32;

    int gm_m = 0;
    DBuf<double> V64, Z64, gH, gcs, gsn, gg, gy, gh1, gh2;
    DBuf<float> V32, Z32;
    DBuf<int32_t> gkdim;

    DBuf<BcDev> bc[2];
    DBuf<int64_t> srows[2];
    DBuf<int32_t> srowptr[2];
    DBuf<SrcEnt> sents[2];
    DBuf<SrcDev> ssrc[2];
    int64_t nsrows[2] = {0, 0};
    DBuf<SrcDev> lsrc;
    int nlsrc = 0;
    DBuf<double> lcoef;
    std::vector<int> lbase;

    Tables massP, massH, app;
    int app_field = -1;
    double app_dt = -1.0;
    bool app_steady = false;
    // pressure hierarchies by (steady, dt, smoothing degree, coarse-level cap)
    // (at most two, least recently used replaced)
    std::map<std::tuple<int, double, int, int>, std::unique_ptr<Hier>> hier;
    std::map<std::tuple<int, double, int, int>, uint64_t> hier_used;
    uint64_t hier_clock = 0;
    std::unique_ptr<Hier> heat;
    std::vector<double> cadv_save;   // advection scale per instance (heat tables)

    // observers used to harvest training pairs for the learned preconditioner:
    // cg_hook(x, k) sees the iterate x_k of every FP64 CG solve (k = 0 first),
    // inner_hook(A, x*) each converged FP64 inner pressure solution
    std::function<void(const double *, int)> cg_hook;
    std::function<void(const Tables &, const double *)> inner_hook;

    // Captured launch sequences (fixed-length Krylov chunks).  Every kernel
    // in them is predicated on the per-instance active flags, so a chunk
    // replayed past convergence does no work for converged instances.
    // Graphs embed buffer addresses: drop them whenever a buffer they use
    // is reallocated.
    struct Graph {
        hipGraph_t g = nullptr;
        hipGraphExec_t e = nullptr;
    };
    std::map<std::string, Graph> graphs;
    hipStream_t cap = nullptr;
    bool use_graph = false;
    std::string graph_tag;   // identifies the preconditioner a captured chunk calls
    // optional: a suffix for the key of the next captured chunk (a
    // preconditioner whose launch sequence changes between chunks)
    std::function<std::string()> chunk_mode;
    int chunk_cap = 0;   // > 0: at most this many CG iterations per captured chunk
    std::map<std::string, int> last_iters;   // iterations of the previous solve per captured system
    int hist_tag = 0;                          // outer refinement step of the current inner solve
    void drop_graphs();
    void replay(const std::string &key, const std::function<void()> &body);

    ~Batch();
    int pick_zc(int field, int prec, const hts_mesh *M, int64_t tiles) const;
    void build_work();
    void make_tables(Tables &t, int field, double dt, bool steady, bool mass_only);
    Tables &apply_tables(int field, double dt, bool steady)
    {
        if (app_field != field || app_dt != dt || app_steady != steady) {
            make_tables(app, field, dt, steady, false);
            app_field = field;
            app_dt = dt;
            app_steady = steady;
        }
        return app;
    }
    void upload_S();
    void export_state();
    void download_S();
    void slots_from_export();      // hS = hexpS (the last export is current)
    void set_active(const std::vector<int32_t> &a);
    std::vector<int32_t> get_active();
    bool any_active();
    VecCtx vctx(bool use_active = true) const;

    template <typename T>
    void fine_apply(int field, const OpDev *ops, int epi, bool masked, const T *x, T *y, const EpiArgs<T> &ep);
    template <typename T> void apply_lvl(Hier &H, int l, int epi, bool masked, const T *x, T *y, EpiArgs<T> ep);
    template <typename T> void apply_op(const Tables &t, int epi, bool masked, const T *x, T *y, EpiArgs<T> ep);

    void estimate_lmax(Hier &H, int l, std::vector<double> &lmax);
    // given: lmax(D^-1 A) per instance (else estimated by power iteration)
    void build_smoother(Hier &H, int l, int steps, double ratio, const std::vector<double> *given = nullptr,
                        const std::vector<double> *beta = nullptr, const std::vector<int> *steps_i = nullptr);
    void build_hierarchy(Hier &H, const hts_solver_opts &o);
    Hier &pressure_hier(bool steady, double dt, const hts_solver_opts &o);
    Hier &heat_prec(double dt, const hts_solver_opts &o);

    template <typename T> void smooth(Hier &H, int l, int steps, int first, const T *b, T *&cur, T *&oth);
    template <typename T> void vcycle(Hier &H, int l, const T *b, T *x);
    template <typename T> void cheb_prec(Hier &H, const T *b, T *x);
    template <typename T> void cheb_from_zero(Hier &H, int l, int deg, const T *b, T *&cur, T *&oth);
    template <typename T> void tmass_prec(Hier &H, const T *b, T *x);
    void build_tmass(Hier &H, double dt);
    template <typename T>
    // x0_zero: x holds zeros on entry, so the initial residual is b itself
    int cg(const Tables &A, const std::function<void(const T *, T *)> &M, const T *b, T *x, int maxit, bool flexible,
           int check_every, bool x0_zero = false);
    template <typename T>
    void fgmres(const Tables &A, const std::function<void(const T *, T *)> &M, const T *b, T *x, int maxit, int mres,
                int check_every, bool x0_zero = false);
    void ensure_gmres(int mres);

    FieldStats solve_field(int field, Hier *mg, const Tables &A, double *b64, double *x64, const hts_solver_opts &o,
                           std::vector<int32_t> participants, Hier *hprec);
    void set_time(const std::vector<double> &tnew, const std::vector<double> &fscale,
                  const std::vector<double> *xtra = nullptr, const std::vector<double> *xtra2 = nullptr);
    void xtra_factors(int field, double dt, const hts_solver_opts &o, std::vector<double> &c1,
                      std::vector<double> &c2) const;
    void pressure_rhs(Hier &H, bool steady);
    void heat_rhs(Hier &H);
    void gather_state();
    void scatter_state();
    FieldStats solve_pressure(double dt, bool steady_all, const hts_solver_opts &o);
    FieldStats solve_heat(double dt, const hts_solver_opts &o);
    int step(double dt, const hts_solver_opts &o, std::vector<hts_step_stats> *stats);
};

std::shared_ptr<Batch> build_batch(const std::vector<hts_mesh *> &ms);
// learned preconditioner on one instance's slice: z = gamma rms(r) Net(r / rms(r), feature);
// gate: device flag of the instance (0: nothing runs, z untouched)
void nn_precondition(hts_nn *nn, Batch &B, int inst, const double *r, double *z, const int32_t *gate);
// network inputs and workspaces of every instance (before graph capture)
void nn_prepare(hts_nn *nn, Batch &B);
uint64_t nn_serial(const hts_nn *nn);
// tuned z-chunk depth of the fine operator kernels (0 = none recorded)
int tuned_zc(int degree, int field, int prec, int NX, int NY, int NZ);
void set_tuned_zc(int degree, int field, int prec, int NX, int NY, int NZ, int zc);
void save_tuning();
std::shared_ptr<Batch> solo_batch(hts_mesh *m);
// cached batch of several meshes (same meshes, same order)
std::shared_ptr<Batch> multi_batch(const std::vector<hts_mesh *> &ms);

}  // namespace hts
