/*
 * hts.h -- C ABI of the MI355X hydrothermal time-stepping library (libhts.so).
 *
 * The library advances the one-way coupled groundwater-pressure /
 * heat-transport model of Sun et al., "An HPC-Based Hydrothermal Finite
 * Element Simulator for Modeling Underground Response to Community-Scale
 * Geothermal Energy Production" (Section 2, Eqs. 1-4), on hexahedral box
 * meshes (uniform, or graded per axis as in the refined site mesh of
 * Section 3.3) with Q1 or Q2 Lagrange elements, one backward-Euler
 * step at a time: first the Darcy pressure P^{n+1} (Eq. 3), then the
 * temperature T^{n+1} (Eq. 4) with the Darcy flux q = -k (grad P + rho_w g)
 * evaluated from P^{n+1} at every quadrature point.
 *
 * Conventions
 *   - z points up.  Faces are 0..5 = x-, x+, y-, y+, z-, z+.
 *   - Per-cell arrays are lexicographic with x fastest (c = i + nx*(j + ny*k));
 *     node arrays likewise over (p*nx+1) x (p*ny+1) x (p*nz+1) nodes.
 *   - Temperatures cross the ABI in kelvin, pressures in pascal, SI units
 *     everywhere else.
 *   - Every call returns an hts_status; C++ exceptions never cross the ABI;
 *     hts_last_error() returns a thread-local message for the last failure.
 *   - Host arrays passed in are copied; the caller keeps ownership.
 *     Device pointers passed in (hts_apply_operator) are caller-owned and
 *     must stay valid until the mesh's stream has been synchronised.
 *   - All device work of a mesh is issued on the stream given at creation
 *     (NULL = the null stream).  Calls on one mesh are not thread-safe.
 */
#ifndef HTS_H
#define HTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hts_mesh hts_mesh;
typedef struct hts_nn hts_nn;

typedef enum {
    HTS_OK = 0,
    HTS_ERR_ARG = -1,            /* invalid argument                          */
    HTS_ERR_STATE = -2,          /* call not valid in the current state       */
    HTS_ERR_NOMEM = -3,          /* device or host allocation failed          */
    HTS_ERR_HIP = -4,            /* a HIP runtime call failed                 */
    HTS_ERR_NOT_CONVERGED = -5,  /* a linear solve missed its tolerance       */
    HTS_ERR_BREAKDOWN = -6,      /* Krylov breakdown or non-finite residual   */
    HTS_ERR_UNSUPPORTED = -7     /* valid request this build does not handle  */
} hts_status;

typedef enum { HTS_PRESSURE = 0, HTS_TEMPERATURE = 1 } hts_field;

/* Arithmetic type of an operator application. */
typedef enum { HTS_FP64 = 0, HTS_FP32 = 1 } hts_precision;

/* Solve mode of a time step:
 *   FP64          - FP64 Krylov, FP64 multigrid;
 *   FP32_REFINED  - FP64 outer defect correction around an FP32 inner
 *                   Krylov solve with an FP32 operator and smoother; dot
 *                   products, the coarse-grid solve and the update stay FP64;
 *   LEARNED       - pressure uses flexible CG preconditioned by the learned
 *                   network (opts.nn) with the multigrid V-cycle as fallback. */
typedef enum { HTS_MODE_FP64 = 0, HTS_MODE_FP32_REFINED = 1, HTS_MODE_LEARNED = 2 } hts_mode;

typedef enum { HTS_BC_DIRICHLET = 0, HTS_BC_NEUMANN = 1, HTS_BC_NONE = 2 } hts_bc_kind;

typedef enum { HTS_LINE_HEAT = 0, HTS_LINE_WELL = 1 } hts_line_kind;

typedef enum { HTS_TF_CONST = 0, HTS_TF_SIN = 1, HTS_TF_SQUARE = 2 } hts_tf_kind;

/* A value affine in space with a periodic time part:
 *   v(x,y,z,t) = c0 + cx*x + cy*y + cz*z + amp*w(t),
 *   w = 0 (CONST), sin(2 pi t/period + phase) (SIN), or the square wave
 *   +1 where that sine is >= 0 and -1 elsewhere (SQUARE).
 * Hydrostatic pressure p_top + rho_w g (z_top - z) is c0 = p_top + rho_w g z_top,
 * cz = -rho_w g.  Neumann fluxes and line rates must have cx = cy = cz = 0. */
typedef struct {
    int32_t kind;
    double c0, cx, cy, cz, amp, period, phase;
} hts_timefn;

/* Device-memory hooks.  When alloc is NULL the library uses hipMalloc/hipFree. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} hts_allocator;

/* Box mesh [origin, origin+extent] with ncells cells of degree 1 or 2.
 * Uniform unless edges[d] is given: then axis d is graded, with the cell
 * edges edges[d][0..ncells[d]] (host array, copied; strictly increasing from
 * origin[d] to origin[d]+extent[d], within 1e-9 of the extent).  Graded
 * (rectilinear) meshes refine around features, as the paper's site mesh is
 * refined around the piles (Section 3.3, Fig. 10b); degree-2 cells keep
 * their mid-edge nodes at the cell midpoints.  Zero-initialise the
 * descriptor so that unused fields are NULL. */
typedef struct {
    double origin[3];
    double extent[3];
    int32_t ncells[3];
    int32_t degree;
    int32_t device;       /* HIP device ordinal */
    void *stream;         /* hipStream_t; NULL = null stream */
    hts_allocator alloc;
    const double *edges[3];   /* NULL = uniform axis */
    /* General hexahedra (degree 1 only): coordinates of every node, host
     * [nnode][3] with x fastest (node i + NX (j + NY k)), copied.  The box
     * topology is kept and each cell is the trilinear image of the unit
     * cube (Section 3.3, Fig. 10b: a site mesh refined around the piles);
     * origin and extent are then not used for geometry and edges must be
     * NULL.  Every cell must keep det J > 0 at its Gauss points (else
     * HTS_ERR_ARG).  Line sources, Dirichlet columns and Neumann faces need
     * the box geometry and return HTS_ERR_UNSUPPORTED on such meshes. */
    const double *coords;
} hts_mesh_desc;

/* Materials (Section 2 mixture rules and mobility, Tables 1 and 3):
 *   k = K_i / mu_w  (or K / (rho_w g) when permeability is NULL),
 *   lambda = (1-phi) lambda_s + phi lambda_w,  c_T = (1-phi) c_s + phi c_w,
 * unless lambda_bulk / rhoc_bulk give the bulk values directly.
 * All arrays are host [ncell] arrays.  B_poro is the storage modulus of
 * Eq. 1 in Pa; B_poro <= 0 selects the steady pressure equation. */
typedef struct {
    const double *permeability;            /* K_i [m^2]              */
    const double *hydraulic_conductivity;  /* K [m/s], if no K_i     */
    const double *porosity;                /* phi [-]                */
    const double *lambda_solid;            /* lambda_s [W/m/K]       */
    const double *rhoc_solid;              /* c_s [J/m^3/K]          */
    const double *lambda_bulk;             /* optional lambda [W/m/K] */
    const double *rhoc_bulk;               /* optional c_T [J/m^3/K]  */
    double rho_w, mu_w, c_w, lambda_w, g, B_poro;
} hts_materials;

typedef struct {
    int32_t mode;            /* hts_mode                                        */
    double rtol;             /* relative residual ||b-Ax|| <= rtol ||b|| (1e-8) */
    int32_t max_iter;        /* Krylov iterations per solve (inner, total)      */
    int32_t gmres_restart;   /* FGMRES restart length (30)                      */
    int32_t cheb_degree;     /* Chebyshev smoothing degree per side (2)         */
    int32_t mg_coarse_max;   /* coarsen each instance until a level has <= this
                                many nodes; that level is solved with a dense
                                FP64 inverse (n^2 entries, read whole by every
                                coarse solve)                                 */
    int32_t heat_cheb_degree;/* degree of the heat Chebyshev-Jacobi preconditioner
                                (0, the default: 4 on degree-1 cells, 2 on
                                degree-2 cells); its polynomial is the Chebyshev one of the
                                ellipse over the real interval of D^-1 A with
                                the imaginary extent of the convection term;
                                instances whose imaginary extent reaches the
                                interval's half-width keep degree 2          */
    double inner_rtol;       /* inner tolerance of FP32_REFINED (1e-5)          */
    int32_t check_every;     /* host convergence check every n iterations (1)   */
    int32_t use_graph;       /* replay captured HIP graphs for time steps       */
    hts_nn *nn;              /* network for HTS_MODE_LEARNED                    */
    int32_t verbose;
    int32_t heat_precond;    /* 0: multigrid V-cycle (Galerkin levels of the
                                symmetric part M_cT + dt K_lambda, Chebyshev
                                smoothing with the full heat operator);
                                1: Chebyshev-Jacobi with the full heat
                                operator (default: the heat operator is mass
                                dominated);
                                2: separable (M_x + a K_x) x (M_y + a K_y) x
                                (M_z + a K_z) line solves scaled by the nodal
                                capacity, a = dt median(lambda / c_T) (Q1;
                                Q2 uses 1)                                      */
    int32_t extrapolate;     /* 2 (default): each field's solve starts from the
                                value at t^n + dt of the polynomial through the
                                known time levels X^n, X^{n-1}, X^{n-2} (at most
                                quadratic; see hts_set_previous_state); 1: at
                                most linear; 0: from X^n.  Either way the step
                                meets the same residual test.                */
} hts_solver_opts;

typedef struct {
    int32_t iters[2];        /* Krylov iterations per field (inner total)     */
    int32_t outer[2];        /* defect-correction outer iterations per field  */
    double relres[2];        /* true FP64 relative residual per field         */
    int32_t fallbacks;       /* learned -> multigrid fallbacks in the step    */
    int32_t status[2];       /* hts_status per field                          */
    double time_ms[2];       /* device time of each field's solve             */
} hts_step_stats;

typedef struct {
    int32_t levels;          /* encoder/decoder levels (4)                    */
    int32_t channels[4];     /* channels per level (16, 32, 48, 64)           */
    int32_t device;
    void *stream;
    uint64_t seed;           /* weight initialisation                         */
} hts_nn_desc;

typedef struct {
    int32_t epochs_done;
    int32_t pairs;
    double loss_first;
    double loss_last;
    double val_loss;
} hts_train_stats;

/* ---------------------------------------------------------------- meshes */

/* Fill opts with defaults (FP64 mode, rtol 1e-8, ...). */
void hts_default_opts(hts_solver_opts *opts);

/* Create a mesh (Section 3.3: a hexahedral mesh of the site box).
 * degree must be 1 or 2; every ncells entry >= 1; extent > 0; fewer than
 * 65535 nodes along an axis and fewer than 2^29 nodes in all (one FP64 vector
 * of the mesh stays below 4 GiB, which the kernels' 32-bit offsets assume).
 * HTS_ERR_ARG on bad geometry, HTS_ERR_HIP if the device cannot be set. */
hts_status hts_create_mesh(const hts_mesh_desc *desc, hts_mesh **out);

void hts_destroy_mesh(hts_mesh *mesh);

/* Copy material arrays to the device and form the cellwise k, lambda, c_T
 * (Section 2, mixture rules).  Must precede any solve or apply.
 * HTS_ERR_ARG if a required array is NULL or a constant is not positive. */
hts_status hts_set_materials(hts_mesh *mesh, const hts_materials *mat);

/* Face boundary condition for one field (Section 3.3, Fig. 12).
 * DIRICHLET: nodal value v(x,y,z,t^{n+1}) imposed strongly.
 * NEUMANN:   outward normal flux (pressure: Darcy flux q.n [m/s]; heat:
 *            heat flux [W/m^2]) entering the right-hand sides of Eqs. 3-4.
 * NONE:      natural no-flux.  Faces are applied in call order (a node on
 *            two Dirichlet faces takes the later value). */
hts_status hts_set_face_bc(hts_mesh *mesh, hts_field field, int32_t face, int32_t kind,
                           const hts_timefn *value);

/* Volumetric heat source f [W/m^3] per cell (host [ncell]); NULL clears. */
hts_status hts_set_volume_source(hts_mesh *mesh, const double *w_per_m3);

/* Vertical line source over [z0, z1] at (x, y):
 *   HTS_LINE_HEAT: heat rate per metre q_l(t) [W/m] (energy piles, Section 3.2);
 *   HTS_LINE_WELL: well rate Q(t) [m^3/s] spread uniformly over the screen;
 *                  Q > 0 injects water at T_inj [K], which adds c_w (Q/L)
 *                  (T_inj - T) to the heat balance.
 * Rates must be spatially constant time functions. */
hts_status hts_add_line_source(hts_mesh *mesh, double x, double y, double z0, double z1,
                               int32_t kind, const hts_timefn *rate, double T_inj);

/* Dirichlet column (an energy pile held at a temperature, Section 3.3): the
 * node column nearest (x, y) over z0 <= z <= z1 is constrained to v(t). */
hts_status hts_add_dirichlet_column(hts_mesh *mesh, hts_field field, double x, double y,
                                    double z0, double z1, const hts_timefn *value);

/* Set / get a field's nodal state (host [nnode]) and the mesh time.
 * Setting a field's state forgets its previous time level. */
hts_status hts_set_state(hts_mesh *mesh, hts_field field, const double *host, double t);
hts_status hts_get_state(hts_mesh *mesh, hts_field field, double *host, double *t);

/* The previous time levels of a field: level 1 is the state before the last
 * committed step and dt_prev that step's size, level 2 the state before the
 * second-last one and its step's size (dt_prev 0: not known).  A committed
 * step (hts_solve_step, hts_advance) shifts them; the next step starts its
 * solve from the extrapolation through the known levels (opts.extrapolate),
 * which changes the iterate's rounding, not the residual test.  A checkpoint
 * that must resume bit for bit saves all three levels: set the state first
 * (it forgets both previous levels), then level 1 (it forgets level 2), then
 * level 2.  host: [nnode], ignored (may be NULL) when dt_prev is 0 on set
 * and when the level is not known on get.  Errors: HTS_ERR_ARG for a bad
 * field or level, negative or non-finite dt_prev, non-finite values, or
 * level 2 without level 1. */
hts_status hts_set_previous_state(hts_mesh *mesh, hts_field field, int32_t level, const double *host,
                                  double dt_prev);
hts_status hts_get_previous_state(hts_mesh *mesh, hts_field field, int32_t level, double *host, double *dt_prev);

/* Spectral estimates behind the heat Chebyshev preconditioner of a mesh:
 * v[0] the step size they were made for (0: none), v[1] and v[2] the largest
 * eigenvalue of D^-1 A without and with the convection term, v[3] the
 * imaginary extent of D^-1 A (the convection term's).  They depend on the
 * Darcy flux of the step in which the preconditioner was first built for
 * that dt, and are reused while dt stays (a new dt or changed coefficients
 * or boundary data estimate again).  A checkpoint that must resume bit for
 * bit saves them with the state and the previous level.  set: entries must
 * be finite and >= 0, v[1], v[2] > 0 unless v[0] is 0; HTS_ERR_ARG else. */
hts_status hts_get_heat_spectrum(hts_mesh *mesh, double *v4);
hts_status hts_set_heat_spectrum(hts_mesh *mesh, const double *v4);

/* Node / cell counts of a mesh. */
hts_status hts_mesh_sizes(const hts_mesh *mesh, int64_t *nnode, int64_t *ncell);

/* ------------------------------------------------------------- operators */

/* y = A x for one field's operator on the constrained space (Eq. 3 or
 * Eq. 4 left-hand side at time step dt): constrained rows are the identity,
 * free rows see only free columns.
 *   PRESSURE:    A = M + dt B_poro K_k   (A = K_k when B_poro <= 0 or dt <= 0)
 *   TEMPERATURE: A = M_{c_T} + dt K_lambda + dt c_w C(q_h) + dt c_w M_inj,
 *                with q_h from the mesh's current pressure state.
 * x_dev, y_dev: device arrays of nnode doubles (HTS_FP64) or floats (HTS_FP32)
 * on the mesh's device; distinct buffers.  Asynchronous on the mesh stream. */
hts_status hts_apply_operator(hts_mesh *mesh, hts_field field, hts_precision prec, double dt,
                              const void *x_dev, void *y_dev);

/* ----------------------------------------------------------------- solves */

/* Replace the pressure state by the steady solution of Eq. 3 (B_poro term
 * dropped) at the current time.  Transactional: unchanged on failure. */
hts_status hts_solve_steady_pressure(hts_mesh *mesh, const hts_solver_opts *opts,
                                     hts_step_stats *stats);

/* One backward-Euler step of size dt: P^{n+1} (Eq. 3), then T^{n+1}
 * (Eq. 4).  Every solve ends with the true FP64 residual check
 * ||b - A x||_2 <= rtol ||b||_2 on the eliminated system.  Transactional: on
 * HTS_ERR_NOT_CONVERGED / HTS_ERR_BREAKDOWN the state and time are not
 * advanced; stats (may be NULL) is filled either way. */
hts_status hts_solve_step(hts_mesh *mesh, double dt, const hts_solver_opts *opts,
                          hts_step_stats *stats);

/* Advance n_instances independent meshes by n_steps steps of size dt as one
 * batch: every kernel launch covers all instances, each with its own
 * convergence state.  stats: [n_instances] (last step), may be NULL.
 * With opts->use_graph the per-step launch sequence is captured once and
 * replayed.  Stops at the first failing step (those instances are not
 * advanced past it).  The batch (work lists, multigrid hierarchies, dense
 * coarse inverses, captured graphs) is kept for the next call with the same
 * meshes in the same order, up to four such sets; changing a mesh's
 * materials or boundary data, autotuning or destroying it drops them.
 * Each mesh may appear once. */
hts_status hts_advance(hts_mesh *const *meshes, int32_t n_instances, int32_t n_steps, double dt,
                       const hts_solver_opts *opts, hts_step_stats *stats);

/* The same operation as hts_apply_operator (same arguments, layout, result
 * bit for bit) for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * It calls no allocator: the descriptors, the work list, the heat
 * operator's time slots, line-source coefficients and FP32 piezometric
 * pressure live in one static 40 MiB device array per GPU, held until the
 * process ends (FP32 heat applies need 4 bytes per node of it, so meshes up
 * to about 10 M nodes; larger ones give HTS_ERR_ARG before any device
 * work).  Every call on a GPU reuses that array: calls that overlap on one
 * GPU (several streams or threads) race and must be serialised by the
 * caller.  The mesh's own derived data must exist: HTS_ERR_STATE if the mesh
 * changed since its last hts_apply_operator, hts_autotune or solve (which
 * rebuild it), or if the heat operator is asked for without a pressure
 * state.  All work is enqueued on the mesh's stream; nothing synchronises. */
hts_status hts_apply_operator_noalloc(hts_mesh *m, hts_field field, hts_precision prec, double dt,
                                      const void *x_dev, void *y_dev);

/* Time the fine-level operators of these meshes at several z-chunk depths
 * (node planes one workgroup marches through) and keep the fastest per
 * (kernel family, field, precision, node dims) for later launches; with
 * HTS_TUNE_CACHE set to a path the choices are also written there and read
 * back by later processes.  Forgets the meshes' cached batches (graphs). */
hts_status hts_autotune(hts_mesh *const *meshes, int32_t n);

/* Device time and algorithmic traffic of the matrix-free fine-level
 * operator launches, per [field][precision] class. */
typedef struct {
    int64_t launches;   /* launches recorded                                  */
    double ms;          /* summed device time (HIP events around each launch) */
    double bytes;       /* algorithmic bytes: every node vector the launch's
                           epilogue reads or writes once, plus the per-cell
                           coefficients, at the operator's precision          */
    double flops;       /* algorithmic floating-point operations              */
} hts_kernel_times;

/* enable = 1: reset and start recording every fine-level operator launch of
 * every mesh (adds two events per launch).  enable = 0: stop, wait for the
 * recorded launches and write the totals to out[field][precision] (out may
 * be NULL).  Not thread-safe. */
hts_status hts_kernel_timing(int32_t enable, hts_kernel_times out[2][2]);

/* Achievable-bandwidth reference for the measurements: copy `bytes` from
 * src to dst (device buffers, 16-byte aligned, caller-owned, not
 * overlapping) with a plain streaming kernel, once untimed, then `reps`
 * times between two HIP events on `stream` (NULL = null stream);
 * ms_per_copy (may be NULL) gets the mean device time of one copy, which
 * reads and writes `bytes` each.  HTS_ERR_ARG on negative sizes or
 * misaligned / missing buffers. */
hts_status hts_stream_copy(const void *src, void *dst, int64_t bytes, int32_t reps, void *stream,
                           double *ms_per_copy);

const char *hts_last_error(void);

/* -------------------------------------------------- learned preconditioner */
/* A 3D convolutional encoder-decoder (levels L in 2..4, widths channels[l],
 * multiples of 8 up to 64; 3x3x3 kernels, zero padding 1, ReLU, stride-2
 * downsampling, linear upsampling, additive skips) maps the normalised
 * pressure residual r / rms(r) and the standardised node log10 permeability
 * to an error estimate e / (gamma rms(r)).  Layers in parameter order:
 * enc0a (2 -> c0), enc0b (c0 -> c0), then down_l (stride 2, c_{l-1} -> c_l)
 * and enc_l (c_l -> c_l) for l = 1..L-1, then dec_l (c_{l+1} -> c_l) for
 * l = L-2..0 with d_l = relu(dec_l(up d_{l+1})) + e_l, then out (c0 -> 1).
 * BF16 weights and activations, FP32 accumulation on the matrix cores, FP32
 * master weights with Adam.  Used by HTS_MODE_LEARNED as the preconditioner
 * of flexible CG for Eq. 3, with the V-cycle as fallback; every converged
 * answer is judged by the FP64 residual. */

/* Create a network with He-normal weights drawn from desc->seed (output
 * layer scaled by 0.1, zero biases).  HTS_ERR_ARG on bad levels/channels. */
hts_status hts_nn_create(const hts_nn_desc *desc, hts_nn **out);
void hts_nn_destroy(hts_nn *nn);

/* Parameter vector in exchange layout: per layer in the order above,
 * W[cout][cin][kz][ky][kx] (cross-correlation weights) then b[cout]; host
 * FP64.  Set converts to FP32 masters and BF16 compute copies.
 * HTS_ERR_ARG when count differs from hts_nn_num_params. */
hts_status hts_nn_num_params(const hts_nn *nn, int64_t *count);
hts_status hts_nn_set_params(hts_nn *nn, const double *theta, int64_t count);
hts_status hts_nn_get_params(const hts_nn *nn, double *theta, int64_t count);

/* One forward pass on a node grid dims = {NX, NY, NZ} (x fastest), host
 * arrays: input [n][2] FP32 (residual, feature; rounded to BF16), out [n]
 * FP32 network output.  With target [n] (rounded to BF16): loss = mean
 * over nodes with mask == 0 (mask NULL: all) of (out - target)^2, and, if
 * grad is not NULL, its gradient in exchange layout (FP64 host array of
 * hts_nn_num_params entries), by the library's backward kernels. */
hts_status hts_nn_eval(hts_nn *nn, const int32_t dims[3], const float *input, const float *target,
                       const uint8_t *mask, float *out, double *loss, double *grad);

/* One 3x3x3 convolution layer (zero padding 1, stride 1 or 2) on the BF16
 * matrix cores, exposed for verification.  Host arrays; tensors are
 * channels-last [voxel][channel] with x fastest, voxel grid din = {NX, NY,
 * NZ} at the input and ((din - 1) / stride + 1) at the output; BF16 as
 * uint16 bit patterns; w [cout][cin][3][3][3] (kz, ky, kx); cin, cout
 * multiples of 8 in [8, 64].
 *   op 0: out[o][co] = bias[co] + sum w x            (x, w, bias optional)
 *   op 1: out[i][ci] = gradient of sum(g * conv(x)) w.r.t. x   (g, w)
 *   op 2: out = gradient w.r.t. w in w's layout; out_bias[co] = sum g (x, g)
 * FP32 results; stream may be NULL. */
hts_status hts_nn_conv3d(int32_t op, int32_t cin, int32_t cout, int32_t stride, const int32_t din[3],
                         const uint16_t *x, const uint16_t *w, const float *bias, const uint16_t *g, float *out,
                         float *out_bias, void *stream);

/* One Adam update (Kingma and Ba) of n FP32 parameters by the kernel that
 * hts_nn_train runs, exposed for verification: with beta1 0.9, beta2 0.999,
 * eps 1e-8 and gi = g[i] * gscale (gscale: 1 / minibatch size),
 *   m = beta1 m + (1 - beta1) gi,  v = beta2 v + (1 - beta2) gi^2,
 *   w -= lr (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps).
 * w, m, v: host arrays [n], updated in place; g: host [n]; wbf (may be NULL):
 * host [n] BF16 bit patterns of the new w (round to nearest even).  step >= 1
 * is the 1-based update count.  HTS_ERR_ARG on n < 0, step < 1, lr <= 0 or
 * a missing array; stream may be NULL. */
hts_status hts_nn_adam(int64_t n, int32_t step, double lr, double gscale, float *w, float *m, float *v,
                       const float *g, uint16_t *wbf, void *stream);

/* Time `reps` forward passes of the network on a node grid dims = {NX, NY,
 * NZ} with HIP events on the network's stream; flop_per_forward (may be
 * NULL) gets 2 * 27 * Cin * Cout * voxels summed over the layers (logical
 * channels).  For measurement. */
hts_status hts_nn_time_forward(hts_nn *nn, const int32_t dims[3], int32_t reps, double *ms_per_forward,
                               double *flop_per_forward);

/* For each of the n_draws meshes (same node grid, pressure state set): run
 * n_steps plain multigrid-CG pressure steps (Eq. 3, FP64, rtol 1e-10) from the
 * mesh's state without changing it, and from every inner CG solve keep up to
 * pairs_per_solve iterates x_k, evenly spaced, as pairs
 * (r_k = A e_k, e_k = x* - x_k), both divided by rms(r_k) and stored as
 * BF16, with the draw's node feature and Dirichlet mask.  Pairs accumulate
 * over calls. */
hts_status hts_nn_harvest(hts_nn *nn, hts_mesh *const *meshes, int32_t n_draws, int32_t n_steps,
                          double dt, int32_t pairs_per_solve);

/* Train on the harvested pairs of every draw but the last val_draws with the
 * library's BF16 forward and backward kernels and FP32 Adam (beta 0.9,
 * 0.999, eps 1e-8), minibatches of `batch` pairs (gradients averaged),
 * shuffled with the network seed.  Gamma is fixed once, by the first call
 * (the median rms(e)/rms(r) of its training pairs) or by hts_nn_load; each
 * call divides the targets of pairs harvested since the previous call by it,
 * so every stored target is scaled exactly once (epochs may be 0).  out: mean training loss of the first and last epoch and the mean loss
 * on the pairs of the held-out draws. */
hts_status hts_nn_train(hts_nn *nn, int32_t epochs, double lr, int32_t batch, int32_t val_draws,
                        hts_train_stats *out);

/* Parameters and gamma to / from a binary file (magic "HTSNN001", levels,
 * channels, gamma, count, FP64 exchange-layout parameters).  Load checks
 * the architecture; HTS_ERR_ARG on mismatch or I/O failure.  Load fixes
 * gamma to the stored value (targets already scaled are rescaled to it). */
hts_status hts_nn_save(const hts_nn *nn, const char *path);
hts_status hts_nn_load(hts_nn *nn, const char *path);

#ifdef __cplusplus
}
#endif
#endif /* HTS_H */
