// Per-instance scalar work of the Krylov solvers (one thread per instance):
// FGMRES Arnoldi bookkeeping with Givens rotations and back substitution,
// and the outer FP64 defect-correction test.
#include "common.h"
#include "krylov.h"
#include "arnoldi.h"

namespace hts {

namespace {

__global__ void k_gm_begin(int ninst, int32_t *active, double *S, double *g, int mres, int32_t *kdim)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    double *Si = S + (int64_t)i * NSLOT;
    Si[S_CYC] = 0.0;
    if (!active[i]) return;
    const double rr = Si[S_RR];
    kdim[i] = 0;
    if (!isfinite(rr)) {
        Si[S_STATUS] = -6;
        active[i] = 0;
        return;
    }
    if (rr <= Si[S_TOL2]) {
        Si[S_STATUS] = 0;
        active[i] = 0;
        return;
    }
    Si[S_CYC] = 1.0;
    const double beta = sqrt(rr);
    double *gi = g + (int64_t)i * (mres + 1);
    gi[0] = beta;
    for (int j = 1; j <= mres; j++) gi[j] = 0.0;
    Si[S_SCALE] = 1.0 / beta;
    Si[S_STATUS] = 1;
}

__global__ void k_gm_solve(int ninst, const int32_t *cyc, int mres, const double *H, const double *g,
                           const int32_t *kdim, double *y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst || !cyc[i]) return;
    const int kd = kdim[i];
    const double *Hi = H + (int64_t)i * (mres + 1) * mres;
    const double *gi = g + (int64_t)i * (mres + 1);
    double *yi = y + (int64_t)i * mres;
    for (int r = kd - 1; r >= 0; r--) {
        double s = gi[r];
        for (int c = r + 1; c < kd; c++) s -= Hi[r * mres + c] * yi[c];
        yi[r] = s / Hi[r * mres + r];
    }
}

// outer defect correction: v0 = ||b - A x||^2
__global__ void k_outer_check(int ninst, int32_t *active, double *S, const double *rr)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst || !active[i]) return;
    double *Si = S + (int64_t)i * NSLOT;
    const double v = rr[i];
    Si[S_ORR] = v;
    Si[S_ONORM] = sqrt(fmax(v, 0.0));
    Si[S_OINV] = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
    if (!isfinite(v)) {
        Si[S_OSTATUS] = -6;
        active[i] = 0;
    } else if (v <= Si[S_OTOL2]) {
        Si[S_OSTATUS] = 0;
        active[i] = 0;
    }
}

__global__ void k_set_otol(int ninst, const int32_t *active, double *S, const double *bb, int stride, double rtol2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst || (active && !active[i])) return;
    double *Si = S + (int64_t)i * NSLOT;
    const double v = bb[(int64_t)i * stride];
    Si[S_OBB] = v;
    Si[S_OTOL2] = rtol2 * v;
    Si[S_OSTATUS] = 1;
}

// inner tolerance of a defect-correction solve whose RHS is r / ||r||:
// TOL2 = max(floor2, factor2 * OTOL2 / ORR)
__global__ void k_set_inner_tol(int ninst, const int32_t *active, double *S, double floor2, double factor2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst || (active && !active[i])) return;
    double *Si = S + (int64_t)i * NSLOT;
    const double rel = Si[S_ORR] > 0.0 ? Si[S_OTOL2] / Si[S_ORR] : 1.0;
    Si[S_BB] = 1.0;
    Si[S_TOL2] = fmax(floor2, factor2 * rel);
    Si[S_ITER] = 0.0;
    Si[S_STATUS] = 1.0;
}

// Learned preconditioner: after two consecutive network-preconditioned
// iterations that each leave ||r_{k+1}||^2 > 0.81 ||r_k||^2 (a residual
// norm reduction weaker than 0.9), or on a non-finite residual or network
// output, the instance takes the V-cycle for the rest of the inner solve.
__global__ void k_nn_gate_init(int ninst, double *S)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    double *Si = S + (int64_t)i * NSLOT;
    Si[S_NN_PREV] = -1.0;
    Si[S_NN_FAIL] = 0.0;
    Si[S_NN_FB] = 0.0;
    Si[S_NN_NFB] = 0.0;
}

__global__ void k_nn_gate_begin(int ninst, const int32_t *active, double *S, int32_t *use_nn, int32_t *use_mg,
                                int32_t *act_save)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    const int32_t act = active[i];
    act_save[i] = act;
    if (!act) {
        use_nn[i] = 0;
        use_mg[i] = 0;
        return;
    }
    double *Si = S + (int64_t)i * NSLOT;
    bool fb = Si[S_NN_FB] != 0.0;
    if (!fb) {
        const double rr = Si[S_RR], prev = Si[S_NN_PREV];
        double fails = Si[S_NN_FAIL];
        if (!isfinite(rr)) {
            fb = true;
        } else if (prev >= 0.0 && rr > 0.81 * prev) {
            fails += 1.0;
            fb = fails >= 2.0;
        } else {
            fails = 0.0;
        }
        Si[S_NN_PREV] = rr;
        Si[S_NN_FAIL] = fails;
        if (fb) {
            Si[S_NN_FB] = 1.0;
            Si[S_NN_NFB] += 1.0;
        }
    }
    use_nn[i] = fb ? 0 : 1;
    use_mg[i] = fb ? 1 : 0;
}

__global__ void k_nn_gate_check(int ninst, double *S, int32_t *use_nn, int32_t *use_mg, int32_t *active)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    double *Si = S + (int64_t)i * NSLOT;
    if (use_nn[i] && !isfinite(Si[S_TMP2])) {
        Si[S_NN_FB] = 1.0;
        Si[S_NN_NFB] += 1.0;
        use_nn[i] = 0;
        use_mg[i] = 1;
    }
    active[i] = use_mg[i];
}

__global__ void k_nn_gate_end(int ninst, const int32_t *act_save, int32_t *active)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ninst) active[i] = act_save[i];
}

__global__ void k_convert_plain_df(int64_t n, const double *in, float *out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

}  // namespace

void set_inner_tol(int ninst, const int32_t *active, double *S, double floor2, double factor2, hipStream_t s)
{
    k_set_inner_tol<<<dim3((ninst + 63) / 64), dim3(64), 0, s>>>(ninst, active, S, floor2, factor2);
    HTS_LAUNCH_CHECK();
}

static dim3 inst_grid(int ninst) { return dim3((unsigned)((ninst + 63) / 64)); }

void nn_gate_init(int ninst, double *S, hipStream_t s)
{
    k_nn_gate_init<<<inst_grid(ninst), dim3(64), 0, s>>>(ninst, S);
    HTS_LAUNCH_CHECK();
}

void nn_gate_begin(int ninst, const int32_t *active, double *S, int32_t *use_nn, int32_t *use_mg,
                   int32_t *act_save, hipStream_t s)
{
    k_nn_gate_begin<<<inst_grid(ninst), dim3(64), 0, s>>>(ninst, active, S, use_nn, use_mg, act_save);
    HTS_LAUNCH_CHECK();
}

void nn_gate_check(int ninst, double *S, int32_t *use_nn, int32_t *use_mg, int32_t *active, hipStream_t s)
{
    k_nn_gate_check<<<inst_grid(ninst), dim3(64), 0, s>>>(ninst, S, use_nn, use_mg, active);
    HTS_LAUNCH_CHECK();
}

void nn_gate_end(int ninst, const int32_t *act_save, int32_t *active, hipStream_t s)
{
    k_nn_gate_end<<<inst_grid(ninst), dim3(64), 0, s>>>(ninst, act_save, active);
    HTS_LAUNCH_CHECK();
}

void convert_plain(int64_t n, const double *in, float *out, hipStream_t s)
{
    if (n <= 0) return;
    k_convert_plain_df<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(n, in, out);
    HTS_LAUNCH_CHECK();
}

static dim3 g1(int n) { return dim3((n + 63) / 64); }

void gm_begin(int ninst, int32_t *active, double *S, double *g, int mres, int32_t *kdim, hipStream_t s)
{
    k_gm_begin<<<g1(ninst), dim3(64), 0, s>>>(ninst, active, S, g, mres, kdim);
    HTS_LAUNCH_CHECK();
}
void gm_solve(int ninst, const int32_t *cyc, int mres, const double *H, const double *g, const int32_t *kdim,
              double *y, hipStream_t s)
{
    k_gm_solve<<<g1(ninst), dim3(64), 0, s>>>(ninst, cyc, mres, H, g, kdim, y);
    HTS_LAUNCH_CHECK();
}
void outer_check(int ninst, int32_t *active, double *S, const double *rr, hipStream_t s)
{
    k_outer_check<<<g1(ninst), dim3(64), 0, s>>>(ninst, active, S, rr);
    HTS_LAUNCH_CHECK();
}
void set_otol(int ninst, const int32_t *active, double *S, const double *bb, int stride, double rtol2, hipStream_t s)
{
    k_set_otol<<<g1(ninst), dim3(64), 0, s>>>(ninst, active, S, bb, stride, rtol2);
    HTS_LAUNCH_CHECK();
}

}  // namespace hts
