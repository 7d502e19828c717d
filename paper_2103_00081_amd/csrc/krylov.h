// Per-instance scalar kernels of the Krylov solvers (krylov.hip).
#pragma once
#include "common.h"

namespace hts {

void gm_begin(int ninst, int32_t *active, double *S, double *g, int mres, int32_t *kdim, hipStream_t s);
// h1: first projection (j+1 per instance); h2: second projection (j+1) and
// the squared norm of w after the first projection (entry j+1)
void gm_solve(int ninst, const int32_t *cyc, int mres, const double *H, const double *g, const int32_t *kdim,
              double *y, hipStream_t s);
void outer_check(int ninst, int32_t *active, double *S, const double *rr, hipStream_t s);
void set_inner_tol(int ninst, const int32_t *active, double *S, double floor2, double factor2, hipStream_t s);
void convert_plain(int64_t n, const double *in, float *out, hipStream_t s);
// Fallback rule of the learned preconditioner, on the device (one thread per
// instance): nn_gate_init clears an inner solve's history; nn_gate_begin,
// before each application, decides from S_RR which instances take the
// network (use_nn) and which the V-cycle (use_mg) and saves the active flags;
// nn_gate_check, after the network and the reduction of |z|^2 into S_TMP2,
// sends instances with a non-finite output to the V-cycle and sets the
// active flags to use_mg; nn_gate_end restores the saved flags.
void nn_gate_init(int ninst, double *S, hipStream_t s);
void nn_gate_begin(int ninst, const int32_t *active, double *S, int32_t *use_nn, int32_t *use_mg,
                   int32_t *act_save, hipStream_t s);
void nn_gate_check(int ninst, double *S, int32_t *use_nn, int32_t *use_mg, int32_t *active, hipStream_t s);
void nn_gate_end(int ninst, const int32_t *act_save, int32_t *active, hipStream_t s);
void set_otol(int ninst, const int32_t *active, double *S, const double *bb, int stride, double rtol2, hipStream_t s);

}  // namespace hts
