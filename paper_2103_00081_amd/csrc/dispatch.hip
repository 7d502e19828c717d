// Degree dispatch of the operator kernels.
#include "common.h"

namespace hts {

template <typename T>
void launch_q1(int field, int epi, bool masked, bool graded, const OpDev *ops, const WorkItem *work, int nwork,
               const T *x, T *y, const EpiArgs<T> &ep, hipStream_t s);
template <typename T>
void launch_q2(int field, int epi, bool masked, bool graded, const OpDev *ops, const WorkItem *work, int nwork,
               const T *x, T *y, const EpiArgs<T> &ep, hipStream_t s);
void launch_q1_inv_diag(const OpDev &op, double *inv_diag, hipStream_t s);
void launch_q2_inv_diag(const OpDev &op, double *inv_diag, hipStream_t s);
void launch_q1_cell_loads(const OpDev &op, const double *alpha, const double *beta, double *y, hipStream_t s);
void launch_q2_cell_loads(const OpDev &op, const double *alpha, const double *beta, double *y, hipStream_t s);
template <typename T>
void launch_hex(int field, int epi, bool masked, const OpDev *ops, const WorkItem *work, int nwork, const T *x,
                T *y, const EpiArgs<T> &ep, hipStream_t s);
void launch_hex_inv_diag(const OpDev &op, double *inv_diag, hipStream_t s);
void launch_hex_stencil(const OpDev &op, double *S, hipStream_t s);
void launch_hex_cell_loads(const OpDev &op, const double *alpha, const double *beta, double *y, hipStream_t s);

// graded: some instance has a graded mesh
template <typename T>
void launch_apply(int degree, int field, int epi, bool masked, bool graded, const OpDev *ops, const WorkItem *work,
                  int nwork, const T *x, T *y, const EpiArgs<T> &ep, hipStream_t s)
{
    if (degree == 1) launch_q1<T>(field, epi, masked, graded, ops, work, nwork, x, y, ep, s);
    else if (degree == DEGREE_HEX) launch_hex<T>(field, epi, masked, ops, work, nwork, x, y, ep, s);
    else launch_q2<T>(field, epi, masked, graded, ops, work, nwork, x, y, ep, s);
}
template void launch_apply<double>(int, int, int, bool, bool, const OpDev *, const WorkItem *, int, const double *,
                                   double *, const EpiArgs<double> &, hipStream_t);
template void launch_apply<float>(int, int, int, bool, bool, const OpDev *, const WorkItem *, int, const float *,
                                  float *, const EpiArgs<float> &, hipStream_t);

void launch_inv_diag(const OpDev &op, double *inv_diag, hipStream_t s)
{
    if (op.xyz) launch_hex_inv_diag(op, inv_diag, s);
    else if (op.p == 1) launch_q1_inv_diag(op, inv_diag, s);
    else launch_q2_inv_diag(op, inv_diag, s);
}

void launch_cell_loads(const OpDev &op, const double *alpha, const double *beta, double *y, hipStream_t s)
{
    if (op.xyz) launch_hex_cell_loads(op, alpha, beta, y, s);
    else if (op.p == 1) launch_q1_cell_loads(op, alpha, beta, y, s);
    else launch_q2_cell_loads(op, alpha, beta, y, s);
}

void launch_fine_stencil(const OpDev &op, double *S, hipStream_t s)
{
    if (op.xyz) launch_hex_stencil(op, S, s);
    else launch_q1_stencil(op, S, s);
}

}  // namespace hts
