// Matrix-free Q2 operators (placeholder until the Q2 kernels land).
#include "common.h"

namespace hts {

template <typename T>
void launch_q2(int, int, bool, const OpDev *, const WorkItem *, int, const T *, T *, const EpiArgs<T> &, hipStream_t)
{
    throw Error(-7, "Q2 operators are not available in this build");
}
template void launch_q2<double>(int, int, bool, const OpDev *, const WorkItem *, int, const double *, double *,
                                const EpiArgs<double> &, hipStream_t);
template void launch_q2<float>(int, int, bool, const OpDev *, const WorkItem *, int, const float *, float *,
                               const EpiArgs<float> &, hipStream_t);
void launch_q2_inv_diag(const OpDev &, double *, hipStream_t) { throw Error(-7, "Q2 not available"); }
void launch_q2_cell_loads(const OpDev &, const double *, const double *, double *, hipStream_t)
{
    throw Error(-7, "Q2 not available");
}

}  // namespace hts
