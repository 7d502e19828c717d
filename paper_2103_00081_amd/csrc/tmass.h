// Host interface of the separable mass preconditioner (tmass.hip).
#pragma once
#include "common.h"

namespace hts {

// One instance: node dims, batch offset, the nodal scaling S (T) and the
// Thomas factors of the 1D matrix B_d of each axis, [3][N_d] doubles:
// sub-diagonal a_i, reciprocal pivot, modified super-diagonal c'_i.
struct TMassInst {
    int32_t N[3], pad;
    int64_t off;
    const void *s;
    const double *fac[3];
};

// z = S (B_x^-1 (x) B_y^-1 (x) B_z^-1) S r over all instances (constrained
// nodes of r ignored, of z zero).  Per axis: bbeg[ninst+1] first block of
// each instance, nblocks in total, lb lines per block, lds bytes per block.
template <typename T>
void launch_tmass(const TMassInst *inst, int ninst, const int64_t *const bbeg[3], const int64_t nblocks[3],
                  const int lb[3], const int lds[3], const int32_t *active, const OpDev *ops, const T *r, T *z,
                  hipStream_t s);

}  // namespace hts
