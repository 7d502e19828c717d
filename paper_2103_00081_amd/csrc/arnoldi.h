// FGMRES Arnoldi column update of one instance, run by the reduction that
// produces its second-pass coefficients (vec.hip).
#pragma once
#include "common.h"

namespace hts {

// Arguments of the column update besides the instance's scalar slots.
struct ArnArgs {
    int32_t j, mres, maxit, pad;
    const double *h1;          // [ninst][j + 1] first-pass coefficients
    double *H, *cs, *sn, *g;   // Hessenberg columns, Givens rotations, rhs
    int32_t *kdim;
};

// Column j of the Hessenberg matrix from classical Gram-Schmidt applied twice:
// h = h1 + h2.  The new basis vector is w' - V h2 with w' the vector after
// the first projection; the basis is orthonormal and w' - V h2 is orthogonal
// to it, so its squared norm is |w'|^2 - |h2|^2, where h2 is small (the
// second pass only removes rounding), so the difference does not cancel.
// a2 = h2 of this instance (j + 1 entries) followed by |w'|^2.
// Called by every thread of the block (blockDim >= j + 2); col, cr, sr are
// LDS arrays of at least j + 2, j and j entries.  The column and the earlier
// rotations are gathered in parallel, one thread applies the rotations in
// order, and the column is written back in parallel.
__device__ inline void arnoldi_column(int i, int32_t *active, double *S, const ArnArgs &A, const double *a2,
                                      double *col, double *cr, double *sr)
{
    const int j = A.j, mres = A.mres, t = threadIdx.x;
    double *Si = S + (int64_t)i * NSLOT;
    double *Hi = A.H + (int64_t)i * (mres + 1) * mres;   // H[r][c] = Hi[r * mres + c]
    double *ci = A.cs + (int64_t)i * mres, *si = A.sn + (int64_t)i * mres;
    double *gi = A.g + (int64_t)i * (mres + 1);
    const double *a1 = A.h1 + (int64_t)i * (j + 1);
    if (t <= j) col[t] = a1[t] + a2[t];
    if (t < j) {
        cr[t] = ci[t];
        sr[t] = si[t];
    }
    __syncthreads();
    if (t == 0) {
        double h22 = 0.0;
        for (int r = 0; r <= j; r++) h22 += a2[r] * a2[r];
        const double hn = sqrt(fmax(a2[j + 1] - h22, 0.0));
        col[j + 1] = hn;
        for (int r = 0; r < j; r++) {
            const double a = col[r], b = col[r + 1];
            col[r] = cr[r] * a + sr[r] * b;
            col[r + 1] = -sr[r] * a + cr[r] * b;
        }
        const double a = col[j], b = col[j + 1];
        const double rho = hypot(a, b);
        ci[j] = rho > 0.0 ? a / rho : 1.0;
        si[j] = rho > 0.0 ? b / rho : 0.0;
        col[j] = rho;
        col[j + 1] = 0.0;
        gi[j + 1] = -si[j] * gi[j];
        gi[j] = ci[j] * gi[j];
        A.kdim[i] = j + 1;
        Si[S_ITER] += 1.0;
        const double res2 = gi[j + 1] * gi[j + 1];
        Si[S_RR] = res2;
        Si[S_SCALE] = hn > 0.0 ? 1.0 / hn : 0.0;
        if (!isfinite(res2) || !isfinite(hn) || rho == 0.0) {
            Si[S_STATUS] = -6;
            active[i] = 0;
        } else if (res2 <= Si[S_TOL2] || hn == 0.0) {
            Si[S_STATUS] = 0;
            active[i] = 0;
        } else if (Si[S_ITER] >= A.maxit) {
            Si[S_STATUS] = -5;
            active[i] = 0;
        } else if (j == mres - 1) {
            active[i] = 0;   // cycle ends; status stays 1 (restart)
        }
    }
    __syncthreads();
    if (t <= j + 1) Hi[t * mres + j] = col[t];
}

}  // namespace hts
