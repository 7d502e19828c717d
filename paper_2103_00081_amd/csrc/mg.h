// Host-side interface of the multigrid kernels (mg.hip).
#pragma once
#include "common.h"

namespace hts {

// One instance on one multigrid level (device table entry).
struct LevelDev {
    int32_t NX, NY, NZ, pad;
    int64_t off;               // offset of the instance in the level's batch vectors
    int64_t n;                 // nodes of the instance on this level
    const void *S;             // 27-point stencil [27][n] (double or float), levels >= 1
};

// Dense inverse of one instance's coarsest operator.
struct CoarseDev {
    const double *Ainv;        // [n][n] row-major
    int64_t n;
    int64_t off;               // offset in the coarsest level's batch vectors
    int64_t row0;              // first global row (rows numbered across instances)
    int32_t inst, pad;         // instance index in the batch
};

template <typename T>
void launch_stencil(int epi, const LevelDev *lev, const Chunk *chunks, int nchunk, const int32_t *active, const T *x,
                    T *y, const EpiArgs<T> &ep, hipStream_t s);
template <typename T>
void launch_cheb0(const Chunk *chunks, int nchunk, const int32_t *active, const double *S, int slot, const T *invd,
                  const T *b, T *d, T *x, hipStream_t s);
template <typename T>
// mask_coarse: zero the result at coarse nodes whose fine node is constrained
// (coarse operators with eliminated rows there, e.g. the Q1 level under Q2)
void launch_restrict(const LevelDev *fine, const LevelDev *coarse, const OpDev *fops, const Chunk *cchunks,
                     int nchunk, const int32_t *active, const T *rf, T *bc, int mask_coarse, hipStream_t s);
template <typename T>
void launch_prolong_add(const LevelDev *fine, const LevelDev *coarse, const OpDev *fops, const Chunk *fchunks,
                        int nchunk, const int32_t *active, const T *xc, T *xf, hipStream_t s);
void launch_rap(int fNX, int fNY, int fNZ, const double *Sf, int cNX, int cNY, int cNZ, double *Sc, hipStream_t s);
void launch_stencil_invdiag(const double *S, int64_t n, double *out, hipStream_t s);
// x = Ainv b for the ncd instances listed in cd (rows numbered across them)
template <typename T>
void launch_coarse_solve(const CoarseDev *cd, int ncd, int64_t total_rows, const int32_t *active, const T *b,
                         T *x, hipStream_t s);

}  // namespace hts
