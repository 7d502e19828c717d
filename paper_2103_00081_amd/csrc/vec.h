// Host-side interface of the batched vector kernels (vec.hip).
#pragma once
#include "arnoldi.h"
#include "common.h"

#include <vector>

namespace hts {

// Chunks: nodes per block of the vector kernels (at most 4 per thread of a
// 256-thread block; the basis kernels assume that bound) and on the coarse
// multigrid levels.
constexpr int CHUNK_LEN = 1024;
constexpr int CHUNK_LEN_COARSE = 256;

struct VecCtx {
    const Chunk *chunks;       // device chunk list of the batch vectors
    int nchunk;
    const int32_t *active;     // per-instance flags (null = all)
    const double *S;           // per-instance scalar slots
    hipStream_t stream;
};

// Partial sums of instance i occupy partial[seg_ptr[i] .. seg_ptr[i+1]) (times
// ncomp), in the natural order of its chunks or tiles (for k_reduce).
struct RedCtx {
    const int32_t *seg_ptr;    // [ninst + 1]
    int nseg;                  // = ninst
    int single = -1;           // one instance: its partial count (seg_ptr not read)
};

enum RedOp {
    RED_NONE = 0,
    RED_STORE = 1,             // S[slot] = v0
    RED_STORE2 = 2,            // S[slot] = v0, S[slot+1] = v1
    RED_CG_ALPHA = 3,          // PQ = v0, ALPHA = RZ / PQ
    RED_CG_CONV = 4,           // RR = v0, ITER++, convergence / breakdown flags
    RED_CG_BETA = 5,           // BETA = (v0 - v1) / RZ, RZ = v0
    RED_CG_INIT = 6,           // RR = RR0 = v0, ITER = 0, converged if RR <= TOL2
    RED_SET_TOL = 7,           // BB = v0, TOL2 = aux * v0
    RED_INVSQRT = 8,           // S[slot] = v0, S[slot+1] = 1/sqrt(v0)
    RED_ARNOLDI = 9            // FGMRES column update (vreduce_arnoldi)
};

template <typename T> void vfill(const VecCtx &v, T *y, T val);
template <typename T> void vcopy(const VecCtx &v, const T *x, T *y);
// y = a x + b y, a = sa*S[ia] (ia >= 0) or sa; same for b.
template <typename T> void vaxpby(const VecCtx &v, double a, int ia, const T *x, double b, int ib, T *y);
// z = c d .* r
template <typename T> void vjacobi(const VecCtx &v, double c, int ic, const T *d, const T *r, T *z);
// partial[2 blk] = x.y, partial[2 blk + 1] = x.w (if w)
template <typename T> void vdot(const VecCtx &v, const T *x, const T *y, const T *w, double *partial);
template <typename T>
void vcg_update(const VecCtx &v, T *x, T *r, const T *p, const T *q, T *r_old, double *partial);
template <typename T>
void vmultidot(const VecCtx &v, const T *V, int64_t ld, int nv, const T *w, double *partial, int ncomp);
template <typename T>
// w -= sum_i h_i V_i; dots: partials of V_i . w (i < nv) and w . w (entry
// nv); without dots: w . w (entry 0) when partial is not null; scale_slot >=
// 0: the result is also scaled by that slot (no partials then)
void vorth_update(const VecCtx &v, const T *V, int64_t ld, int nv, const double *H, int hld, T *w, int dots,
                  double *partial, int ncomp, int scale_slot = -1);
template <typename T, typename TX>
void vbasis_update(const VecCtx &v, const T *Z, int64_t ld, const int32_t *kdim, const double *Y, int yld,
                   double scale, int iscale, TX *x);
template <typename TX, typename TY> void vconvert(const VecCtx &v, double sc, int ic, const TX *x, TY *y);
template <typename T> void vadd_scaled(const VecCtx &v, double sc, int ic, const T *d, double *x);
// x = Xn + c1 (Xn - Xp) + c2 (Xp - Xpp), c1 = S[slot1], c2 = S[slot2] per
// instance (Xp read only if a factor is nonzero, Xpp only if c2 is); 0 at
// the constrained nodes of ops when ops is given
void vextrapolate(const VecCtx &v, int slot1, int slot2, const OpDev *ops, const double *Xn, const double *Xp,
                  const double *Xpp, double *x);
// b = (b - y) + S[slot] ld
void vrhs_combine(const VecCtx &v, const double *y, const double *ld, int slot, double *b);
// z = x + y
void vadd(const VecCtx &v, const double *x, const double *y, double *z);
// time-level shift: Xpp = Xp, Xp = Xn, Xn = X1
void vshift(const VecCtx &v, const double *X1, double *Xn, double *Xp, double *Xpp);
template <typename T> void vmask(const VecCtx &v, const OpDev *ops, T *y, T val);

// P32 = (P - P[node 0 of the instance]) + rho_w g z (FP32 heat operator input)
void vpiezo32(const VecCtx &v, const OpDev *ops64, const double *P, float *P32);

struct FlagBlock {
    static constexpr int N = 256;
    int32_t v[N];
};
struct PtrBlock {
    static constexpr int N = 128;
    double *p[N];
    int64_t off[N];
};
// Copy between a batch vector and per-instance device arrays ptrs[i] (which
// hold the entries off[i] .. of the batch vector); hchunks is the host copy
// of the chunk list (ordered by instance).
void vgather_scatter(const Chunk *chunks, const std::vector<Chunk> &hchunks, const std::vector<double *> &ptrs,
                     const std::vector<int64_t> &off, double *batch, bool to_batch, hipStream_t s);
// dst[0 .. n) = flags (host array), in launches of up to 256 values
void vset_flags(const int32_t *flags, int n, int32_t *dst, hipStream_t s);
// hs[0 .. nS) = S, ha[0 .. n) = act, then *seq_ptr = seq; hs, ha and seq_ptr
// are host memory the device can write (pinned, coherent).  Once the host
// reads seq from *seq_ptr, hs and ha hold the values.
void vexport(const double *S, int nS, const int32_t *act, int n, double *hs, int32_t *ha, uint32_t *seq_ptr,
             uint32_t seq, hipStream_t s);
struct SlotBlock {
    static constexpr int N = 64, NS = 4;
    int32_t slot[NS];
    double v[NS][N];
};
// S[i][slots[j]] = vals[j][i] (host arrays) for every instance i < n
void vset_slots(const int *slots, int nslots, const double *const *vals, int n, double *S, hipStream_t s);

void vreduce(const RedCtx &r, const double *partial, int ncomp, int op, int slot, double *S, int32_t *active,
             int maxit, double aux, double *out, hipStream_t s);
// reduction of the second Gram-Schmidt pass (h2 and |w'|^2, ncomp = j + 2)
// followed by the Arnoldi column update of each active instance
void vreduce_arnoldi(const RedCtx &r, const double *partial, int ncomp, double *S, int32_t *active,
                     const ArnArgs &arn, double *out, hipStream_t s);

}  // namespace hts
