// Boundary data, time functions and time-dependent sources (bc.hip).
#pragma once
#include "common.h"

namespace hts {

struct TimeFnDev {
    int32_t kind, pad;
    double c0, cx, cy, cz, amp, period, phase;
};

__host__ __device__ inline double tf_wave(const TimeFnDev &f, double t)
{
    if (f.kind == 0) return 0.0;
    const double s = sin(2.0 * 3.14159265358979323846 * t / f.period + f.phase);
    if (f.kind == 1) return s;
    return s >= 0.0 ? 1.0 : -1.0;
}

__host__ __device__ inline double tf_eval(const TimeFnDev &f, double x, double y, double z, double t)
{
    return f.c0 + f.cx * x + f.cy * y + f.cz * z + f.amp * tf_wave(f, t);
}

// Dirichlet data of one field of one instance.
struct BcDev {
    int32_t nface;
    int32_t faces[6];          // Dirichlet faces in the order they were set
    TimeFnDev ftf[6];
    double x0, y0, z0;         // origin
    double dx, dy, dz;         // node spacing (uniform meshes)
    const double *xn, *yn, *zn;   // node coordinates per axis (graded meshes; null = uniform)
    const double *xyz;         // general hexahedra: node coordinates [nnode][3] (null = box)
    const int32_t *colspec;    // [NX*NY] Dirichlet column spec per node column or -1 (null = none)
    const TimeFnDev *coltf;    // column specs
};

// One time-dependent source: value(t) = S[inst][S_FSCALE] * scale * f(t), with f
// replaced by max(f, 0) when posonly; t = S[inst][S_TNEW].
struct SrcDev {
    TimeFnDev tf;
    double scale;
    int32_t posonly;
    int32_t inst;
};

struct SrcEnt {
    int32_t src;               // index into the batch source table
    int32_t pad;
    double w;
};

// g = Dirichlet values at t = S[inst][S_TNEW] on constrained nodes, 0 elsewhere.
void launch_dirichlet_values(const OpDev *ops, const BcDev *bcs, const Chunk *chunks, int nchunk, const double *S,
                             double *g, hipStream_t s);
// y[rows[r]] += sum_e w_e value(src_e) for every source row.
void launch_sources(const int64_t *rows, const int32_t *rowptr, const SrcEnt *ents, int64_t nrows,
                    const SrcDev *srcs, const double *S, double *y, hipStream_t s);
// coef[i] = value(src i) for a list of sources (line mass coefficients).
void launch_source_values(const SrcDev *srcs, int n, const double *S, double *coef, hipStream_t s);

}  // namespace hts
