// Dirichlet values and time-dependent sources, evaluated on the device at
// t^{n+1} (backward Euler evaluates every time-dependent datum at the new
// time level).
#include "bc.h"
#include "dev_util.h"
#include "vec.h"

namespace hts {

namespace {

__global__ __launch_bounds__(256) void k_dirichlet(const OpDev *__restrict__ ops, const BcDev *__restrict__ bcs,
                                                   const Chunk *__restrict__ chunks, const double *__restrict__ S,
                                                   double *__restrict__ g)
{
    const Chunk ch = chunks[blockIdx.x];
    const OpDev &o = ops[ch.inst];
    const BcDev &b = bcs[ch.inst];
    const double t = S[(int64_t)ch.inst * NSLOT + S_TNEW];
    // at most 4 nodes per thread (the batch's fine chunks): the face and
    // column tests first, coordinates and time functions only on
    // constrained nodes
    static_assert(CHUNK_LEN <= 4 * 256, "k_dirichlet covers 4 nodes per thread");
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int64_t e = ch.beg + threadIdx.x + 256 * u;
        if (e >= ch.end) break;
        // instance-local node index (below 2^31): 32-bit index arithmetic
        const int n = (int)(e - o.off);
        const int nxy = n / o.NX, i = n - nxy * o.NX, k = nxy / o.NY, j = nxy - k * o.NY;
        int fsel = -1;   // the last Dirichlet face through the node
        for (int f = 0; f < b.nface; f++) {
            const int face = b.faces[f];
            const bool on = (face == 0 && i == 0) || (face == 1 && i == o.NX - 1) || (face == 2 && j == 0) ||
                            (face == 3 && j == o.NY - 1) || (face == 4 && k == 0) || (face == 5 && k == o.NZ - 1);
            if (on) fsel = f;
        }
        int csel = -1;   // a Dirichlet column through the node (it takes precedence)
        if (b.colspec && o.dcol) {
            const int64_t c = i + (int64_t)o.NX * j;
            const int packed = o.dcol[c];
            const int lo = packed & 0xFFFF, hi = (packed >> 16) & 0xFFFF;
            const int sp = b.colspec[c];
            if (sp >= 0 && k >= lo && k <= hi) csel = sp;
        }
        double v = 0.0;
        if (fsel >= 0 || csel >= 0) {
            double x = b.xn ? b.xn[i] : b.x0 + i * b.dx, y = b.yn ? b.yn[j] : b.y0 + j * b.dy,
                   z = b.zn ? b.zn[k] : b.z0 + k * b.dz;
            if (b.xyz) {
                x = b.xyz[3 * (int64_t)n];
                y = b.xyz[3 * (int64_t)n + 1];
                z = b.xyz[3 * (int64_t)n + 2];
            }
            v = csel >= 0 ? tf_eval(b.coltf[csel], x, y, z, t) : tf_eval(b.ftf[fsel], x, y, z, t);
        }
        g[e] = v;
    }
}

__device__ __forceinline__ double src_value(const SrcDev &s, const double *S)
{
    const double *Si = S + (int64_t)s.inst * NSLOT;
    double f = tf_eval(s.tf, 0.0, 0.0, 0.0, Si[S_TNEW]);
    if (s.posonly && f < 0.0) f = 0.0;
    return Si[S_FSCALE] * s.scale * f;
}

__global__ void k_sources(const int64_t *__restrict__ rows, const int32_t *__restrict__ rowptr,
                          const SrcEnt *__restrict__ ents, int64_t nrows, const SrcDev *__restrict__ srcs,
                          const double *__restrict__ S, double *__restrict__ y)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    double acc = 0.0;
    for (int e = rowptr[r]; e < rowptr[r + 1]; e++) acc += ents[e].w * src_value(srcs[ents[e].src], S);
    y[rows[r]] += acc;
}

__global__ void k_source_values(const SrcDev *__restrict__ srcs, int n, const double *__restrict__ S,
                                double *__restrict__ coef)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) coef[i] = src_value(srcs[i], S);
}

}  // namespace

void launch_dirichlet_values(const OpDev *ops, const BcDev *bcs, const Chunk *chunks, int nchunk, const double *S,
                             double *g, hipStream_t s)
{
    if (nchunk <= 0) return;
    k_dirichlet<<<dim3(nchunk), dim3(256), 0, s>>>(ops, bcs, chunks, S, g);
    HTS_LAUNCH_CHECK();
}

void launch_sources(const int64_t *rows, const int32_t *rowptr, const SrcEnt *ents, int64_t nrows,
                    const SrcDev *srcs, const double *S, double *y, hipStream_t s)
{
    if (nrows <= 0) return;
    k_sources<<<dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, s>>>(rows, rowptr, ents, nrows, srcs, S, y);
    HTS_LAUNCH_CHECK();
}

void launch_source_values(const SrcDev *srcs, int n, const double *S, double *coef, hipStream_t s)
{
    if (n <= 0) return;
    k_source_values<<<dim3((n + 255) / 256), dim3(256), 0, s>>>(srcs, n, S, coef);
    HTS_LAUNCH_CHECK();
}

}  // namespace hts
