// Kernels of the learned preconditioner: 3x3x3 convolutions as implicit
// GEMMs on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation), their two backward products, and the elementwise pieces of
// the encoder-decoder (upsampling and its adjoint, ReLU masks, loss, Adam).
//
// Activations are channels-last BF16: x[v][c], v = i + NX (j + NY k).
// Weights are [Cout][Kp] BF16 with K index k = tap * Cin + ci, tap =
// dx + 3 (dy + 3 dz), Kp = 27 Cin rounded up to 32 (zero tail).  A
// convolution of stride s with zero padding 1 maps output voxel o to input
// o s + d - 1 per axis (d = 0, 1, 2).
//
// Matrix-core lane layout (16x16x32 BF16, 64 lanes): lane l holds row l%16 of
// A with K entries 8(l/16) .. 8(l/16)+7, column l%16 of B with the same K
// entries, and rows 4(l/16) .. 4(l/16)+3 of column l%16 of the FP32 result.
#include "nnk.h"

namespace hts {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b)
{
    return __uint_as_float(((uint32_t)b) << 16);
}

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFF) ? 0x40 : 0));
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t *p)
{
    uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x8 zero8()
{
    uint4 v = make_uint4(0, 0, 0, 0);
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ void vox_ijk(int64_t v, const int3 d, int &i, int &j, int &k)
{
    i = (int)(v % d.x);
    j = (int)((v / d.x) % d.y);
    k = (int)(v / ((int64_t)d.x * d.y));
}

// ------------------------------------------------------------ forward
// y[o][co] = act(bias[co] + sum_k W[co][k] x[in(o, k)]) (+ skip[o][co])
template <int NT>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t *__restrict__ X, int cin, int3 din,
                                                  const uint16_t *__restrict__ W, int kp,
                                                  const float *__restrict__ bias, int cout, int3 dout, int stride,
                                                  int relu, const uint16_t *__restrict__ skip,
                                                  uint16_t *__restrict__ Ybf, float *__restrict__ Yf, int ldy,
                                                  const int32_t *gate)
{
    if (gate && !*gate) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t nout = (int64_t)dout.x * dout.y * dout.z;
    const int64_t vbase = ((int64_t)blockIdx.x * 4 + w) * 16;
    const int64_t v = vbase + (lane & 15);
    const int kq = lane >> 4;
    int oi = 0, oj = 0, ok = 0;
    const bool vok = v < nout;
    if (vok) vox_ijk(v, dout, oi, oj, ok);
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int ktot = 27 * cin;
    // unrolled so that the gathers of several K steps are in flight together
#pragma unroll 4
    for (int kc = 0; kc < kp; kc += 32) {
        const int k0 = kc + 8 * kq;
        bf16x8 a = zero8();
        if (vok && k0 < ktot) {
            const int tap = k0 / cin, c0 = k0 - tap * cin;
            const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
            const int ii = oi * stride + dx - 1, jj = oj * stride + dy - 1, kk = ok * stride + dz - 1;
            if (ii >= 0 && ii < din.x && jj >= 0 && jj < din.y && kk >= 0 && kk < din.z)
                a = load8(X + ((int64_t)ii + (int64_t)din.x * (jj + (int64_t)din.y * kk)) * cin + c0);
        }
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const int co = t * 16 + (lane & 15);
            const bf16x8 b = load8(W + (int64_t)co * kp + k0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; t++) {
        const int co = t * 16 + (lane & 15);
        if (co >= cout) continue;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int64_t vo = vbase + 4 * kq + j;
            if (vo >= nout) continue;
            float y = acc[t][j] + bias[co];
            if (relu) y = fmaxf(y, 0.f);
            if (skip) y += bf2f(skip[vo * cout + co]);
            if (Yf) Yf[vo * ldy + co] = y;
            else Ybf[vo * ldy + co] = f2bf(y);
        }
    }
}

// k_conv_fwd for small grids: the four waves of a block share one group of 16
// output voxels and split the K steps (wave w takes steps w, w + 4, ...);
// the four partial products are added in wave order through LDS.
template <int NT>
__global__ __launch_bounds__(256) void k_conv_fwd_splitk(const uint16_t *__restrict__ X, int cin, int3 din,
                                                         const uint16_t *__restrict__ W, int kp,
                                                         const float *__restrict__ bias, int cout, int3 dout,
                                                         int stride, int relu, const uint16_t *__restrict__ skip,
                                                         uint16_t *__restrict__ Ybf, float *__restrict__ Yf, int ldy,
                                                         const int32_t *gate)
{
    if (gate && !*gate) return;
    __shared__ f32x4 part[4][NT][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t nout = (int64_t)dout.x * dout.y * dout.z;
    const int64_t vbase = (int64_t)blockIdx.x * 16;
    const int64_t v = vbase + (lane & 15);
    const int kq = lane >> 4;
    int oi = 0, oj = 0, ok = 0;
    const bool vok = v < nout;
    if (vok) vox_ijk(v, dout, oi, oj, ok);
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int ktot = 27 * cin;
#pragma unroll 2
    for (int kc = 32 * w; kc < kp; kc += 128) {
        const int k0 = kc + 8 * kq;
        bf16x8 a = zero8();
        if (vok && k0 < ktot) {
            const int tap = k0 / cin, c0 = k0 - tap * cin;
            const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
            const int ii = oi * stride + dx - 1, jj = oj * stride + dy - 1, kk = ok * stride + dz - 1;
            if (ii >= 0 && ii < din.x && jj >= 0 && jj < din.y && kk >= 0 && kk < din.z)
                a = load8(X + ((int64_t)ii + (int64_t)din.x * (jj + (int64_t)din.y * kk)) * cin + c0);
        }
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const int co = t * 16 + (lane & 15);
            const bf16x8 b = load8(W + (int64_t)co * kp + k0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; t++) part[w][t][lane] = acc[t];
    __syncthreads();
    if (w != 0) return;
#pragma unroll
    for (int t = 0; t < NT; t++) {
        const f32x4 sum = ((part[0][t][lane] + part[1][t][lane]) + part[2][t][lane]) + part[3][t][lane];
        const int co = t * 16 + (lane & 15);
        if (co >= cout) continue;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int64_t vo = vbase + 4 * kq + j;
            if (vo >= nout) continue;
            float y = sum[j] + bias[co];
            if (relu) y = fmaxf(y, 0.f);
            if (skip) y += bf2f(skip[vo * cout + co]);
            if (Yf) Yf[vo * ldy + co] = y;
            else Ybf[vo * ldy + co] = f2bf(y);
        }
    }
}

// Stride-1 convolution with the input tile in LDS.  A block computes an
// 8 x 8 x 4 tile of output voxels (wave w: tile voxels 64 w .. 64 w + 63,
// x fastest, as four 16-row A fragments); the 10 x 10 x 6 input voxels
// around the tile are staged once with all their channels (voxel stride cs
// bf16 in LDS), and each K step reads its A fragments from there.  Same
// products and FP32 accumulation order as k_conv_fwd (K ascending).
constexpr int CT_X = 8, CT_Y = 8, CT_Z = 4;
constexpr int CH_X = CT_X + 2, CH_Y = CT_Y + 2, CH_Z = CT_Z + 2, CH_V = CH_X * CH_Y * CH_Z;

template <int NT>
__global__ __launch_bounds__(256) void k_conv_fwd_tile(const uint16_t *__restrict__ X, int cin, int3 d,
                                                       const uint16_t *__restrict__ W, int kp,
                                                       const float *__restrict__ bias, int cout, int relu,
                                                       const uint16_t *__restrict__ skip,
                                                       uint16_t *__restrict__ Ybf, float *__restrict__ Yf, int ldy,
                                                       int cs, int flip, const int32_t *gate)
{
    if (gate && !*gate) return;
    extern __shared__ uint4 conv_tile_raw[];
    uint16_t *tile = reinterpret_cast<uint16_t *>(conv_tile_raw);
    const int nbx = (d.x + CT_X - 1) / CT_X, nby = (d.y + CT_Y - 1) / CT_Y;
    const int bx = blockIdx.x % nbx, by = (blockIdx.x / nbx) % nby, bz = blockIdx.x / (nbx * nby);
    const int x0 = bx * CT_X - 1, y0 = by * CT_Y - 1, z0 = bz * CT_Z - 1;   // halo origin
    const int units = cin / 8;
    for (int u = threadIdx.x; u < CH_V * units; u += 256) {
        const int hv = u / units, cu = u - hv * units;
        const int hx = hv % CH_X, hy = (hv / CH_X) % CH_Y, hz = hv / (CH_X * CH_Y);
        const int gx = x0 + hx, gy = y0 + hy, gz = z0 + hz;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (gx >= 0 && gx < d.x && gy >= 0 && gy < d.y && gz >= 0 && gz < d.z)
            val = *reinterpret_cast<const uint4 *>(
                X + ((int64_t)gx + (int64_t)d.x * (gy + (int64_t)d.y * gz)) * cin + cu * 8);
        *reinterpret_cast<uint4 *>(tile + hv * cs + cu * 8) = val;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, kq = lane >> 4, r = lane & 15;
    int abase[4];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const int vt = w * 64 + a * 16 + r;
        const int tx = vt % CT_X, ty = (vt / CT_X) % CT_Y, tz = vt / (CT_X * CT_Y);
        abase[a] = (tz * CH_Y + ty) * CH_X + tx;   // halo index of the (0, 0, 0) neighbour
    }
    f32x4 acc[4][NT];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int t = 0; t < NT; t++) acc[a][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int ktot = 27 * cin;
    int tap = (8 * kq) / cin, c0 = 8 * kq - tap * cin;   // K index 8 kq of the first step
    for (int kc = 0; kc < kp; kc += 32) {
        const int k0 = kc + 8 * kq;
        const bool kin = k0 < ktot;
        // flip: the data gradient of a stride-1 convolution, the same
        // product with every spatial offset mirrored (K index unchanged)
        const int tq = flip ? 26 - tap : tap;
        const int dz = tq / 9, dy = (tq / 3) % 3, dx = tq % 3;
        const int toff = (dz * CH_Y + dy) * CH_X + dx;
        bf16x8 bfr[NT];
#pragma unroll
        for (int t = 0; t < NT; t++) bfr[t] = load8(W + (int64_t)(t * 16 + r) * kp + k0);
        bf16x8 afr[4];
#pragma unroll
        for (int a = 0; a < 4; a++) afr[a] = kin ? load8(tile + (abase[a] + toff) * cs + c0) : zero8();
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int t = 0; t < NT; t++) acc[a][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[a], bfr[t], acc[a][t], 0, 0, 0);
        c0 += 32;
        while (c0 >= cin) {
            c0 -= cin;
            tap++;
        }
    }
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const int co = t * 16 + r;
            if (co >= cout) continue;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int vt = w * 64 + a * 16 + 4 * kq + j;
                const int gx = x0 + 1 + vt % CT_X, gy = y0 + 1 + (vt / CT_X) % CT_Y, gz = z0 + 1 + vt / (CT_X * CT_Y);
                if (gx >= d.x || gy >= d.y || gz >= d.z) continue;
                const int64_t vo = (int64_t)gx + (int64_t)d.x * (gy + (int64_t)d.y * gz);
                float y = acc[a][t][j] + (bias ? bias[co] : 0.f);
                if (relu) y = fmaxf(y, 0.f);
                if (skip) y += bf2f(skip[vo * cout + co]);
                if (Yf) Yf[vo * ldy + co] = y;
                else Ybf[vo * ldy + co] = f2bf(y);
            }
        }
}

// ------------------------------------------------------- backward, data
// gx[i][ci] = sum_{tap, co} W[co][tap][ci] g[o(i, tap)][co], o = (i + 1 - d)/s
// Wt is the transposed weight [Cin][Kt], Kt index = tap * Cout + co.
template <int NT>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const uint16_t *__restrict__ G, int cout, int3 dout,
                                                       const uint16_t *__restrict__ Wt, int ktp, int cin,
                                                       int3 din, int stride, float *__restrict__ GX)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t nin = (int64_t)din.x * din.y * din.z;
    const int64_t vbase = ((int64_t)blockIdx.x * 4 + w) * 16;
    const int64_t v = vbase + (lane & 15);
    const int kq = lane >> 4;
    int ii = 0, ij = 0, ik = 0;
    const bool vok = v < nin;
    if (vok) vox_ijk(v, din, ii, ij, ik);
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int ktot = 27 * cout;
    for (int kc = 0; kc < ktp; kc += 32) {
        const int k0 = kc + 8 * kq;
        bf16x8 a = zero8();
        if (vok && k0 < ktot) {
            const int tap = k0 / cout, c0 = k0 - tap * cout;
            const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
            const int nx = ii + 1 - dx, ny = ij + 1 - dy, nz = ik + 1 - dz;
            bool ok = nx >= 0 && ny >= 0 && nz >= 0 && nx % stride == 0 && ny % stride == 0 && nz % stride == 0;
            const int ox = nx / stride, oy = ny / stride, oz = nz / stride;
            ok = ok && ox < dout.x && oy < dout.y && oz < dout.z;
            if (ok) a = load8(G + ((int64_t)ox + (int64_t)dout.x * (oy + (int64_t)dout.y * oz)) * cout + c0);
        }
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const int ci = t * 16 + (lane & 15);
            const bf16x8 b = load8(Wt + (int64_t)ci * ktp + k0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; t++) {
        const int ci = t * 16 + (lane & 15);
        if (ci >= cin) continue;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int64_t vi = vbase + 4 * kq + j;
            if (vi < nin) GX[vi * cin + ci] = acc[t][j];
        }
    }
}

// ----------------------------------------------------- backward, weights
// partial[chunk][co][k] = sum_{o in chunk} g[o][co] x[in(o, k)], k = tap*Cin+ci.
// One block per (voxel chunk, tap); each wave stages 32 voxels of g and x in
// LDS and multiplies them transposed on the matrix cores.
constexpr int BW_CHUNK = 2048;   // output voxels per block (weight gradient)
constexpr int BB_CHUNK = 512;    // output voxels per block (bias gradient)

template <int MT, int NTC>
__global__ __launch_bounds__(256) void k_conv_bwd_weight(const uint16_t *__restrict__ G, int cout, int3 dout,
                                                         const uint16_t *__restrict__ X, int cin, int3 din,
                                                         int stride, float *__restrict__ partial, int kp)
{
    // the wave reduction reuses the staging space once the loop has ended
    // (its last barrier follows the last fragment reads): 36 KB per block
    __shared__ uint4 bw_smem[2 * 4 * 32 * 72 * 2 / 16];
    typedef uint16_t Stage[32][64 + 8];
    Stage *gs = reinterpret_cast<Stage *>(bw_smem);
    Stage *xs = gs + 4;
    float(*red)[65] = reinterpret_cast<float(*)[65]>(bw_smem);
    static_assert(sizeof(float) * 64 * 65 <= sizeof(uint16_t) * 2 * 4 * 32 * 72, "reduction space");
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // columns beyond cin / cout of the last 16-wide tile stay zero
    if ((cout | cin) & 15) {
        for (int e = threadIdx.x; e < 4 * 32 * 72; e += 256) {
            (&gs[0][0][0])[e] = 0;
            (&xs[0][0][0])[e] = 0;
        }
        __syncthreads();
    }
    // the 27 taps of a chunk are consecutive blocks, so the chunk's g rows
    // and the x neighbourhood are read while still in cache
    const int tap = blockIdx.x;
    const int64_t chunk = blockIdx.y;
    const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
    const int64_t nout = (int64_t)dout.x * dout.y * dout.z;
    const int64_t c0v = chunk * BW_CHUNK;
    f32x4 acc[MT][NTC];
#pragma unroll
    for (int a = 0; a < MT; a++)
#pragma unroll
        for (int b = 0; b < NTC; b++) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int sub = w; sub < BW_CHUNK / 32; sub += 4) {
        const int64_t sv = c0v + sub * 32;
        // stage g rows and x rows of 32 voxels (zero outside)
        for (int e = lane; e < 32 * (cout / 8); e += 64) {
            const int r = e / (cout / 8), q = (e % (cout / 8)) * 8;
            const int64_t o = sv + r;
            uint4 val = make_uint4(0, 0, 0, 0);
            if (o < nout) val = *reinterpret_cast<const uint4 *>(G + o * cout + q);
            *reinterpret_cast<uint4 *>(&gs[w][r][q]) = val;
        }
        for (int e = lane; e < 32 * (cin / 8); e += 64) {
            const int r = e / (cin / 8), q = (e % (cin / 8)) * 8;
            const int64_t o = sv + r;
            uint4 val = make_uint4(0, 0, 0, 0);
            if (o < nout) {
                int oi, oj, ok;
                vox_ijk(o, dout, oi, oj, ok);
                const int ii = oi * stride + dx - 1, jj = oj * stride + dy - 1, kk = ok * stride + dz - 1;
                if (ii >= 0 && ii < din.x && jj >= 0 && jj < din.y && kk >= 0 && kk < din.z)
                    val = *reinterpret_cast<const uint4 *>(
                        X + ((int64_t)ii + (int64_t)din.x * (jj + (int64_t)din.y * kk)) * cin + q);
            }
            *reinterpret_cast<uint4 *>(&xs[w][r][q]) = val;
        }
        __syncthreads();
        const int kq = lane >> 4, rr = lane & 15;
#pragma unroll
        for (int a = 0; a < MT; a++) {
            uint16_t av[8];
#pragma unroll
            for (int j = 0; j < 8; j++) av[j] = gs[w][8 * kq + j][a * 16 + rr];
            const bf16x8 A = __builtin_bit_cast(bf16x8, av);
#pragma unroll
            for (int b = 0; b < NTC; b++) {
                uint16_t bv[8];
#pragma unroll
                for (int j = 0; j < 8; j++) bv[j] = xs[w][8 * kq + j][b * 16 + rr];
                const bf16x8 Bm = __builtin_bit_cast(bf16x8, bv);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bm, acc[a][b], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // reduce the four waves in a fixed order
    const int kq = lane >> 4, cc = lane & 15;
    for (int ww = 0; ww < 4; ww++) {
        if (w == ww) {
#pragma unroll
            for (int a = 0; a < MT; a++)
#pragma unroll
                for (int b = 0; b < NTC; b++)
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const int co = a * 16 + 4 * kq + j, ci = b * 16 + cc;
                        if (ww == 0) red[co][ci] = acc[a][b][j];
                        else red[co][ci] += acc[a][b][j];
                    }
        }
        __syncthreads();
    }
    float *P = partial + chunk * cout * kp;
    for (int e = threadIdx.x; e < cout * cin; e += 256) {
        const int co = e / cin, ci = e % cin;
        P[(int64_t)co * kp + tap * cin + ci] = red[co][ci];
    }
}

// sum the per-chunk partials in chunk order: out[i] (+)= sum_c partial[c][i];
// entries whose index within a row of length ld is >= valid are not
// produced by the partial kernels and read as zero
// In two stages with a fixed grouping (independent of the launch): group g
// of SUM_GROUPS sums chunks [g L, (g + 1) L), L = ceil(nchunk / SUM_GROUPS),
// in chunk order into tmp[g][i]; then the groups are added in order.
__global__ void k_sum_partials_groups(const float *__restrict__ partial, int64_t nchunk, int64_t n, int ld,
                                      int valid, float *__restrict__ tmp)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (i >= n) return;
    const int64_t L = (nchunk + SUM_GROUPS - 1) / SUM_GROUPS;
    const int64_t c0 = g * L, c1 = min(nchunk, c0 + L);
    float s = 0.f;
    if ((int)(i % ld) < valid)
        for (int64_t c = c0; c < c1; c++) s += partial[c * n + i];
    tmp[g * n + i] = s;
}

__global__ void k_sum_partials(const float *__restrict__ tmp, int64_t n, float *__restrict__ out, int accumulate)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int g = 0; g < SUM_GROUPS; g++) s += tmp[g * n + i];
    out[i] = accumulate ? out[i] + s : s;
}

// bias gradient partials: partial[chunk][co] = sum_{v in chunk} g[v][co]
__global__ void k_bias_partial(const uint16_t *__restrict__ G, int64_t nvox, int cout, float *__restrict__ partial)
{
    __shared__ float sh[256];
    const int co = threadIdx.x % 64, r = threadIdx.x / 64;
    const int64_t b0 = (int64_t)blockIdx.x * BB_CHUNK;
    float s = 0.f;
    if (co < cout)
        for (int64_t v = b0 + r; v < b0 + BB_CHUNK && v < nvox; v += 4) s += bf2f(G[v * cout + co]);
    sh[threadIdx.x] = s;
    __syncthreads();
    if (r == 0 && co < cout)
        partial[(int64_t)blockIdx.x * cout + co] = ((sh[co] + sh[64 + co]) + sh[128 + co]) + sh[192 + co];
}

// Wt[ci][tap * Cout + co] = W[co][tap * Cin + ci] for ci < rows (zero where
// ci >= cin or the K index is in the padded tail)
__global__ void k_transpose_w(const uint16_t *__restrict__ W, int cout, int cin, int kp, uint16_t *__restrict__ Wt,
                              int ktp, int rows)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * ktp) return;
    const int ci = (int)(e / ktp), k = (int)(e % ktp);
    uint16_t v = 0;
    if (k < 27 * cout && ci < cin) {
        const int tap = k / cout, co = k % cout;
        v = W[(int64_t)co * kp + tap * cin + ci];
    }
    Wt[e] = v;
}

// ------------------------------------------------------- elementwise
// linear upsampling from the stride-2 grid: coarse o sits on fine 2o
__device__ __forceinline__ int up_parents(int i, int nc, int *p, float *wt)
{
    if ((i & 1) == 0) { p[0] = i >> 1; wt[0] = 1.f; return 1; }
    const int a = i >> 1, b = (i + 1) >> 1;
    if (b >= nc) { p[0] = a; wt[0] = 1.f; return 1; }
    p[0] = a; p[1] = b; wt[0] = wt[1] = 0.5f;
    return 2;
}

__global__ void k_upsample(const uint16_t *__restrict__ C, int3 dc, int ch, uint16_t *__restrict__ F, int3 df,
                           const int32_t *gate)
{
    if (gate && !*gate) return;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nf = (int64_t)df.x * df.y * df.z;
    if (e >= nf * ch) return;
    const int64_t v = e / ch;
    const int c = (int)(e % ch);
    int i, j, k;
    vox_ijk(v, df, i, j, k);
    int px[2], py[2], pz[2];
    float wx[2], wy[2], wz[2];
    const int nx = up_parents(i, dc.x, px, wx), ny = up_parents(j, dc.y, py, wy), nz = up_parents(k, dc.z, pz, wz);
    float s = 0.f;
    for (int c2 = 0; c2 < nz; c2++)
        for (int b = 0; b < ny; b++)
            for (int a = 0; a < nx; a++)
                s += wx[a] * wy[b] * wz[c2] *
                     bf2f(C[((int64_t)px[a] + (int64_t)dc.x * (py[b] + (int64_t)dc.y * pz[c2])) * ch + c]);
    F[e] = f2bf(s);
}

// k_upsample for ch a multiple of 8: one thread per fine voxel and group of
// 8 channels (16-byte loads and stores), parents summed in the same order
__global__ void k_upsample8(const uint16_t *__restrict__ C, int3 dc, int ch, uint16_t *__restrict__ F, int3 df,
                            const int32_t *gate)
{
    if (gate && !*gate) return;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nf = (int64_t)df.x * df.y * df.z;
    const int groups = ch / 8;
    if (e >= nf * groups) return;
    const int64_t v = e / groups;
    const int c0 = (int)(e - v * groups) * 8;
    int i, j, k;
    vox_ijk(v, df, i, j, k);
    int px[2], py[2], pz[2];
    float wx[2], wy[2], wz[2];
    const int nx = up_parents(i, dc.x, px, wx), ny = up_parents(j, dc.y, py, wy), nz = up_parents(k, dc.z, pz, wz);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int c2 = 0; c2 < nz; c2++)
        for (int b = 0; b < ny; b++)
            for (int a = 0; a < nx; a++) {
                const float w = wx[a] * wy[b] * wz[c2];
                const uint4 q = *reinterpret_cast<const uint4 *>(
                    C + ((int64_t)px[a] + (int64_t)dc.x * (py[b] + (int64_t)dc.y * pz[c2])) * ch + c0);
                const uint32_t u[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                for (int h = 0; h < 4; h++) {
                    s[2 * h] += w * bf2f((uint16_t)(u[h] & 0xFFFFu));
                    s[2 * h + 1] += w * bf2f((uint16_t)(u[h] >> 16));
                }
            }
    uint32_t o[4];
#pragma unroll
    for (int h = 0; h < 4; h++) o[h] = (uint32_t)f2bf(s[2 * h]) | ((uint32_t)f2bf(s[2 * h + 1]) << 16);
    *reinterpret_cast<uint4 *>(F + v * ch + c0) = make_uint4(o[0], o[1], o[2], o[3]);
}

// adjoint of k_upsample: gc[o] = sum_i w(i, o) gf[i]
__global__ void k_upsample_adj(const float *__restrict__ GF, int3 df, int ch, float *__restrict__ GC, int3 dc)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nc = (int64_t)dc.x * dc.y * dc.z;
    if (e >= nc * ch) return;
    const int64_t v = e / ch;
    const int c = (int)(e % ch);
    int I, J, K;
    vox_ijk(v, dc, I, J, K);
    float s = 0.f;
    for (int dz = -1; dz <= 1; dz++) {
        const int k = 2 * K + dz;
        if (k < 0 || k >= df.z) continue;
        int pz[2]; float wz[2];
        const int nz = up_parents(k, dc.z, pz, wz);
        float az = 0.f;
        for (int q = 0; q < nz; q++) if (pz[q] == K) az = wz[q];
        if (az == 0.f) continue;
        for (int dy = -1; dy <= 1; dy++) {
            const int j = 2 * J + dy;
            if (j < 0 || j >= df.y) continue;
            int py[2]; float wy[2];
            const int ny = up_parents(j, dc.y, py, wy);
            float ay = 0.f;
            for (int q = 0; q < ny; q++) if (py[q] == J) ay = wy[q];
            if (ay == 0.f) continue;
            for (int dx = -1; dx <= 1; dx++) {
                const int i = 2 * I + dx;
                if (i < 0 || i >= df.x) continue;
                int px[2]; float wx[2];
                const int nx = up_parents(i, dc.x, px, wx);
                float ax = 0.f;
                for (int q = 0; q < nx; q++) if (px[q] == I) ax = wx[q];
                if (ax == 0.f) continue;
                s += ax * ay * az * GF[((int64_t)i + (int64_t)df.x * (j + (int64_t)df.y * k)) * ch + c];
            }
        }
    }
    GC[e] = s;
}

// g_bf16 = bf16(gx * (y > 0)) (mask off when y == null); optionally gx += add
__global__ void k_relu_mask(const float *__restrict__ GX, const uint16_t *__restrict__ Y, int64_t n,
                            uint16_t *__restrict__ G)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n) return;
    float g = GX[e];
    if (Y && !(bf2f(Y[e]) > 0.f)) g = 0.f;
    G[e] = f2bf(g);
}

__global__ void k_add_f32(float *__restrict__ a, const float *__restrict__ b, int64_t n)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) a[e] += b[e];
}

// network input: channel 0 = r * sc, channel 1 = feature, channels 2..7 = 0
__global__ void k_pack_input(const double *__restrict__ r, double sc, const float *__restrict__ feat, int64_t n,
                             uint16_t *__restrict__ X)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= n) return;
    uint16_t o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    o[0] = f2bf((float)(r[v] * sc));
    o[1] = f2bf(feat[v]);
    *reinterpret_cast<uint4 *>(X + v * 8) = __builtin_bit_cast(uint4, o);
}

// z = sc * out[v][0], zeroed where mask
__global__ void k_unpack_output(const float *__restrict__ Y, int ldy, double sc, const uint8_t *__restrict__ mask,
                                int64_t n, double *__restrict__ z)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= n) return;
    double val = sc * (double)Y[v * ldy];
    if (mask && mask[v]) val = 0.0;
    z[v] = val;
}

// squared error over free nodes: per-block partial of sum (y - t)^2; grad
// gy[v][0] = 2 (y - t) / nfree, other channels 0
__global__ void k_loss(const float *__restrict__ Y, int ldy, const uint16_t *__restrict__ T,
                       const uint8_t *__restrict__ mask, int64_t n, double inv_nfree, float *__restrict__ GY,
                       double *__restrict__ partial)
{
    __shared__ double sh[256];
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double s = 0.0;
    if (v < n) {
        const bool m = mask && mask[v];
        const double d = m ? 0.0 : (double)Y[v * ldy] - (double)bf2f(T[v]);
        s = d * d;
        for (int c = 0; c < ldy; c++) GY[v * ldy + c] = c == 0 ? (float)(2.0 * d * inv_nfree) : 0.f;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2, float gscale, uint16_t *__restrict__ wbf, const uint8_t *__restrict__ live)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (live && !live[i]) {
        if (wbf) wbf[i] = 0;
        return;
    }
    const float gi = g[i] * gscale;
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    if (wbf) wbf[i] = f2bf(wi);
}

__global__ void k_f32_to_bf16(const float *__restrict__ a, int64_t n, uint16_t *__restrict__ b)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = f2bf(a[i]);
}

// network input from a stored pair: channel 0 = r (BF16), channel 1 = feature
__global__ void k_pack_input_bf(const uint16_t *__restrict__ r, const float *__restrict__ feat, int64_t n,
                                uint16_t *__restrict__ X)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= n) return;
    uint16_t o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    o[0] = r[v];
    o[1] = f2bf(feat[v]);
    *reinterpret_cast<uint4 *>(X + v * 8) = __builtin_bit_cast(uint4, o);
}

// network input in a solve: channel 0 = r / rms(r) with rms(r)^2 = rr / nfree
// read from device memory
__global__ void k_pack_input_dev(const double *__restrict__ r, const double *__restrict__ rr, double nfree,
                                 const float *__restrict__ feat, int64_t n, uint16_t *__restrict__ X,
                                 const int32_t *gate)
{
    if (gate && !*gate) return;
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= n) return;
    const double q = *rr;
    const double sc = q > 0.0 ? sqrt(nfree / q) : 0.0;
    uint16_t o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    o[0] = f2bf((float)(r[v] * sc));
    o[1] = f2bf(feat[v]);
    *reinterpret_cast<uint4 *>(X + v * 8) = __builtin_bit_cast(uint4, o);
}

// z = gamma rms(r) out[v][0], zero where mask
__global__ void k_unpack_output_dev(const float *__restrict__ Y, int ldy, const double *__restrict__ rr,
                                    double nfree, const double *__restrict__ gamma_p,
                                    const uint8_t *__restrict__ mask, int64_t n, double *__restrict__ z,
                                    const int32_t *gate)
{
    if (gate && !*gate) return;
    const double gamma = *gamma_p;
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= n) return;
    const double q = *rr;
    const double sc = q > 0.0 ? sqrt(q / nfree) : 0.0;
    double val = gamma * sc * (double)Y[v * ldy];
    if (mask && mask[v]) val = 0.0;
    z[v] = val;
}

// c = bf16(a + b), 8 entries per thread (n a multiple of 8)
__global__ void k_add_bf16x8(const uint16_t *__restrict__ a, const uint16_t *__restrict__ b, int64_t n8,
                             uint16_t *__restrict__ c, const int32_t *gate)
{
    if (gate && !*gate) return;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n8) return;
    const uint4 qa = reinterpret_cast<const uint4 *>(a)[e], qb = reinterpret_cast<const uint4 *>(b)[e];
    const uint32_t ua[4] = {qa.x, qa.y, qa.z, qa.w}, ub[4] = {qb.x, qb.y, qb.z, qb.w};
    uint32_t o[4];
#pragma unroll
    for (int h = 0; h < 4; h++) {
        const uint16_t lo = f2bf(bf2f((uint16_t)(ua[h] & 0xFFFFu)) + bf2f((uint16_t)(ub[h] & 0xFFFFu)));
        const uint16_t hi = f2bf(bf2f((uint16_t)(ua[h] >> 16)) + bf2f((uint16_t)(ub[h] >> 16)));
        o[h] = (uint32_t)lo | ((uint32_t)hi << 16);
    }
    reinterpret_cast<uint4 *>(c)[e] = make_uint4(o[0], o[1], o[2], o[3]);
}

// c = bf16(a + b)
__global__ void k_add_bf16(const uint16_t *__restrict__ a, const uint16_t *__restrict__ b, int64_t n,
                           uint16_t *__restrict__ c, const int32_t *gate)
{
    if (gate && !*gate) return;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) c[e] = f2bf(bf2f(a[e]) + bf2f(b[e]));
}

// a = bf16(a * c)
__global__ void k_scale_bf16(uint16_t *__restrict__ a, int64_t n, float c)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) a[e] = f2bf(bf2f(a[e]) * c);
}

inline dim3 g256(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

// ------------------------------------------------------------- launchers
void nn_conv_fwd(const uint16_t *X, int cin, Dims din, const uint16_t *W, int kp, const float *bias, int cout,
                 Dims dout, int stride, int relu, const uint16_t *skip, uint16_t *Ybf, float *Yf, int ldy,
                 hipStream_t s, const int32_t *gate)
{
    const int64_t nout = dout.n();
    const dim3 g((unsigned)((nout + 63) / 64)), b(256);
    const int3 di{din.x, din.y, din.z}, dn{dout.x, dout.y, dout.z};
    const int nt = (cout + 15) / 16;
    if (nout < 32768) {
        // small grids (fewer than 2048 groups of 16 voxels): split K over the
        // four waves of a block
        const dim3 gs((unsigned)((nout + 15) / 16));
        switch (nt) {
        case 1: k_conv_fwd_splitk<1><<<gs, b, 0, s>>>(X, cin, di, W, kp, bias, cout, dn, stride, relu, skip, Ybf, Yf, ldy, gate); break;
        case 2: k_conv_fwd_splitk<2><<<gs, b, 0, s>>>(X, cin, di, W, kp, bias, cout, dn, stride, relu, skip, Ybf, Yf, ldy, gate); break;
        case 3: k_conv_fwd_splitk<3><<<gs, b, 0, s>>>(X, cin, di, W, kp, bias, cout, dn, stride, relu, skip, Ybf, Yf, ldy, gate); break;
        case 4: k_conv_fwd_splitk<4><<<gs, b, 0, s>>>(X, cin, di, W, kp, bias, cout, dn, stride, relu, skip, Ybf, Yf, ldy, gate); break;
        default: throw Error(-7, "at most 64 output channels");
        }
        HTS_LAUNCH_CHECK();
        return;
    }
    // stride 1: the LDS-tiled kernel when the halo tile fits 64 KB (voxel
    // stride padded by 8 channels where that still fits, which spreads the
    // 16 rows of a fragment over distinct banks)
    if (stride == 1 && din.x == dout.x && din.y == dout.y && din.z == dout.z && cin % 8 == 0 && nt <= 4) {
        int cs = cin + 8;
        if ((int64_t)CH_V * cs * 2 > 65536) cs = cin;
        if ((int64_t)CH_V * cs * 2 <= 65536) {
            const int64_t nb = (int64_t)((din.x + CT_X - 1) / CT_X) * ((din.y + CT_Y - 1) / CT_Y) *
                               ((din.z + CT_Z - 1) / CT_Z);
            const dim3 gt((unsigned)nb);
            const size_t lds = (size_t)CH_V * cs * 2;
            switch (nt) {
            case 1: k_conv_fwd_tile<1><<<gt, b, lds, s>>>(X, cin, di, W, kp, bias, cout, relu, skip, Ybf, Yf, ldy, cs, 0, gate); break;
            case 2: k_conv_fwd_tile<2><<<gt, b, lds, s>>>(X, cin, di, W, kp, bias, cout, relu, skip, Ybf, Yf, ldy, cs, 0, gate); break;
            case 3: k_conv_fwd_tile<3><<<gt, b, lds, s>>>(X, cin, di, W, kp, bias, cout, relu, skip, Ybf, Yf, ldy, cs, 0, gate); break;
            default: k_conv_fwd_tile<4><<<gt, b, lds, s>>>(X, cin, di, W, kp, bias, cout, relu, skip, Ybf, Yf, ldy, cs, 0, gate); break;
            }
            HTS_LAUNCH_CHECK();
            return;
        }
    }
    switch (nt) {
    case 1: k_conv_fwd<1><<<g, b, 0, s>>>(X, cin, di, W, kp, bias, cout, dn, stride, relu, skip, Ybf, Yf, ldy, gate); break;
    case 2: k_conv_fwd<2><<<g, b, 0, s>>>(X, cin, di, W, kp, bias, cout, dn, stride, relu, skip, Ybf, Yf, ldy, gate); break;
    case 3: k_conv_fwd<3><<<g, b, 0, s>>>(X, cin, di, W, kp, bias, cout, dn, stride, relu, skip, Ybf, Yf, ldy, gate); break;
    case 4: k_conv_fwd<4><<<g, b, 0, s>>>(X, cin, di, W, kp, bias, cout, dn, stride, relu, skip, Ybf, Yf, ldy, gate); break;
    default: throw Error(-7, "at most 64 output channels");
    }
    HTS_LAUNCH_CHECK();
}

void nn_conv_bwd_data(const uint16_t *G, int cout, Dims dout, const uint16_t *Wt, int ktp, int cin, Dims din,
                      int stride, float *GX, hipStream_t s)
{
    const int64_t nin = din.n();
    const dim3 g((unsigned)((nin + 63) / 64)), b(256);
    const int3 di{din.x, din.y, din.z}, dn{dout.x, dout.y, dout.z};
    const int nt = (cin + 15) / 16;
    // stride 1 on large grids: the LDS-tiled forward kernel over g with the
    // transposed weights and mirrored offsets
    if (stride == 1 && nin >= 32768 && din.x == dout.x && din.y == dout.y && din.z == dout.z && cout % 8 == 0 &&
        nt <= 4) {
        int cs = cout + 8;
        if ((int64_t)CH_V * cs * 2 > 65536) cs = cout;
        if ((int64_t)CH_V * cs * 2 <= 65536) {
            const int64_t nb = (int64_t)((din.x + CT_X - 1) / CT_X) * ((din.y + CT_Y - 1) / CT_Y) *
                               ((din.z + CT_Z - 1) / CT_Z);
            const dim3 gt((unsigned)nb);
            const size_t lds = (size_t)CH_V * cs * 2;
            switch (nt) {
            case 1: k_conv_fwd_tile<1><<<gt, b, lds, s>>>(G, cout, di, Wt, ktp, nullptr, cin, 0, nullptr, nullptr, GX, cin, cs, 1, nullptr); break;
            case 2: k_conv_fwd_tile<2><<<gt, b, lds, s>>>(G, cout, di, Wt, ktp, nullptr, cin, 0, nullptr, nullptr, GX, cin, cs, 1, nullptr); break;
            case 3: k_conv_fwd_tile<3><<<gt, b, lds, s>>>(G, cout, di, Wt, ktp, nullptr, cin, 0, nullptr, nullptr, GX, cin, cs, 1, nullptr); break;
            default: k_conv_fwd_tile<4><<<gt, b, lds, s>>>(G, cout, di, Wt, ktp, nullptr, cin, 0, nullptr, nullptr, GX, cin, cs, 1, nullptr); break;
            }
            HTS_LAUNCH_CHECK();
            return;
        }
    }
    switch (nt) {
    case 1: k_conv_bwd_data<1><<<g, b, 0, s>>>(G, cout, dn, Wt, ktp, cin, di, stride, GX); break;
    case 2: k_conv_bwd_data<2><<<g, b, 0, s>>>(G, cout, dn, Wt, ktp, cin, di, stride, GX); break;
    case 3: k_conv_bwd_data<3><<<g, b, 0, s>>>(G, cout, dn, Wt, ktp, cin, di, stride, GX); break;
    case 4: k_conv_bwd_data<4><<<g, b, 0, s>>>(G, cout, dn, Wt, ktp, cin, di, stride, GX); break;
    default: throw Error(-7, "at most 64 input channels");
    }
    HTS_LAUNCH_CHECK();
}

int64_t nn_bwd_weight_chunks(Dims dout) { return (dout.n() + BW_CHUNK - 1) / BW_CHUNK; }

// out (+)= sum over the nchunk partials [c][n]; the group sums go to
// partial + nchunk n (the buffer holds (nchunk + SUM_GROUPS) n floats)
static void sum_partials(float *partial, int64_t nch, int64_t n, int ld, int valid, float *out, int accumulate,
                         hipStream_t s)
{
    float *tmp = partial + nch * n;
    k_sum_partials_groups<<<dim3((unsigned)((n + 255) / 256), SUM_GROUPS), dim3(256), 0, s>>>(partial, nch, n, ld,
                                                                                             valid, tmp);
    HTS_LAUNCH_CHECK();
    k_sum_partials<<<g256(n), dim3(256), 0, s>>>(tmp, n, out, accumulate);
    HTS_LAUNCH_CHECK();
}

template <int MT>
static void bw_dispatch(int ntc, dim3 g, hipStream_t s, const uint16_t *G, int cout, int3 dn, const uint16_t *X,
                        int cin, int3 di, int stride, float *partial, int kp)
{
    switch (ntc) {
    case 1: k_conv_bwd_weight<MT, 1><<<g, dim3(256), 0, s>>>(G, cout, dn, X, cin, di, stride, partial, kp); break;
    case 2: k_conv_bwd_weight<MT, 2><<<g, dim3(256), 0, s>>>(G, cout, dn, X, cin, di, stride, partial, kp); break;
    case 3: k_conv_bwd_weight<MT, 3><<<g, dim3(256), 0, s>>>(G, cout, dn, X, cin, di, stride, partial, kp); break;
    case 4: k_conv_bwd_weight<MT, 4><<<g, dim3(256), 0, s>>>(G, cout, dn, X, cin, di, stride, partial, kp); break;
    default: throw Error(-7, "at most 64 input channels");
    }
}

void nn_conv_bwd_weight(const uint16_t *G, int cout, Dims dout, const uint16_t *X, int cin, Dims din, int stride,
                        float *partial, int kp, float *gw, int accumulate, hipStream_t s)
{
    if (cout % 8 != 0 || cin % 8 != 0 || cout > 64 || cin > 64)
        throw Error(-7, "weight gradient needs channel counts that are multiples of 8 up to 64");
    const int64_t nch = nn_bwd_weight_chunks(dout);
    if (nch > 65535) throw Error(-7, "weight gradient: more than 65535 chunks of 512 voxels");
    const dim3 g(27, (unsigned)nch);
    const int3 di{din.x, din.y, din.z}, dn{dout.x, dout.y, dout.z};
    const int ntc = (cin + 15) / 16;
    switch ((cout + 15) / 16) {
    case 1: bw_dispatch<1>(ntc, g, s, G, cout, dn, X, cin, di, stride, partial, kp); break;
    case 2: bw_dispatch<2>(ntc, g, s, G, cout, dn, X, cin, di, stride, partial, kp); break;
    case 3: bw_dispatch<3>(ntc, g, s, G, cout, dn, X, cin, di, stride, partial, kp); break;
    case 4: bw_dispatch<4>(ntc, g, s, G, cout, dn, X, cin, di, stride, partial, kp); break;
    default: throw Error(-7, "at most 64 output channels");
    }
    HTS_LAUNCH_CHECK();
    const int64_t n = (int64_t)cout * kp;
    sum_partials(partial, nch, n, kp, 27 * cin, gw, accumulate, s);
}

void nn_bias_grad(const uint16_t *G, int64_t nvox, int cout, float *partial, float *gb, int accumulate, hipStream_t s)
{
    const int64_t nch = (nvox + BB_CHUNK - 1) / BB_CHUNK;
    k_bias_partial<<<dim3((unsigned)nch), dim3(256), 0, s>>>(G, nvox, cout, partial);
    HTS_LAUNCH_CHECK();
    sum_partials(partial, nch, cout, cout, cout, gb, accumulate, s);
}

void nn_transpose_w(const uint16_t *W, int cout, int cin, int kp, uint16_t *Wt, int ktp, hipStream_t s)
{
    const int rows = (cin + 15) / 16 * 16;
    k_transpose_w<<<g256((int64_t)rows * ktp), dim3(256), 0, s>>>(W, cout, cin, kp, Wt, ktp, rows);
    HTS_LAUNCH_CHECK();
}

static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

void nn_upsample(const uint16_t *C, Dims dc, int ch, uint16_t *F, Dims df, hipStream_t s, const int32_t *gate)
{
    if (ch % 8 == 0 && aligned16(C) && aligned16(F))
        k_upsample8<<<g256(df.n() * (ch / 8)), dim3(256), 0, s>>>(C, int3{dc.x, dc.y, dc.z}, ch, F,
                                                                   int3{df.x, df.y, df.z}, gate);
    else
        k_upsample<<<g256(df.n() * ch), dim3(256), 0, s>>>(C, int3{dc.x, dc.y, dc.z}, ch, F, int3{df.x, df.y, df.z},
                                                           gate);
    HTS_LAUNCH_CHECK();
}

void nn_upsample_adj(const float *GF, Dims df, int ch, float *GC, Dims dc, hipStream_t s)
{
    k_upsample_adj<<<g256(dc.n() * ch), dim3(256), 0, s>>>(GF, int3{df.x, df.y, df.z}, ch, GC,
                                                           int3{dc.x, dc.y, dc.z});
    HTS_LAUNCH_CHECK();
}

void nn_relu_mask(const float *GX, const uint16_t *Y, int64_t n, uint16_t *G, hipStream_t s)
{
    k_relu_mask<<<g256(n), dim3(256), 0, s>>>(GX, Y, n, G);
    HTS_LAUNCH_CHECK();
}

void nn_add_f32(float *a, const float *b, int64_t n, hipStream_t s)
{
    k_add_f32<<<g256(n), dim3(256), 0, s>>>(a, b, n);
    HTS_LAUNCH_CHECK();
}

void nn_pack_input(const double *r, double sc, const float *feat, int64_t n, uint16_t *X, hipStream_t s)
{
    k_pack_input<<<g256(n), dim3(256), 0, s>>>(r, sc, feat, n, X);
    HTS_LAUNCH_CHECK();
}

void nn_unpack_output(const float *Y, int ldy, double sc, const uint8_t *mask, int64_t n, double *z, hipStream_t s)
{
    k_unpack_output<<<g256(n), dim3(256), 0, s>>>(Y, ldy, sc, mask, n, z);
    HTS_LAUNCH_CHECK();
}

int64_t nn_loss_blocks(int64_t n) { return (n + 255) / 256; }

void nn_loss(const float *Y, int ldy, const uint16_t *T, const uint8_t *mask, int64_t n, double inv_nfree, float *GY,
             double *partial, hipStream_t s)
{
    k_loss<<<g256(n), dim3(256), 0, s>>>(Y, ldy, T, mask, n, inv_nfree, GY, partial);
    HTS_LAUNCH_CHECK();
}

void nn_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2, float eps,
             int step, float gscale, uint16_t *wbf, const uint8_t *live, hipStream_t s)
{
    const float c1 = 1.f / (1.f - powf(b1, (float)step)), c2 = 1.f / (1.f - powf(b2, (float)step));
    k_adam<<<g256(n), dim3(256), 0, s>>>(w, m, v, g, n, lr, b1, b2, eps, c1, c2, gscale, wbf, live);
    HTS_LAUNCH_CHECK();
}

void nn_pack_input_bf(const uint16_t *r, const float *feat, int64_t n, uint16_t *X, hipStream_t s)
{
    k_pack_input_bf<<<g256(n), dim3(256), 0, s>>>(r, feat, n, X);
    HTS_LAUNCH_CHECK();
}

void nn_pack_input_dev(const double *r, const double *rr, double nfree, const float *feat, int64_t n, uint16_t *X,
                       hipStream_t s, const int32_t *gate)
{
    k_pack_input_dev<<<g256(n), dim3(256), 0, s>>>(r, rr, nfree, feat, n, X, gate);
    HTS_LAUNCH_CHECK();
}

void nn_unpack_output_dev(const float *Y, int ldy, const double *rr, double nfree, const double *gamma,
                          const uint8_t *mask, int64_t n, double *z, hipStream_t s, const int32_t *gate)
{
    k_unpack_output_dev<<<g256(n), dim3(256), 0, s>>>(Y, ldy, rr, nfree, gamma, mask, n, z, gate);
    HTS_LAUNCH_CHECK();
}

void nn_add_bf16(const uint16_t *a, const uint16_t *b, int64_t n, uint16_t *c, hipStream_t s, const int32_t *gate)
{
    if (n % 8 == 0 && aligned16(a) && aligned16(b) && aligned16(c))
        k_add_bf16x8<<<g256(n / 8), dim3(256), 0, s>>>(a, b, n / 8, c, gate);
    else
        k_add_bf16<<<g256(n), dim3(256), 0, s>>>(a, b, n, c, gate);
    HTS_LAUNCH_CHECK();
}

void nn_scale_bf16(uint16_t *a, int64_t n, float c, hipStream_t s)
{
    k_scale_bf16<<<g256(n), dim3(256), 0, s>>>(a, n, c);
    HTS_LAUNCH_CHECK();
}

void nn_f32_to_bf16(const float *a, int64_t n, uint16_t *b, hipStream_t s)
{
    k_f32_to_bf16<<<g256(n), dim3(256), 0, s>>>(a, n, b);
    HTS_LAUNCH_CHECK();
}

}  // namespace hts
