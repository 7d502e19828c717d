// Kernels of the learned preconditioner (nnk.hip): BF16 matrix-core 3x3x3
// convolutions and the elementwise pieces of the encoder-decoder.
#pragma once
#include "common.h"

namespace hts {

struct Dims {
    int x = 1, y = 1, z = 1;
    int64_t n() const { return (int64_t)x * y * z; }
};

// The forward-pass kernels take an optional device flag (gate): when it
// points to 0 every block returns at once, so a captured sequence of
// launches can be switched off from the device.
// y = act(bias + conv(x)) (+ skip); Ybf (BF16, row stride ldy) or Yf (FP32)
void nn_conv_fwd(const uint16_t *X, int cin, Dims din, const uint16_t *W, int kp, const float *bias, int cout,
                 Dims dout, int stride, int relu, const uint16_t *skip, uint16_t *Ybf, float *Yf, int ldy,
                 hipStream_t s, const int32_t *gate = nullptr);
// gx = conv^T(g) with transposed weights Wt [Cin_pad16][ktp]
void nn_conv_bwd_data(const uint16_t *G, int cout, Dims dout, const uint16_t *Wt, int ktp, int cin, Dims din,
                      int stride, float *GX, hipStream_t s);
int64_t nn_bwd_weight_chunks(Dims dout);
// group count of the two-stage partial sums
constexpr int SUM_GROUPS = 32;
// gw [Cout][kp] (+)= sum_o g[o] x[in(o, k)]; partial: (chunks + SUM_GROUPS) *
// cout * kp floats (the chunk partials, then the group sums)
void nn_conv_bwd_weight(const uint16_t *G, int cout, Dims dout, const uint16_t *X, int cin, Dims din, int stride,
                        float *partial, int kp, float *gw, int accumulate, hipStream_t s);
// gb (+)= sum_o g[o]; partial: (ceil(nvox / 512) + SUM_GROUPS) * cout floats
// (within the weight-gradient buffer of the same layer, since kp >= 32)
void nn_bias_grad(const uint16_t *G, int64_t nvox, int cout, float *partial, float *gb, int accumulate, hipStream_t s);
void nn_transpose_w(const uint16_t *W, int cout, int cin, int kp, uint16_t *Wt, int ktp, hipStream_t s);
void nn_upsample(const uint16_t *C, Dims dc, int ch, uint16_t *F, Dims df, hipStream_t s,
                 const int32_t *gate = nullptr);
void nn_upsample_adj(const float *GF, Dims df, int ch, float *GC, Dims dc, hipStream_t s);
void nn_relu_mask(const float *GX, const uint16_t *Y, int64_t n, uint16_t *G, hipStream_t s);
void nn_add_f32(float *a, const float *b, int64_t n, hipStream_t s);
void nn_pack_input(const double *r, double sc, const float *feat, int64_t n, uint16_t *X, hipStream_t s);
void nn_unpack_output(const float *Y, int ldy, double sc, const uint8_t *mask, int64_t n, double *z, hipStream_t s);
int64_t nn_loss_blocks(int64_t n);
void nn_loss(const float *Y, int ldy, const uint16_t *T, const uint8_t *mask, int64_t n, double inv_nfree, float *GY,
             double *partial, hipStream_t s);
void nn_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2, float eps,
             int step, float gscale, uint16_t *wbf, const uint8_t *live, hipStream_t s);
void nn_f32_to_bf16(const float *a, int64_t n, uint16_t *b, hipStream_t s);
void nn_pack_input_bf(const uint16_t *r, const float *feat, int64_t n, uint16_t *X, hipStream_t s);
void nn_pack_input_dev(const double *r, const double *rr, double nfree, const float *feat, int64_t n, uint16_t *X,
                       hipStream_t s, const int32_t *gate = nullptr);
// gamma: device scalar (read when the kernel runs)
void nn_unpack_output_dev(const float *Y, int ldy, const double *rr, double nfree, const double *gamma,
                          const uint8_t *mask, int64_t n, double *z, hipStream_t s, const int32_t *gate = nullptr);
void nn_scale_bf16(uint16_t *a, int64_t n, float c, hipStream_t s);
void nn_add_bf16(const uint16_t *a, const uint16_t *b, int64_t n, uint16_t *c, hipStream_t s,
                 const int32_t *gate = nullptr);

}  // namespace hts
