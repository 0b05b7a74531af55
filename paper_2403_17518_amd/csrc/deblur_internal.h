// Internal declarations of the deblurring network (deblur_kernels.hip,
// deblur_api.hip). Activations and gradients are NHWC bf16 (batch 1), with a
// channel stride and offset so that concatenated tensors are slices of one
// buffer; parameters are FP32 masters with a bf16 copy for the MFMA kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dbl {

using bf16 = __bf16;

// Source-pixel map of an implicit-GEMM operand: output pixel p = (i, j) of an
// H x W grid and tap t read source pixel (i*stride + t/tapw + d0,
// j*stride + t%tapw + d0) of an Hs x Ws grid, channels [coff, coff + Cb) of
// a tensor with channel stride ld; outside the source grid the value is 0.
//   3x3 conv (pad 1): stride 1, tapw 3, d0 -1, ntaps 9
//   2x2 up-sampling taps (transposed-conv gradient): stride 2, tapw 2, d0 0
//   identity: stride 1, tapw 1, d0 0, ntaps 1
struct Gather {
    const bf16 *src;
    int32_t ld, coff, Cb;
    int32_t Hs, Ws;
    int32_t H, W;
    int32_t stride, tapw, d0, ntaps;
};

// C[m][p] = sum_k A[m][k] * B[k][p] with A row-major [M][K] (K = ntaps*Cb,
// k = tap*Cb + c) and B gathered from g. Epilogue: + bias[co], activation
// (slope for x < 0; act = 0 means none), bf16 store to out[pix][coff + co].
// scatter 0: pix = p, co = m. scatter 1 (2x2 stride-2 transposed conv):
// m = ab*Cout + co, pix = (2i + ab/2, 2j + ab%2) of the Ho x Wo grid.
struct GemmArgs {
    int32_t M, N, K;
    const bf16 *A;
    int32_t lda;
    Gather g;
    bf16 *out;
    int32_t out_ld, out_coff, Cout, scatter, Ho, Wo;
    const float *bias;
    int32_t act;
    float slope;
    // activation derivative folded into the epilogue (data gradients): the
    // result is scaled by (y > 0 ? 1 : slope) with y = act_y[pix*act_ld +
    // act_coff + co], the activated output of the layer below
    const bf16 *act_y;
    int32_t act_ld, act_coff;
    // set by gemm(): channel offsets and strides allow 8-byte stores of 4
    // consecutive output channels
    int32_t out_vec;
    // split-K scratch (FP32, kpart_cap floats; null: no split): layers with
    // few output tiles split K over workgroups and a second pass sums the
    // parts in order and applies the epilogue
    float *kpart;
    int64_t kpart_cap;
};
constexpr int64_t kGemmSplitFloats = 480 * 128 * 128;   // split-K scratch per network

// C[m][n] = sum_p A[p][acoff + m] * Bg(p, n), n = tap*Cb + c, reduced over the
// pixels p of the gather grid in nsplit chunks: partial[z][m][n] (FP32), then
// out[m*ldm + n*ldn] = sum_z partial[z][m][n].
struct WgradArgs {
    int32_t M, N;
    const bf16 *A;
    int32_t lda, acoff;
    Gather g;
    int32_t nsplit, chunk;  // pixels per split, multiple of 64
    int32_t bm, bn;         // output tile of the kernel: 128x128, 64x128, 32x128 or 64x64
    float *partial;         // [nsplit][M][N] when nsplit > 1
    float *out;
    int32_t ldm, ldn;
    // optional bias gradient into bias_out: bias_from_b = 0, sum_p A[p][acoff
    // + m] (partials [nsplit][M]); bias_from_b = 1, sum_p sum_tap Bg(p, tap*Cb
    // + c) (partials [nsplit][N]), the bias of a transposed convolution
    float *bias_partial;
    float *bias_out;
    int32_t bias_from_b;
    int32_t fin_groups;     // deferred second pass: split groups per output (wgrad_finish_groups)
};

hipError_t gemm(const GemmArgs &a, hipStream_t s);
// the input layer (one input channel): direct 3x3 convolution and its
// weight/bias gradients (part: scratch of part_floats floats)
hipError_t conv1_fwd(const bf16 *x, int32_t H, int32_t W, const bf16 *w, const float *b, int32_t C, int32_t act,
                     float slope, bf16 *out, int32_t ld, int32_t coff, hipStream_t s);
hipError_t conv1_wgrad(const bf16 *dz, int32_t ld, int32_t zoff, const bf16 *x, int32_t H, int32_t W, int32_t C,
                       float *part, int64_t part_floats, float *dw, float *db, hipStream_t s);
// defer_finish: the second pass of a vectorised weight gradient is left to
// wgrad_finish_all (its outputs count wgrad_finish_count(a)); the generic
// path always finishes itself (count 0)
hipError_t wgrad(const WgradArgs &a, hipStream_t s, bool defer_finish = false);
int64_t wgrad_finish_count(const WgradArgs &a);
// split groups of a deferred second pass (1, 2, 4 or 8); its finish blocks
// cover kFinishOutputs / groups outputs each
int wgrad_finish_groups(const WgradArgs &a);
// the deferred second passes of n weight gradients (device table tab; entry
// l owns blocks bbeg[l] .. bbeg[l+1]-1, nblk = bbeg[n])
constexpr int kFinishOutputs = 1024;
hipError_t wgrad_finish_all(const WgradArgs *tab, const int64_t *bbeg, int32_t n, int64_t nblk, hipStream_t s);
// bias gradient: db[c] = sum_p dz[p][coff + c]; scratch holds nsplit * C floats
hipError_t bias_grad(const bf16 *dz, int32_t ld, int32_t coff, int32_t C, int32_t P, float *db, float *scratch,
                     int32_t nsplit, hipStream_t s);
// dz = dy * (y > 0 ? 1 : slope), same layout for y and dy (slices allowed)
hipError_t act_bwd(bf16 *dz, int32_t ldz, int32_t zoff, const bf16 *dy, int32_t ldy, int32_t yoff,
                   const bf16 *y, int32_t ld, int32_t coff, int32_t C, int32_t P, float slope, hipStream_t s);
// 3x3 stride-2 pad-1 average pooling (count_include_pad) and its adjoint
hipError_t pool_fwd(const bf16 *in, int32_t ldi, int32_t coff, int32_t C, int32_t H, int32_t W, bf16 *out,
                    hipStream_t s);
// pool_bwd with act_y: the result (after accumulating) is scaled by the
// activation derivative at act_y (same layout as din)
hipError_t pool_bwd(const bf16 *dout, int32_t C, int32_t H, int32_t W, bf16 *din, int32_t ldi, int32_t coff,
                    int32_t accumulate, const bf16 *act_y, float slope, hipStream_t s);
// 1x1 output conv (C -> 1) to FP32, MSE loss partials and its gradient
hipError_t outc_fwd(const bf16 *x, int32_t C, int32_t P, const float *w, const float *b, float *y,
                    hipStream_t s);
hipError_t mse(const float *y, const float *t, int32_t P, double *partials, int32_t nblk, float *dy,
               hipStream_t s);
// dx = w dy scaled by the activation derivative at x (x is the activated
// output of the last 3x3 convolution)
hipError_t outc_bwd(const bf16 *x, int32_t C, int32_t P, const float *w, const float *dy, bf16 *dx,
                    float *part_w, int32_t nblk, float slope, hipStream_t s);
hipError_t outc_wgrad_reduce(const float *part_w, int32_t C, int32_t nblk, float *dw, float *db, hipStream_t s);
hipError_t sum_partials_d(const double *p, int32_t n, double *out, float scale, float *out_f, hipStream_t s);
// Adam on a flat FP32 parameter vector; also refreshes the bf16 copy.
// hyper[0] = learning rate, [1] = 1 - beta1^t, [2] = 1 - beta2^t (device).
hipError_t adam(float *p, const float *g, float *m, float *v, bf16 *pb, int64_t n, const float *hyper,
                float beta1, float beta2, float eps, hipStream_t s);
// A weight tensor and its bf16 data-gradient matrix at aux_off: kind 0, a
// 3x3 convolution [co][tap][ci] -> [ci][(8 - tap)*Cout + co]; kind 1, a 2x2
// transposed convolution [ab][co][ci] -> [ci][ab*Cout + co]. tile0: the
// first of the tensor's 64 x 64 transpose tiles.
struct AuxSeg {
    int64_t off, n, aux_off, tile0;
    int32_t kind, cin, cout, pad;
};
// aux from the bf16 weights pb for the nseg tensors of segs (device, in
// tile order; ntiles tiles in all)
hipError_t aux_from_pb(const AuxSeg *segs, int32_t nseg, int64_t ntiles, const bf16 *pb, bf16 *aux, hipStream_t s);
hipError_t to_bf16(const float *x, bf16 *y, int64_t n, hipStream_t s);
// max |x| into out[0] (part: scratch of kAbsmaxBlocks floats)
constexpr int kAbsmaxBlocks = 256;
hipError_t absmax(const float *x, int64_t n, float *out, float *part, hipStream_t s);
// normalised, reflect-padded input: dst[(i,j)] = src[refl(i-py)][refl(j-px)] / max
hipError_t pad_norm(const float *src, int32_t nz, int32_t nx, int32_t H, int32_t W, int32_t py, int32_t px,
                    const float *maxabs, bf16 *dst_b, float *dst_f, hipStream_t s);
// crop and rescale: out[i][j] = y[(i+py)*W + j+px] * max
hipError_t crop_scale(const float *y, int32_t H, int32_t W, int32_t py, int32_t px, int32_t nz, int32_t nx,
                      const float *maxabs, float *out, hipStream_t s);
hipError_t fill_f(float *p, int64_t n, float v, hipStream_t s);

}  // namespace dbl
