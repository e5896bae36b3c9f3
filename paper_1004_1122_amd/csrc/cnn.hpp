// Warm-start network: kernel arguments and launchers (internal).
//
// Activations are NHWC bfloat16 (stored as raw 16-bit words, round to nearest
// even); accumulation is FP32 on the matrix cores.  A view of a tensor is a
// base pointer, a channel count and the element stride between pixels, so a
// layer can read or write a channel slice of a wider buffer (the skip
// concatenation needs no copies).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lshom {
namespace cnn {

using bf16_t = uint16_t;

// Pixel maps of the implicit GEMM (output pixel (b, i, j) on an Ho x Wo grid).
enum ConvMode : int {
  CM_CONV3 = 0,    // 9 taps, input ((i + p - 1) mod Ho) / up, ((j + q - 1) mod Wo) / up
  CM_DOWN3 = 1,    // 9 taps, input (3 i + p, 3 j + q)
  CM_POINT = 2,    // 1 tap, input (i, j)
  CM_DOWN3_T = 3,  // 1 tap per launch slice z = 3 p + q: input (i, j), output (3 i + p, 3 j + q)
};

struct ConvArgs {
  const bf16_t* in0;     // channels [0, C0)
  const bf16_t* in1;     // channels [C0, C0 + C1) (may be null when C1 == 0)
  int C0, C1, ld0, ld1;  // channel counts (multiples of 8) and pixel strides
  int B, Hi, Wi, Ho, Wo;
  int mode, up;
  const bf16_t* w;       // element (k, n) of the reduction k < taps (C0 + C1) at w[n * ldw + k]
                         // (CM_DOWN3_T: slice z starts at w + z * (C0 + C1))
  int ldw;
  int N, Np;             // output channels, padded to a multiple of 8
  const float* bias;     // [N] or null
  int relu;
  bf16_t* out_b;         // bf16 output (or null): pixel stride ldb
  int ldb;
  float* out_f;          // FP32 output (or null): pixel stride ldf; accumulate adds
  int ldf, accumulate;
};

struct WgradArgs {
  const bf16_t* in0;
  const bf16_t* in1;
  int C0, C1, ld0, ld1;
  int B, Hi, Wi, Ho, Wo;
  int mode, up;          // CM_CONV3, CM_DOWN3 or CM_POINT
  const bf16_t* gy;      // [B Ho Wo][ldg], Np channels used
  int ldg, Np;
  int taps;
  int rows;              // taps (C0 + C1) + 1: the last row sums gy (bias gradient)
  long long pix_per_split;
  float* partial;        // [splits][rows][Np]
};

hipError_t launch_conv(const ConvArgs& a, hipStream_t s);
hipError_t launch_wgrad(const WgradArgs& a, int splits, hipStream_t s);
// grad[r][n] = sum_s partial[s][r][n] for r < rows (fixed order).
hipError_t launch_wgrad_reduce(const float* partial, int splits, int rows, int Np, float* grad_w, float* grad_b,
                               hipStream_t s);

// gpre[p][c] = bf16((g0[p * ld0 + c] + g1[p * ld1 + c]) * mask), c < C, zero
// for C <= c < Cp; mask = act[p * lda + c] > 0 when act is given.
hipError_t launch_grad_prep(long long P, int C, int Cp, const float* g0, int ld0, const float* g1, int ld1,
                            const bf16_t* act, int lda, bf16_t* gpre, hipStream_t s);
// coarse[b, I, J, c] (+)= sum over the 3 x 3 fine pixels of fine[b, 3I+p, 3J+q, c]
hipError_t launch_pool3_sum(int B, int Hc, int Wc, int C, const float* fine, float* coarse, hipStream_t s);
// Network input [B, N, N, 8]: phase indicator (phase != 0), log10(rho) / 4, zeros.
// transpose: read the image transposed (load case E = e2).  scale 3: the
// image is 3N x 3N and pixel (i, j) is the majority of block (3i.., 3j..).
hipError_t launch_make_input(int B, int N, const uint8_t* phase, const float* log10_rho, int transpose, int scale,
                             bf16_t* x, hipStream_t s);
// Relative MSE of pred [B, N, N, 2] (FP32, pixel stride 2) against the
// fluctuation of FP64 planar fields e [B][2][N][N] for E = e1; writes the
// loss (device scalar) and the FP32 gradient [B, N, N, 2].  part: 2 B * 256
// doubles of scratch.
hipError_t launch_rel_mse(int B, int N, const float* pred, const double* e, double* part, double* loss,
                          float* grad, hipStream_t s);
// Predicted field (FP64 planar [B][2][N][N]): E + prediction; transpose maps
// the prediction for the transposed image to the load case E = e2.
// scale 3: the field is 3N x 3N, pixel (i, j) takes prediction (i / 3, j / 3).
hipError_t launch_make_field(int B, int N, const float* pred, int transpose, int scale, double* e, hipStream_t s);
// Weight copies, rows contiguous in the reduction index: master w[t][c][o]
// (taps x cin x np) -> w16[o][t cin + c] for the forward convolution and
// wt16[c][t' np + o] for the input gradient (conv3 flips the taps, t' = 8 - t;
// down3 and 1x1 keep them).
hipError_t launch_cast_weights(const float* w, int taps, int cin, int np, int flip, bf16_t* w16, bf16_t* wt16,
                               hipStream_t s);
hipError_t launch_adam(long long n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);
hipError_t launch_fill_f32(float* p, long long n, float v, hipStream_t s);

}  // namespace cnn
}  // namespace lshom
