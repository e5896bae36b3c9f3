// Warm-start network kernels for gfx950: implicit-GEMM convolutions on the
// matrix cores (bfloat16 inputs, FP32 accumulation), the weight gradient as
// a split-K GEMM with a fixed-order reduction, and the elementwise steps.
#include "cnn.hpp"

namespace lshom {
namespace cnn {

typedef float float4_t __attribute__((ext_vector_type(4)));

// Round to nearest even (finite inputs).
__device__ __forceinline__ bf16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// LDS rows of the tiles hold 32 reduction elements plus 8 of padding (80
// bytes: 16-byte aligned rows, fewer bank conflicts for the fragment reads).
constexpr int kTK = 32, kLd = kTK + 8;
constexpr int kTN = 64;  // weight-gradient tile channels
constexpr int kWM = 64;  // weight-gradient tile rows

// Input pixel read by output pixel (b, i, j) at tap t.
__device__ __forceinline__ long long in_pixel(int mode, int up, int Hi, int Wi, int Ho, int Wo, int b, int i, int j,
                                              int t) {
  if (mode == CM_CONV3) {
    const int p = t / 3, q = t - 3 * (t / 3);
    int ii = i + p - 1, jj = j + q - 1;
    ii += ii < 0 ? Ho : 0;
    ii -= ii >= Ho ? Ho : 0;
    jj += jj < 0 ? Wo : 0;
    jj -= jj >= Wo ? Wo : 0;
    if (up == 3) {
      ii /= 3;
      jj /= 3;
    }
    return ((long long)b * Hi + ii) * Wi + jj;
  }
  if (mode == CM_DOWN3) {
    const int p = t / 3, q = t - 3 * (t / 3);
    return ((long long)b * Hi + 3 * i + p) * Wi + 3 * j + q;
  }
  return ((long long)b * Hi + i) * Wi + j;
}

// Implicit-GEMM convolution: out[pixel][n] = sum_k im2col(in)[pixel][k] w[k][n]
// on the matrix cores (16x16x32 bfloat16 MFMA, FP32 accumulation).  A block
// of 4 waves computes TM = 4 WM output pixels x WN output channels, each
// wave a WM x WN slab of 16 x 16 tiles.  The reduction runs 32 at a time
// through two LDS buffers: the global loads of step s + 1 are in flight
// while step s multiplies, and one block barrier per step separates the
// writes of one buffer from the reads of the other.  Both operands are
// K-contiguous (activations: channels of one pixel and tap; weights: rows
// w[n][k] of ldw elements), so every LDS store and fragment read is 16
// bytes.  A lane's fragment is eight consecutive k of one row of each
// operand, the same k for both operands, so the contraction pairs them.
template <int WM, int WN>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs a) {
  constexpr int TM = 4 * WM, TN = WN, MT = WM / 16, NT = WN / 16;
  constexpr int A_PER = TM * 4 / 256;                        // uint4 loads of the pixel tile per thread
  constexpr int B_THREADS = TN * 4;                          // threads loading the weight tile
  __shared__ __align__(16) bf16_t As[2][TM * kLd];  // [pixel][k]
  __shared__ __align__(16) bf16_t Bs[2][TN * kLd];  // [channel][k]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const long long hw = (long long)a.Ho * a.Wo;
  const long long M = (long long)a.B * hw;
  const long long m0 = (long long)blockIdx.x * TM;
  const int n0 = blockIdx.y * TN;
  const int z = blockIdx.z;
  const int Cin = a.C0 + a.C1;
  const int taps = (a.mode == CM_CONV3 || a.mode == CM_DOWN3) ? 9 : 1;
  const int K = taps * Cin;
  const bf16_t* W = a.w + (a.mode == CM_DOWN3_T ? (long long)z * Cin : 0);

  // pixel rows (tid / 4) + 64 u of the tile, 8 reduction elements at column 8 (tid % 4)
  const int kg = tid & 3;
  int ab[A_PER], ai[A_PER], aj[A_PER];
  bool av[A_PER];
#pragma unroll
  for (int u = 0; u < A_PER; ++u) {
    const long long m = m0 + (tid >> 2) + 64 * u;
    av[u] = m < M;
    const long long mm = av[u] ? m : 0;
    ab[u] = (int)(mm / hw);
    const int rem = (int)(mm - (long long)ab[u] * hw);
    ai[u] = rem / a.Wo;
    aj[u] = rem - ai[u] * a.Wo;
  }
  // weight row n0 + tid / 4 (threads below B_THREADS), 8 elements at column 8 (tid % 4)
  const int bn = n0 + (tid >> 2);
  const bool bv = tid < B_THREADS && bn < a.Np;
  const bf16_t* wrow = W + (long long)(bv ? bn : 0) * a.ldw;

  uint4 ra[A_PER], rb = {0u, 0u, 0u, 0u};
  auto fetch = [&](int k0) {
    const int k = k0 + 8 * kg;
#pragma unroll
    for (int u = 0; u < A_PER; ++u) {
      ra[u] = uint4{0u, 0u, 0u, 0u};
      if (av[u] && k < K) {
        const int t = k / Cin;
        const int c = k - t * Cin;
        const long long pix = in_pixel(a.mode, a.up, a.Hi, a.Wi, a.Ho, a.Wo, ab[u], ai[u], aj[u], t);
        const bf16_t* src = c < a.C0 ? a.in0 + pix * a.ld0 + c : a.in1 + pix * a.ld1 + (c - a.C0);
        ra[u] = *reinterpret_cast<const uint4*>(src);
      }
    }
    rb = uint4{0u, 0u, 0u, 0u};
    if (bv && k < K) rb = *reinterpret_cast<const uint4*>(wrow + k);
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < A_PER; ++u)
      *reinterpret_cast<uint4*>(&As[buf][((tid >> 2) + 64 * u) * kLd + 8 * kg]) = ra[u];
    if (tid < B_THREADS) *reinterpret_cast<uint4*>(&Bs[buf][(tid >> 2) * kLd + 8 * kg]) = rb;
  };

  float4_t acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = float4_t{0.f, 0.f, 0.f, 0.f};

  fetch(0);
  stash(0);
  __syncthreads();
  const int steps = (K + kTK - 1) / kTK;
  for (int s = 0; s < steps; ++s) {
    const int cur = s & 1;
    if (s + 1 < steps) fetch((s + 1) * kTK);
    bf16x8_t af[MT], bfr[NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      af[mt] = *reinterpret_cast<const bf16x8_t*>(&As[cur][(wave * WM + mt * 16 + (lane & 15)) * kLd + 8 * (lane >> 4)]);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      bfr[nt] = *reinterpret_cast<const bf16x8_t*>(&Bs[cur][(nt * 16 + (lane & 15)) * kLd + 8 * (lane >> 4)]);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], bfr[nt], acc[mt][nt], 0, 0, 0);
    if (s + 1 < steps) stash(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long long m = m0 + wave * WM + mt * 16 + 4 * (lane >> 4) + i;
      if (m >= M) continue;
      long long op = m;
      if (a.mode == CM_DOWN3_T) {
        const int b = (int)(m / hw);
        const int rem = (int)(m - (long long)b * hw);
        const int ii = rem / a.Wo, jj = rem - (rem / a.Wo) * a.Wo;
        const int p = z / 3, q = z - 3 * (z / 3);
        op = ((long long)b * 3 * a.Ho + 3 * ii + p) * (3LL * a.Wo) + 3 * jj + q;
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int n = n0 + nt * 16 + (lane & 15);
        if (n >= a.N) continue;
        float v = acc[mt][nt][i] + (a.bias ? a.bias[n] : 0.f);
        if (a.relu) v = fmaxf(v, 0.f);
        if (a.out_b) a.out_b[op * a.ldb + n] = f2bf(v);
        if (a.out_f) {
          float* d = a.out_f + op * a.ldf + n;
          *d = a.accumulate ? *d + v : v;
        }
      }
    }
  }
}

// Weight gradient: partial[s][r][n] = sum over the pixels of split s of
// im2col(in)[pixel][r] * gy[pixel][n]; row r = taps * Cin is all ones (the
// bias gradient).
__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a) {
  __shared__ __align__(16) bf16_t As[kWM * kLd];  // [row][pixel]
  __shared__ __align__(16) bf16_t Bs[kTN * kLd];  // [channel][pixel]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int r0 = blockIdx.x * kWM, n0 = blockIdx.y * kTN, s = blockIdx.z;
  const long long hw = (long long)a.Ho * a.Wo;
  const long long M = (long long)a.B * hw;
  const long long pb0 = (long long)s * a.pix_per_split;
  const long long pend = (pb0 + a.pix_per_split < M) ? pb0 + a.pix_per_split : M;
  const int Cin = a.C0 + a.C1;
  const int Kf = a.taps * Cin;
  const int pl = tid >> 3, g = tid & 7;
  float4_t acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) acc[nt] = float4_t{0.f, 0.f, 0.f, 0.f};

  for (long long pb = pb0; pb < pend; pb += kTK) {
    const long long p = pb + pl;
    const bool pv = p < pend;
    int b = 0, i = 0, j = 0;
    if (pv) {
      b = (int)(p / hw);
      const int rem = (int)(p - (long long)b * hw);
      i = rem / a.Wo;
      j = rem - i * a.Wo;
    }
    {
      const int r = r0 + 8 * g;
      uint4 val = {0u, 0u, 0u, 0u};
      if (pv && r < Kf) {
        const int t = r / Cin;
        const int c = r - t * Cin;
        const long long pix = in_pixel(a.mode, a.up, a.Hi, a.Wi, a.Ho, a.Wo, b, i, j, t);
        const bf16_t* src = c < a.C0 ? a.in0 + pix * a.ld0 + c : a.in1 + pix * a.ld1 + (c - a.C0);
        val = *reinterpret_cast<const uint4*>(src);
      } else if (pv && r == Kf) {
        val.x = 0x3F80u;  // 1.0 in the first row of the group
      }
      const bf16_t* e = reinterpret_cast<const bf16_t*>(&val);
#pragma unroll
      for (int q = 0; q < 8; ++q) As[(8 * g + q) * kLd + pl] = e[q];
    }
    {
      const int n = n0 + 8 * g;
      uint4 val = {0u, 0u, 0u, 0u};
      if (pv && n < a.Np) val = *reinterpret_cast<const uint4*>(a.gy + p * a.ldg + n);
      const bf16_t* e = reinterpret_cast<const bf16_t*>(&val);
#pragma unroll
      for (int q = 0; q < 8; ++q) Bs[(8 * g + q) * kLd + pl] = e[q];
    }
    __syncthreads();
    {
      const bf16x8_t af = *reinterpret_cast<const bf16x8_t*>(&As[(wave * 16 + (lane & 15)) * kLd + 8 * (lane >> 4)]);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const bf16x8_t bfr =
            *reinterpret_cast<const bf16x8_t*>(&Bs[(nt * 16 + (lane & 15)) * kLd + 8 * (lane >> 4)]);
        acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr, acc[nt], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + wave * 16 + 4 * (lane >> 4) + i;
      const int n = n0 + nt * 16 + (lane & 15);
      if (r < a.rows && n < a.Np) a.partial[((long long)s * a.rows + r) * a.Np + n] = acc[nt][i];
    }
}

__global__ void wgrad_reduce_kernel(const float* partial, int splits, int rows, int Np, float* gw, float* gb) {
  const long long n_el = (long long)rows * Np;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n_el; e += (long long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int k = 0; k < splits; ++k) s += partial[(long long)k * n_el + e];
    const long long r = e / Np;
    if (r < rows - 1) gw[e] = s;
    else gb[e - r * Np] = s;
  }
}

__global__ void grad_prep_kernel(long long P, int C, int Cp, const float* g0, int ld0, const float* g1, int ld1,
                                 const bf16_t* act, int lda, bf16_t* gpre) {
  const long long n = P * Cp;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const long long p = e / Cp;
    const int c = (int)(e - p * Cp);
    float v = 0.f;
    if (c < C) {
      v = g0[p * ld0 + c];
      if (g1) v += g1[p * ld1 + c];
      if (act && !(bf2f(act[p * lda + c]) > 0.f)) v = 0.f;
    }
    gpre[e] = f2bf(v);
  }
}

__global__ void pool3_sum_kernel(int B, int Hc, int Wc, int C, const float* fine, float* coarse) {
  const long long n = (long long)B * Hc * Wc * C;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const long long pc = e / C;
    const int J = (int)(pc % Wc);
    const long long t = pc / Wc;
    const int I = (int)(t % Hc);
    const int b = (int)(t / Hc);
    float s = 0.f;
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q)
        s += fine[(((long long)b * 3 * Hc + 3 * I + p) * (3LL * Wc) + 3 * J + q) * C + c];
    coarse[e] = s;
  }
}

__global__ void make_input_kernel(int B, int N, const uint8_t* phase, const float* lr, int transpose, int scale,
                                  bf16_t* x) {
  const long long n = (long long)B * N * N;
  const int NF = N * scale;  // side of the stored image
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e % N);
    const long long t = e / N;
    const int i = (int)(t % N);
    const int b = (int)(t / N);
    int cnt = 0;
    for (int p = 0; p < scale; ++p)
      for (int q = 0; q < scale; ++q) {
        const int fi = scale * i + p, fj = scale * j + q;
        const long long src = transpose ? ((long long)b * NF + fj) * NF + fi : ((long long)b * NF + fi) * NF + fj;
        cnt += phase[src] != 0;
      }
    uint4 v0 = {0u, 0u, 0u, 0u};
    const uint32_t ph = 2 * cnt > scale * scale ? 0x3F80u : 0u;
    const uint32_t rr = f2bf(lr[b] * 0.25f);
    v0.x = ph | (rr << 16);
    *reinterpret_cast<uint4*>(x + e * 8) = v0;
  }
}

__global__ void mse_sums_kernel(int N, const float* pred, const double* e, double* part) {
  const int b = blockIdx.y;
  const long long nn = (long long)N * N;
  double s_num = 0.0, s_den = 0.0;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nn; p += (long long)gridDim.x * blockDim.x) {
    for (int c = 0; c < 2; ++c) {
      const double t = e[((long long)b * 2 + c) * nn + p] - (c == 0 ? 1.0 : 0.0);
      const double d = (double)pred[((long long)b * nn + p) * 2 + c] - t;
      s_num += d * d;
      s_den += t * t;
    }
  }
  __shared__ double red[2][256];
  red[0][threadIdx.x] = s_num;
  red[1][threadIdx.x] = s_den;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((long long)b * 2 + 0) * gridDim.x + blockIdx.x] = red[0][0];
    part[((long long)b * 2 + 1) * gridDim.x + blockIdx.x] = red[1][0];
  }
}

__global__ void mse_grad_kernel(int B, int N, int nb, const float* pred, const double* e, const double* part,
                                float* grad) {
  const int b = blockIdx.y;
  double den = 0.0;
  for (int k = 0; k < nb; ++k) den += part[((long long)b * 2 + 1) * nb + k];
  den = den > 1e-30 ? den : 1e-30;
  const double scale = 2.0 / (den * B);
  const long long nn = (long long)N * N;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nn; p += (long long)gridDim.x * blockDim.x)
    for (int c = 0; c < 2; ++c) {
      const double t = e[((long long)b * 2 + c) * nn + p] - (c == 0 ? 1.0 : 0.0);
      const long long q = ((long long)b * nn + p) * 2 + c;
      grad[q] = (float)(scale * ((double)pred[q] - t));
    }
}

__global__ void mse_loss_kernel(int B, int nb, const double* part, double* loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double l = 0.0;
  for (int b = 0; b < B; ++b) {
    double num = 0.0, den = 0.0;
    for (int k = 0; k < nb; ++k) {
      num += part[((long long)b * 2 + 0) * nb + k];
      den += part[((long long)b * 2 + 1) * nb + k];
    }
    l += num / (den > 1e-30 ? den : 1e-30);
  }
  *loss = l / B;
}

__global__ void make_field_kernel(int B, int N, const float* pred, int transpose, int scale, double* e) {
  const int NF = N * scale;
  const long long nn = (long long)N * N, nnf = (long long)NF * NF;
  const long long n = (long long)B * nnf;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(q / nnf);
    const long long pf = q - (long long)b * nnf;
    const int fi = (int)(pf / NF), fj = (int)(pf - (pf / NF) * NF);
    const int i = fi / scale, j = fj / scale;
    for (int c = 0; c < 2; ++c) {
      double v;
      if (!transpose) {
        v = (c == 0 ? 1.0 : 0.0) + (double)pred[((long long)b * nn + (long long)i * N + j) * 2 + c];
      } else {
        // field of the load case e2 from the prediction for the transposed image
        const long long pt = (long long)j * N + i;
        v = (c == 1 ? 1.0 : 0.0) + (double)pred[((long long)b * nn + pt) * 2 + (1 - c)];
      }
      e[((long long)b * 2 + c) * nnf + pf] = v;
    }
  }
}

__global__ void cast_weights_kernel(const float* w, int taps, int cin, int np, int flip, bf16_t* w16, bf16_t* wt16) {
  const long long n = (long long)taps * cin * np;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int o = (int)(e % np);
    const long long t2 = e / np;
    const int c = (int)(t2 % cin);
    const int t = (int)(t2 / cin);
    const bf16_t h = f2bf(w[e]);
    // forward: row o, k = t cin + c; input gradient: row c, k = t' np + o
    w16[(long long)o * taps * cin + t2] = h;
    const int tt = flip ? taps - 1 - t : t;
    wt16[((long long)c * taps + tt) * np + o] = h;
  }
}

__global__ void adam_kernel(long long n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

__global__ void fill_f32_kernel(float* p, long long n, float v) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    p[e] = v;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static unsigned grid_for(long long n, int per = 256, long long cap = 8192) {
  long long b = (n + per - 1) / per;
  if (b < 1) b = 1;
  return (unsigned)(b > cap ? cap : b);
}

hipError_t launch_conv(const ConvArgs& a, hipStream_t s) {
  const long long M = (long long)a.B * a.Ho * a.Wo;
  const unsigned zs = a.mode == CM_DOWN3_T ? 9 : 1;
  // channel tile sized to the layer (32 or 64 columns; 32 x 32 wave slabs
  // beat 64 x 32 ones on the 32-channel layers: more blocks per CU)
  if (a.Np <= 32) {
    hipLaunchKernelGGL((conv_kernel<32, 32>), dim3((unsigned)((M + 127) / 128), (unsigned)((a.Np + 31) / 32), zs),
                       dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL((conv_kernel<32, 64>), dim3((unsigned)((M + 127) / 128), (unsigned)((a.Np + 63) / 64), zs),
                       dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_wgrad(const WgradArgs& a, int splits, hipStream_t s) {
  const dim3 grid((unsigned)((a.rows + kWM - 1) / kWM), (unsigned)((a.Np + kTN - 1) / kTN), (unsigned)splits);
  hipLaunchKernelGGL(wgrad_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_wgrad_reduce(const float* partial, int splits, int rows, int Np, float* gw, float* gb, hipStream_t s) {
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(grid_for((long long)rows * Np)), dim3(256), 0, s, partial, splits, rows,
                     Np, gw, gb);
  return hipGetLastError();
}

hipError_t launch_grad_prep(long long P, int C, int Cp, const float* g0, int ld0, const float* g1, int ld1,
                            const bf16_t* act, int lda, bf16_t* gpre, hipStream_t s) {
  hipLaunchKernelGGL(grad_prep_kernel, dim3(grid_for(P * Cp)), dim3(256), 0, s, P, C, Cp, g0, ld0, g1, ld1, act, lda,
                     gpre);
  return hipGetLastError();
}

hipError_t launch_pool3_sum(int B, int Hc, int Wc, int C, const float* fine, float* coarse, hipStream_t s) {
  hipLaunchKernelGGL(pool3_sum_kernel, dim3(grid_for((long long)B * Hc * Wc * C)), dim3(256), 0, s, B, Hc, Wc, C, fine,
                     coarse);
  return hipGetLastError();
}

hipError_t launch_make_input(int B, int N, const uint8_t* phase, const float* log10_rho, int transpose, int scale,
                             bf16_t* x, hipStream_t s) {
  hipLaunchKernelGGL(make_input_kernel, dim3(grid_for((long long)B * N * N)), dim3(256), 0, s, B, N, phase, log10_rho,
                     transpose, scale, x);
  return hipGetLastError();
}

hipError_t launch_rel_mse(int B, int N, const float* pred, const double* e, double* part, double* loss, float* grad,
                          hipStream_t s) {
  const int nb = 256;
  hipLaunchKernelGGL(mse_sums_kernel, dim3(nb, B), dim3(256), 0, s, N, pred, e, part);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if (grad) {
    hipLaunchKernelGGL(mse_grad_kernel, dim3(64, B), dim3(256), 0, s, B, N, nb, pred, e, part, grad);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  hipLaunchKernelGGL(mse_loss_kernel, dim3(1), dim3(64), 0, s, B, nb, part, loss);
  return hipGetLastError();
}

hipError_t launch_make_field(int B, int N, const float* pred, int transpose, int scale, double* e, hipStream_t s) {
  hipLaunchKernelGGL(make_field_kernel, dim3(grid_for((long long)B * N * N * scale * scale)), dim3(256), 0, s, B, N,
                     pred, transpose, scale, e);
  return hipGetLastError();
}

hipError_t launch_cast_weights(const float* w, int taps, int cin, int np, int flip, bf16_t* w16, bf16_t* wt16,
                               hipStream_t s) {
  hipLaunchKernelGGL(cast_weights_kernel, dim3(grid_for((long long)taps * cin * np)), dim3(256), 0, s, w, taps, cin,
                     np, flip, w16, wt16);
  return hipGetLastError();
}

hipError_t launch_adam(long long n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, w, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, long long n, float v, hipStream_t s) {
  hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace lshom
