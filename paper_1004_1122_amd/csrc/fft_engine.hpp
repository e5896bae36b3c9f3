// Batched 1-D FFTs in LDS for gfx950: register-level radix butterflies and a
// self-sorting (Stockham) stage loop.  Used by every pass kernel of the
// operator apply: the discrete Fourier transforms F and F^-1 of the
// collocation system (Sec. 2.2, Eqs. (12)-(14); Sec. 2.3 costs the operator by
// them).  Forward transforms carry exp(-2 pi i k m / N), inverse ones
// exp(+2 pi i k m / N); neither is normalised here.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "radix_consts.hpp"

namespace lshom {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
// multiply by S*i (S = +1 or -1)
template <typename T, int S>
__device__ __forceinline__ cx<T> mul_si(cx<T> a) {
  return S > 0 ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

// Multiply by exp(S * 2 pi i m / R) for a compile-time-foldable m.
template <typename T, int R, int S>
__device__ __forceinline__ cx<T> rot(cx<T> x, int m) {
  m = m % R;
  if (m == 0) return x;
  if (2 * m == R) return {-x.re, -x.im};
  if (4 * m == R) return mul_si<T, S>(x);
  if (4 * m == 3 * R) return mul_si<T, -S>(x);
  const T c = (T)RadixConst<R>::c[m];
  const T s = (T)(S * RadixConst<R>::s[m]);
  return {x.re * c - x.im * s, x.re * s + x.im * c};
}

// ---------------------------------------------------------------------------
// Small DFTs in registers.  y_k = sum_j x_j exp(S 2 pi i j k / R).
// ---------------------------------------------------------------------------

template <typename T, int R, int S>
__device__ __forceinline__ void dft(cx<T>* x);

// Prime R: pair j with R-j so that each cosine/sine multiplies a sum/difference.
template <typename T, int R, int S>
__device__ __forceinline__ void dft_prime(cx<T>* x) {
  constexpr int H = (R - 1) / 2;
  cx<T> a[H + 1], b[H + 1];
  cx<T> y0 = x[0];
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    a[j] = cadd(x[j], x[R - j]);
    b[j] = csub(x[j], x[R - j]);
    y0 = cadd(y0, a[j]);
  }
  cx<T> out[R];
  out[0] = y0;
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    cx<T> P = x[0];
    cx<T> Q = {T(0), T(0)};
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const int idx = (j * m) % R;
      const T c = (T)RadixConst<R>::c[idx];
      const T s = (T)RadixConst<R>::s[idx];
      P = {P.re + c * a[j].re, P.im + c * a[j].im};
      Q = {Q.re + s * b[j].re, Q.im + s * b[j].im};
    }
    const cx<T> iQ = mul_si<T, S>(Q);
    out[m] = cadd(P, iQ);
    out[R - m] = csub(P, iQ);
  }
#pragma unroll
  for (int m = 0; m < R; ++m) x[m] = out[m];
}

// Composite R = R1 * R2 (Cooley-Tukey in registers): index j = R2 j1 + j2,
// output k = k1 + R1 k2.
template <typename T, int R1, int R2, int S>
__device__ __forceinline__ void dft_ct(cx<T>* x) {
  constexpr int R = R1 * R2;
  cx<T> z[R];
#pragma unroll
  for (int j2 = 0; j2 < R2; ++j2) {
    cx<T> t[R1];
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) t[j1] = x[R2 * j1 + j2];
    dft<T, R1, S>(t);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) z[j2 * R1 + k1] = rot<T, R, S>(t[k1], j2 * k1);
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cx<T> t[R2];
#pragma unroll
    for (int j2 = 0; j2 < R2; ++j2) t[j2] = z[j2 * R1 + k1];
    dft<T, R2, S>(t);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) x[k1 + R1 * k2] = t[k2];
  }
}

// R = 3 with the sine term fused into the outputs: y1,2 = P -+ S s3 (b.im, -b.re)
// with P = x0 - a / 2, a = x1 + x2, b = x1 - x2, s3 = sin(2 pi / 3); twelve
// operations, eight of them fused multiply-adds.
template <typename T, int S>
__device__ __forceinline__ void dft3(cx<T>* x) {
  const T s3 = (T)(S * RadixConst<3>::s[1]);
  const cx<T> a = cadd(x[1], x[2]), b = csub(x[1], x[2]);
  const cx<T> P = {x[0].re - T(0.5) * a.re, x[0].im - T(0.5) * a.im};
  x[0] = cadd(x[0], a);
  x[1] = cx<T>{P.re - s3 * b.im, P.im + s3 * b.re};
  x[2] = cx<T>{P.re + s3 * b.im, P.im - s3 * b.re};
}

template <typename T, int R, int S>
__device__ __forceinline__ void dft(cx<T>* x) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    const cx<T> a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (R == 3) {
    dft3<T, S>(x);
  } else if constexpr (R == 5 || R == 7 || R == 11 || R == 13 || R == 17) {
    dft_prime<T, R, S>(x);
  } else if constexpr (R == 4) {
    dft_ct<T, 2, 2, S>(x);
  } else if constexpr (R == 6) {
    dft_ct<T, 2, 3, S>(x);
  } else if constexpr (R == 8) {
    dft_ct<T, 2, 4, S>(x);
  } else if constexpr (R == 9) {
    dft_ct<T, 3, 3, S>(x);
  } else {
    static_assert(R <= 9 || R == 11 || R == 13 || R == 17, "unsupported radix");
  }
}

// ---------------------------------------------------------------------------
// Plans and the LDS stage loop
// ---------------------------------------------------------------------------

constexpr int kMaxStages = 16;

// Unsigned division by a runtime constant d >= 1, for 0 <= x < 2^31, as a
// multiply-high and a shift: with s = ceil(log2 d) and
// m = floor(2^32 (2^s - d) / d) + 1, floor(x / d) = (mulhi(x, m) + x) >> s
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, the round-up multiplier; x < 2^31 keeps the sum
// within 32 bits).
struct FastDiv {
  uint32_t d, m, s;
};

__host__ inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f{d, 1u, 0u};
  if (d <= 1) return f;
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.s = s;
  f.m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << s) - d)) / d + 1);
  return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FastDiv& f) {
  return (__umulhi(x, f.m) + x) >> f.s;
}

// Radix schedule of one axis; the product of radix[0..nstages) is n.  nr[st]
// and ns[st] divide by n / radix[st] and by the product of the radices before
// stage st (filled by the host planner).
struct FftPlan {
  int n;
  int nstages;
  int radix[kMaxStages];
  FastDiv nr[kMaxStages];
  FastDiv ns[kMaxStages];
};

// Butterflies held per thread across the stage barrier, per radix.  The host
// sizes every batch so that nseq * n / R <= jobs_per_thread(R) * threads.
__host__ __device__ constexpr int jobs_per_thread(int R) {
  return R <= 3 ? 4 : (R <= 5 ? 3 : (R <= 9 ? 2 : 1));
}

// Largest number of points (nseq * n) one batch may hold for a plan.
__host__ __device__ inline int plan_batch_cap(const FftPlan& p, int threads) {
  int cap = 1 << 30;
  for (int s = 0; s < p.nstages; ++s) {
    const int c = jobs_per_thread(p.radix[s]) * p.radix[s] * threads;
    cap = c < cap ? c : cap;
  }
  return cap;
}

// Number of twiddle-table entries kept in LDS for an n-point transform:
// exp(-2 pi i m / n) for every 0 <= m < n.  A stage twiddle index
// r k n / (Ns R) (r < R, k < Ns) is below n, so the lookup is one LDS read:
// folding the upper half onto the lower one by conjugate symmetry would cost
// a compare and two selects per twiddle (measured: the passes are VALU-issue
// bound, and the half table was 3-5% slower).
__host__ __device__ constexpr int twiddle_entries(int n) { return n; }

template <typename T>
__device__ __forceinline__ cx<T> twiddle(const cx<T>* __restrict__ tw, int m) {
  return tw[m];
}

// One self-sorting stage, in place: every thread loads its butterflies into
// registers, the block synchronises, then every thread stores them.
// Sequence s, element e lives at buf[s * ss + e].  Twiddle table tw[m] holds
// exp(-2 pi i m / n) for 0 <= m < n (conjugated for the inverse direction,
// S = +1).
template <typename T, int R, int S, int NT>
__device__ __forceinline__ void fft_stage(cx<T>* buf, int nseq, int ss, int n, int Ns,
                                          const cx<T>* __restrict__ tw, int tid, const FastDiv& fnr,
                                          const FastDiv& fns) {
  constexpr int JM = jobs_per_thread(R);
  const int NR = (int)fnr.d;
  const int jobs = nseq * NR;
  const int step = NR / Ns;  // n / (Ns R)
  cx<T> v[JM][R];
  int out_at[JM];  // store offset of each job, kept across the barrier
#pragma unroll
  for (int q = 0; q < JM; ++q) {
    const int job = tid + q * NT;
    out_at[q] = 0;
    if (job < jobs) {
      const int s = (int)fdiv((uint32_t)job, fnr);
      const int j = job - s * NR;
      const cx<T>* b = buf + s * ss + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = b[r * NR];
      const int k = Ns > 1 ? j - (int)fdiv((uint32_t)j, fns) * Ns : 0;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = twiddle(tw, r * k * step);
          if (S > 0) w.im = -w.im;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      dft<T, R, S>(v[q]);
      out_at[q] = s * ss + (j - k) * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < JM; ++q) {
    if (tid + q * NT < jobs) {
      cx<T>* b = buf + out_at[q];
#pragma unroll
      for (int r = 0; r < R; ++r) b[r * Ns] = v[q][r];
    }
  }
  __syncthreads();
}

// Radix sets a kernel is compiled for: the register footprint of a kernel is
// that of its largest butterfly, so grids whose lengths are powers of 3 (or
// of 2) get kernels without the radix-5/7 code, and only grids with a prime
// factor 11, 13 or 17 get the kernels that carry those butterflies.
enum RadixSet : int { RADIX_POW3 = 0, RADIX_POW2 = 1, RADIX_ALL = 2, RADIX_WIDE = 3 };

__host__ __device__ constexpr bool is_wide_prime(int R) { return R == 11 || R == 13 || R == 17; }

__host__ __device__ inline bool radix_in_set(int R, int set) {
  if (set == RADIX_POW3) return R == 3 || R == 9;
  if (set == RADIX_POW2) return R == 2 || R == 4 || R == 8;
  if (set == RADIX_ALL) return R >= 2 && R <= 9;
  return (R >= 2 && R <= 9) || is_wide_prime(R);
}

// Transform nseq sequences of length plan.n in LDS.  Callers synchronise
// before (data written) and may read the result right after.  Every radix of
// the plan must belong to RS.
template <typename T, int S, int NT, int RS>
__device__ __forceinline__ void fft_lds(cx<T>* buf, int nseq, int ss, const FftPlan& plan,
                        const cx<T>* __restrict__ tw, int tid) {
  int Ns = 1;
  for (int st = 0; st < plan.nstages; ++st) {
    const int R = plan.radix[st];
    if constexpr (RS == RADIX_POW3) {
      if (R == 9) fft_stage<T, 9, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]);
      else fft_stage<T, 3, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]);
    } else if constexpr (RS == RADIX_POW2) {
      if (R == 8) fft_stage<T, 8, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]);
      else if (R == 4) fft_stage<T, 4, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]);
      else fft_stage<T, 2, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]);
    } else {
      switch (R) {
        case 2: fft_stage<T, 2, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]); break;
        case 3: fft_stage<T, 3, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]); break;
        case 4: fft_stage<T, 4, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]); break;
        case 5: fft_stage<T, 5, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]); break;
        case 6: fft_stage<T, 6, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]); break;
        case 7: fft_stage<T, 7, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]); break;
        case 8: fft_stage<T, 8, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]); break;
        case 9: fft_stage<T, 9, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]); break;
        default:
          if constexpr (RS == RADIX_WIDE) {
            if (R == 11) fft_stage<T, 11, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]);
            else if (R == 13) fft_stage<T, 13, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]);
            else if (R == 17) fft_stage<T, 17, S, NT>(buf, nseq, ss, plan.n, Ns, tw, tid, plan.nr[st], plan.ns[st]);
          }
          break;
      }
    }
    Ns *= R;
  }
}

__host__ __device__ inline int plan_radix_set(const FftPlan& p) {
  bool p3 = true, p2 = true, wide = false;
  for (int s = 0; s < p.nstages; ++s) {
    p3 = p3 && radix_in_set(p.radix[s], RADIX_POW3);
    p2 = p2 && radix_in_set(p.radix[s], RADIX_POW2);
    wide = wide || is_wide_prime(p.radix[s]);
  }
  return p3 ? RADIX_POW3 : (p2 ? RADIX_POW2 : (wide ? RADIX_WIDE : RADIX_ALL));
}

}  // namespace lshom
