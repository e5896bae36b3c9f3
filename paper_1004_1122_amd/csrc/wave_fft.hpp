// Wave-level FFTs of length N = 9^m 3^e <= 243 for gfx950.
//
// One sequence of N complex points is owned by LPS = N / 9 lanes of a
// wavefront, each lane holding 9 points; a wave holds SPW = 64 / LPS
// sequences (243: 2 sequences on 54 lanes, 81: 7 on 63, 27: 21 on 63).
// The self-sorting (Stockham) stages exchange data through a wave-private
// region of LDS, so no block-wide barrier is needed: the lanes of a wave
// issue every LDS read of a stage before any write of it (the writes depend on
// all nine values of the lane's butterfly), LDS executes a wave's
// instructions in order, and a wave barrier keeps the compiler from moving
// memory operations across a stage boundary.
//
// Stage with radix R and Ns = product of the radices before it: job q
// (q < N / R) reads x[q + r N / R], multiplies by W_{Ns R}^{r k} with
// k = q mod Ns, applies a DFT of length R and writes x[(q - k) R + k + r Ns].
// Radix-9 stages give each lane one job, a final radix-3 stage three.  These
// are the discrete Fourier transforms F, F^-1 of the collocation system
// (Sec. 2.2, Eqs. (12)-(14)); forward transforms carry exp(-2 pi i k m / N),
// inverse ones exp(+2 pi i k m / N), neither normalised.
#pragma once

#include "fft_engine.hpp"

namespace lshom {

template <int N>
struct WaveGeom {
  static_assert(N == 9 || N == 27 || N == 81 || N == 243, "wave FFT lengths: 9, 27, 81, 243");
  static constexpr int LPS = N / 9;         // lanes per sequence
  static constexpr int SPW = 64 / LPS;      // sequences per wave
};

namespace wfft_detail {

// The stages after the first (radix 9, Ns = 1) one, for the length
// M = N / NS still to combine: radix 9 while 9 divides M, then radix 3.
// Barriers stay outside the lane predicate (they only order the compiler's
// memory operations; the whole wave passes them).
//
// With KEEP the last stage leaves its outputs in registers instead of LDS:
// its jobs q = j + (N / 9) t write x[q + r N / R] = x[j + (N / 9) s] (the
// last stage has Ns = N / R and k = q), so the lane keeps out[s] = x[j +
// (N / 9) s], s < 9: the input order of the first stage, and the order of
// the lane's nodes in wave_fft.
template <typename T, int N, int S, int NS, bool KEEP = false>
__device__ __forceinline__ void stages_from(cx<T>* buf, const cx<T>* __restrict__ tw, int j, bool act,
                                            cx<T>* out = nullptr) {
  constexpr int M = N / NS;
  if constexpr (M == 1) {
    return;
  } else if constexpr (M % 9 == 0) {
    constexpr int R = 9, NR = N / R, step = NR / NS;
    cx<T> v[R];
    const int k = j % NS;
    if (act) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = buf[j + r * NR];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cx<T> w = tw[r * k * step];
        if (S > 0) w.im = -w.im;
        v[r] = cmul(v[r], w);
      }
    }
    __builtin_amdgcn_wave_barrier();
    if constexpr (KEEP && M == R) {
      // last stage (one job per lane, q = j = k): x[j + r N / 9]
      if (act) {
        dft<T, R, S>(v);
#pragma unroll
        for (int r = 0; r < R; ++r) out[r] = v[r];
      }
    } else {
      if (act) {
        dft<T, R, S>(v);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[(j - k) * R + k + r * NS] = v[r];
      }
      __builtin_amdgcn_wave_barrier();
      stages_from<T, N, S, NS * R, KEEP>(buf, tw, j, act, out);
    }
  } else {
    static_assert(M == 3, "a radix-3 stage ends the plan");
    constexpr int R = 3, NR = N / R, step = NR / NS, LPS = N / 9;
    cx<T> u[3][R];
    int kk[3];
    if (act) {
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int q = j + LPS * t;
        const int k = q % NS;
        kk[t] = (q - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) u[t][r] = buf[q + r * NR];
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[r * k * step];
          if (S > 0) w.im = -w.im;
          u[t][r] = cmul(u[t][r], w);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    if constexpr (KEEP) {
      // jobs q = j + LPS t (k = q): x[j + LPS (t + 3 r)]
      (void)kk;
      if (act) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          dft<T, R, S>(u[t]);
#pragma unroll
          for (int r = 0; r < R; ++r) out[t + 3 * r] = u[t][r];
        }
      }
    } else {
      if (act) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          dft<T, R, S>(u[t]);
#pragma unroll
          for (int r = 0; r < R; ++r) buf[kk[t] + r * NS] = u[t][r];
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

}  // namespace wfft_detail

// Transform one sequence held by the lane group of this lane (j = index of
// the lane in its group, 0 <= j < N / 9).  v holds x[j + (N / 9) r] for
// r < 9 (the input order of the first stage); buf is the sequence's LDS
// region (N entries) and receives the transform in natural order; tw[m] =
// exp(-2 pi i m / N), 0 <= m < N.  Lanes outside a group pass act = false.
// The whole wave must call this together.
template <typename T, int N, int S>
__device__ __forceinline__ void wave_fft(cx<T> (&v)[9], cx<T>* buf, const cx<T>* __restrict__ tw, int j,
                                         bool act) {
  // first stage: radix 9, Ns = 1 (no twiddles): writes x[9 j + r]
  __builtin_amdgcn_wave_barrier();
  if (act) {
    dft<T, 9, S>(v);
#pragma unroll
    for (int r = 0; r < 9; ++r) buf[9 * j + r] = v[r];
  }
  __builtin_amdgcn_wave_barrier();
  wfft_detail::stages_from<T, N, S, 9>(buf, tw, j, act);
}

// The same transform for a sequence already stored in natural order in buf
// (by this wave's lanes or, after a block barrier, by others).
template <typename T, int N, int S>
__device__ __forceinline__ void wave_fft_lds(cx<T>* buf, const cx<T>* __restrict__ tw, int j, bool act) {
  constexpr int LPS = N / 9;
  cx<T> v[9];
  __builtin_amdgcn_wave_barrier();
  if (act) {
#pragma unroll
    for (int r = 0; r < 9; ++r) v[r] = buf[j + LPS * r];
  }
  wave_fft<T, N, S>(v, buf, tw, j, act);
}

// As wave_fft, the transform left in registers: out[s] = X[j + (N / 9) s]
// for s < 9 (the sequence's LDS region holds intermediate values after it).
template <typename T, int N, int S>
__device__ __forceinline__ void wave_fft_regs(cx<T> (&v)[9], cx<T>* buf, const cx<T>* __restrict__ tw, int j,
                                              bool act, cx<T> (&out)[9]) {
  __builtin_amdgcn_wave_barrier();
  if constexpr (N == 9) {
    if (act) {
      dft<T, 9, S>(v);
#pragma unroll
      for (int r = 0; r < 9; ++r) out[r] = v[r];
    }
  } else {
    if (act) {
      dft<T, 9, S>(v);
#pragma unroll
      for (int r = 0; r < 9; ++r) buf[9 * j + r] = v[r];
    }
    __builtin_amdgcn_wave_barrier();
    wfft_detail::stages_from<T, N, S, 9, true>(buf, tw, j, act, out);
  }
}

// As wave_fft_lds, the transform left in registers (see wave_fft_regs).
template <typename T, int N, int S>
__device__ __forceinline__ void wave_fft_lds_regs(cx<T>* buf, const cx<T>* __restrict__ tw, int j, bool act,
                                                  cx<T> (&out)[9]) {
  constexpr int LPS = N / 9;
  cx<T> v[9];
  __builtin_amdgcn_wave_barrier();
  if (act) {
#pragma unroll
    for (int r = 0; r < 9; ++r) v[r] = buf[j + LPS * r];
  }
  wave_fft_regs<T, N, S>(v, buf, tw, j, act, out);
}

}  // namespace lshom
