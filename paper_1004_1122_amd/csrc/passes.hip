// Pass kernels of the operator apply and the CG update.
//
// The CG vectors live in the spectral coordinate of the subspace U of
// zero-mean curl-free fields: a vector u of U is held as the Hermitian scalar
// c(k) with u_hat(k) = i khat(k) c(k) (khat = k / |k|), on the half spectrum
// (last-axis frequency in [0, N_last / 2]).  The operator of the collocation
// system (Sec. 2.2, Eqs. (15)-(17)) restricted to U then reads
//
//   A c = c + (1 / l0) (-i khat) . F[ dL (E + F^-1[i khat c]) ]      (E = 0 in CG)
//
// i.e. the Green operator of Sec. 2.1, Eq. (7) (k (x) k / (l0 |k|^2), zero at
// k = 0) becomes a projection on khat followed by 1 / l0.  One apply is:
//   axis-0 pass  (COL_INV_C):   c -> i khat_a c -> inverse FFT along axis 0
//   [axis-1 pass (COL_PLAIN):   inverse FFT along axis 1]               (3-D)
//   row pass     (ROW_FUSED):   inverse FFT along the last axis, dL (E + u),
//                               forward FFT along the last axis
//   [axis-1 pass (COL_PLAIN):   forward FFT along axis 1]               (3-D)
//   axis-0 pass  (COL_FWD_PROJ): forward FFT along axis 0, projection on
//                               khat, q = p + s / l0 and the dot (p, q).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "reduce.hpp"

namespace lshom {

// Integer frequency of DFT index m on an axis of n nodes (the set Z^N of
// Sec. 2.2, Eq. (9)).
__device__ __forceinline__ int freq_of(int m, int n) { return (m <= n / 2) ? m : m - n; }

// Unit frequency vector of the axis-0 element (l, inner index ii).  Returns
// false where the Green operator vanishes: k = 0, and for even N any
// k_a = N_a / 2.
template <typename T>
__device__ __forceinline__ bool khat_axis0(const ColArgs<T>& a, int l, long long ii, double* kh) {
  int idx[kMaxDim];
  idx[0] = l;
  if (a.dims == 2) {
    idx[1] = (int)ii;
  } else {
    idx[1] = (int)(ii / a.h);
    idx[2] = (int)(ii - (long long)idx[1] * a.h);
  }
  double k2 = 0.0;
  double kf[kMaxDim];
  for (int t = 0; t < a.dims; ++t) {
    const int n = a.nd[t];
    if ((n & 1) == 0 && idx[t] == n / 2) return false;
    // the last axis is stored as its non-negative half
    const int k = (t == a.dims - 1) ? idx[t] : freq_of(idx[t], n);
    kf[t] = (double)k;
    k2 += kf[t] * kf[t];
  }
  if (k2 == 0.0) return false;
  const double inv = 1.0 / sqrt(k2);
  for (int t = 0; t < a.dims; ++t) kh[t] = kf[t] * inv;
  return true;
}

// Weight of a half-spectrum entry in a full-spectrum sum: columns k_last = 0
// (and N/2 for even N) hold their own mirror images, the others stand for two.
__device__ __forceinline__ double half_weight(long long k_last, int n_last) {
  if (k_last == 0) return 1.0;
  if ((n_last & 1) == 0 && k_last == n_last / 2) return 1.0;
  return 2.0;
}

// ---------------------------------------------------------------------------
// Row pass
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kThreads) void row_kernel(RowArgs<T> a) {
  if (gated_out(a.st, a.gate)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* Z = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int n = a.n, h = a.h, ss = a.ss, d = a.d;
  const long long row0 = (long long)blockIdx.x * a.rows_per_block;
  const int nsig = d * a.rows_per_block;
  const int npairs = (nsig + 1) / 2;

  auto sig_valid = [&](int sg) -> bool { return sg < nsig && row0 + sg / d < a.nrows; };
  auto sig_row = [&](int sg) -> long long { return row0 + sg / d; };
  auto sig_comp = [&](int sg) -> int { return sg % d; };
  auto dl_at = [&](long long row, int x) -> T {
    return a.cond[a.phase[row * n + x]] - a.l0;
  };

  if (a.mode == ROW_FWD) {
    for (int idx = tid; idx < npairs * n; idx += kThreads) {
      const int p = idx / n;
      const int x = idx - p * n;
      T v[2] = {T(0), T(0)};
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int sg = 2 * p + u;
        if (!sig_valid(sg)) continue;
        const long long row = sig_row(sg);
        const int c = sig_comp(sg);
        T val = (a.flags & ROWF_CONST_E) ? a.E[c] : (T)a.real_in[c][row * n + x];
        if (a.flags & ROWF_DL) val *= dl_at(row, x);
        v[u] = val;
      }
      Z[p * ss + x] = cx<T>{v[0], v[1]};
    }
    __syncthreads();
  } else {
    // Hermitian half rows of two signals -> one full complex row
    for (int idx = tid; idx < npairs * h; idx += kThreads) {
      const int p = idx / h;
      const int k = idx - p * h;
      cx<T> sa = {T(0), T(0)}, sb = {T(0), T(0)};
      if (sig_valid(2 * p)) sa = a.spec[sig_comp(2 * p)][sig_row(2 * p) * h + k];
      if (sig_valid(2 * p + 1)) sb = a.spec[sig_comp(2 * p + 1)][sig_row(2 * p + 1) * h + k];
      Z[p * ss + k] = cx<T>{sa.re - sb.im, sa.im + sb.re};
      if (k >= 1 && n - k >= h) Z[p * ss + n - k] = cx<T>{sa.re + sb.im, sb.re - sa.im};
    }
    __syncthreads();
    fft_lds<T, +1, kThreads>(Z, npairs, ss, a.plan, a.tw, tid);

    if (a.mode == ROW_INV) {
      double acc[kMaxDim] = {0.0, 0.0, 0.0};
      for (int idx = tid; idx < npairs * n; idx += kThreads) {
        const int p = idx / n;
        const int x = idx - p * n;
        const cx<T> z = Z[p * ss + x];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int sg = 2 * p + u;
          if (!sig_valid(sg)) continue;
          const long long row = sig_row(sg);
          const int c = sig_comp(sg);
          const long long g = row * n + x;
          double val = (double)a.E[c] + (double)((u == 0 ? z.re : z.im) * a.inv_n);
          if (a.flags & ROWF_ADD) val += a.real_add[c][g];
          if (a.real_out[c]) a.real_out[c][g] = val;
          if (a.flags & ROWF_LEFF) acc[c] += (double)a.cond[a.phase[g]] * val;
        }
      }
      if (a.flags & ROWF_LEFF) grid_reduce_finalize<kThreads>(acc, d, a.partials, a.st, a.fin, (double)a.inv_n);
      return;
    }

    // ROW_FUSED: polarisation dL (E + u) at the nodes (Sec. 2.2, Eq. (17))
    for (int idx = tid; idx < npairs * n; idx += kThreads) {
      const int p = idx / n;
      const int x = idx - p * n;
      const cx<T> z = Z[p * ss + x];
      T t[2] = {T(0), T(0)};
      const T zz[2] = {z.re, z.im};
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int sg = 2 * p + u;
        if (!sig_valid(sg)) continue;
        const long long row = sig_row(sg);
        const int c = sig_comp(sg);
        t[u] = dl_at(row, x) * (a.E[c] + zz[u] * a.inv_n);
      }
      Z[p * ss + x] = cx<T>{t[0], t[1]};
    }
    __syncthreads();
  }

  fft_lds<T, -1, kThreads>(Z, npairs, ss, a.plan, a.tw, tid);

  // split the two real signals' spectra and store the half rows
  for (int idx = tid; idx < npairs * h; idx += kThreads) {
    const int p = idx / h;
    const int k = idx - p * h;
    const cx<T> Y = Z[p * ss + k];
    const cx<T> Ym = Z[p * ss + (k == 0 ? 0 : n - k)];
    const T half = T(0.5);
    const cx<T> ta = {(Y.re + Ym.re) * half, (Y.im - Ym.im) * half};
    const cx<T> tb = {(Y.im + Ym.im) * half, (Ym.re - Y.re) * half};
    if (sig_valid(2 * p)) a.spec[sig_comp(2 * p)][sig_row(2 * p) * h + k] = ta;
    if (sig_valid(2 * p + 1)) a.spec[sig_comp(2 * p + 1)][sig_row(2 * p + 1) * h + k] = tb;
  }
}

// ---------------------------------------------------------------------------
// Strided-axis pass
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kThreads) void col_kernel(ColArgs<T> a) {
  if (gated_out(a.st, a.gate)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* Z = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int L = a.L, C = a.tile, ss = a.ss, d = a.d;
  const long long o = blockIdx.x / a.tiles_per_outer;
  const long long i0 = (long long)(blockIdx.x - o * a.tiles_per_outer) * C;
  const long long rem = a.inner - i0;
  const int width = rem < C ? (int)rem : C;
  const int nseq = d * C;
  const cx<T> zero = {T(0), T(0)};

  if (a.mode == COL_INV_C) {
    const T beta = a.fuse_p ? (T)a.st->beta : T(0);
    for (int idx = tid; idx < L * C; idx += kThreads) {
      const int l = idx / C;
      const int c = idx - l * C;
      if (c < width) {
        const long long g = (o * L + l) * a.inner + i0 + c;
        cx<T> cv;
        if (a.fuse_p) {
          const cx<T> r = a.r_in[g];
          const cx<T> p = a.p_io[g];
          cv = cx<T>{r.re + beta * p.re, r.im + beta * p.im};
          a.p_io[g] = cv;
        } else {
          cv = a.c_in[g];
        }
        double kh[kMaxDim];
        const bool nz = khat_axis0(a, l, i0 + c, kh);
        for (int al = 0; al < d; ++al) {
          const T k = nz ? (T)kh[al] : T(0);
          Z[(al * C + c) * ss + l] = cx<T>{-k * cv.im, k * cv.re};  // i khat_a c
        }
      } else {
        for (int al = 0; al < d; ++al) Z[(al * C + c) * ss + l] = zero;
      }
    }
    __syncthreads();
    fft_lds<T, +1, kThreads>(Z, nseq, ss, a.plan, a.tw, tid);
    for (int idx = tid; idx < L * C; idx += kThreads) {
      const int l = idx / C;
      const int c = idx - l * C;
      if (c < width) {
        const long long g = (o * L + l) * a.inner + i0 + c;
        for (int al = 0; al < d; ++al) a.comp[al][g] = Z[(al * C + c) * ss + l];
      }
    }
    return;
  }

  for (int idx = tid; idx < L * C; idx += kThreads) {
    const int l = idx / C;
    const int c = idx - l * C;
    if (c < width) {
      const long long g = (o * L + l) * a.inner + i0 + c;
      for (int al = 0; al < d; ++al) Z[(al * C + c) * ss + l] = a.comp[al][g];
    } else {
      for (int al = 0; al < d; ++al) Z[(al * C + c) * ss + l] = zero;
    }
  }
  __syncthreads();

  if (a.mode == COL_PLAIN) {
    if (a.dir > 0)
      fft_lds<T, +1, kThreads>(Z, nseq, ss, a.plan, a.tw, tid);
    else
      fft_lds<T, -1, kThreads>(Z, nseq, ss, a.plan, a.tw, tid);
    for (int idx = tid; idx < L * C; idx += kThreads) {
      const int l = idx / C;
      const int c = idx - l * C;
      if (c < width) {
        const long long g = (o * L + l) * a.inner + i0 + c;
        for (int al = 0; al < d; ++al) a.comp[al][g] = Z[(al * C + c) * ss + l];
      }
    }
    return;
  }

  // COL_FWD_PROJ
  fft_lds<T, -1, kThreads>(Z, nseq, ss, a.plan, a.tw, tid);
  double acc = 0.0;
  const int n_last = a.nd[a.dims - 1];
  for (int idx = tid; idx < L * C; idx += kThreads) {
    const int l = idx / C;
    const int c = idx - l * C;
    if (c < width) {
      const long long g = (o * L + l) * a.inner + i0 + c;
      double kh[kMaxDim];
      const bool nz = khat_axis0(a, l, i0 + c, kh);
      cx<T> t = zero;
      if (nz) {
        for (int al = 0; al < d; ++al) {
          const cx<T> v = Z[(al * C + c) * ss + l];
          const T k = (T)kh[al];
          t.re += k * v.re;
          t.im += k * v.im;
        }
      }
      // s = -i khat . tau_hat
      cx<T> val = {a.coef_s * t.im, -a.coef_s * t.re};
      cx<T> b = zero;
      if (a.base) {
        b = a.base[g];
        val.re += a.coef_base * b.re;
        val.im += a.coef_base * b.im;
      }
      a.out[g] = val;
      if (a.dot) {
        const double w = half_weight((i0 + c) % a.h, n_last);
        if (a.dot == 1)
          acc += w * ((double)b.re * (double)val.re + (double)b.im * (double)val.im);
        else
          acc += w * ((double)val.re * (double)val.re + (double)val.im * (double)val.im);
      }
    }
  }
  if (a.dot) grid_reduce_finalize<kThreads>(&acc, 1, a.partials, a.st, a.fin, a.inv_n);
}

// ---------------------------------------------------------------------------
// CG update: x += alpha p, r -= alpha q, (r, r)
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kThreads) void update_kernel(UpdArgs<T> a) {
  if (gated_out(a.st, a.gate)) return;
  const T alpha = (T)a.st->alpha;
  double acc = 0.0;
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < a.n; i += stride) {
    const cx<T> p = a.p[i];
    const cx<T> q = a.q[i];
    cx<T> x = a.x[i];
    cx<T> r = a.r[i];
    x.re += alpha * p.re;
    x.im += alpha * p.im;
    r.re -= alpha * q.re;
    r.im -= alpha * q.im;
    a.x[i] = x;
    a.r[i] = r;
    const double w = half_weight(i % a.h, a.n_last);
    acc += w * ((double)r.re * (double)r.re + (double)r.im * (double)r.im);
  }
  grid_reduce_finalize<kThreads>(&acc, 1, a.partials, a.st, FIN_UPDATE, a.inv_n);
}

__global__ __launch_bounds__(kThreads) void mix_accumulate_kernel(MixArgs a) {
  if (gated_out(a.st, a.gate)) return;
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < a.n; i += stride) {
    const cx<float> y = a.x32[i];
    cx<double> x = a.x64[i];
    x.re += (double)y.re;
    x.im += (double)y.im;
    a.x64[i] = x;
    a.x32[i] = cx<float>{0.f, 0.f};
  }
}

__global__ __launch_bounds__(kThreads) void mix_convert_kernel(MixArgs a) {
  if (gated_out(a.st, a.gate)) return;
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < a.n; i += stride) {
    const cx<double> r = a.r64[i];
    a.r32[i] = cx<float>{(float)r.re, (float)r.im};
  }
  if (a.clear_refresh) {
    // every block must have read the flag before it is cleared
    double none = 0.0;
    grid_reduce_finalize<kThreads>(&none, 1, a.partials, a.st, FIN_CLEAR_REFRESH, 1.0);
  }
}

__global__ void state_init_kernel(DevState* st, DevState init) { *st = init; }

template <typename T>
__global__ __launch_bounds__(kThreads) void fill_zero_kernel(cx<T>* p, long long n) {
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
    p[i] = cx<T>{T(0), T(0)};
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

static int odd_stride(int n) { return (n & 1) ? n : n + 1; }

size_t row_lds_bytes(int n, int rows_per_block, int d, int elem_bytes, int* ss_out) {
  const int ss = odd_stride(n);
  if (ss_out) *ss_out = ss;
  const int npairs = (d * rows_per_block + 1) / 2;
  return (size_t)npairs * ss * elem_bytes;
}

size_t col_lds_bytes(int L, int tile, int d, int elem_bytes, int* ss_out) {
  const int ss = odd_stride(L);
  if (ss_out) *ss_out = ss;
  return (size_t)d * tile * ss * elem_bytes;
}

template <typename T>
long long row_blocks(const RowArgs<T>& a) {
  return (a.nrows + a.rows_per_block - 1) / a.rows_per_block;
}

template <typename T>
long long col_blocks(const ColArgs<T>& a) {
  return a.outer * (long long)a.tiles_per_outer;
}

long long update_blocks(long long n) {
  long long b = (n + kThreads - 1) / kThreads;
  return b > 2048 ? 2048 : (b < 1 ? 1 : b);
}

template <typename T>
hipError_t launch_row(const RowArgs<T>& a, hipStream_t s) {
  const size_t lds = row_lds_bytes(a.n, a.rows_per_block, a.d, (int)sizeof(cx<T>), nullptr);
  const long long nb = row_blocks(a);
  hipLaunchKernelGGL(row_kernel<T>, dim3((unsigned)nb), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col(const ColArgs<T>& a, hipStream_t s) {
  const size_t lds = col_lds_bytes(a.L, a.tile, a.d, (int)sizeof(cx<T>), nullptr);
  const long long nb = col_blocks(a);
  hipLaunchKernelGGL(col_kernel<T>, dim3((unsigned)nb), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_update(const UpdArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL(update_kernel<T>, dim3((unsigned)a.blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mix_accumulate(const MixArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(mix_accumulate_kernel, dim3((unsigned)a.blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mix_convert(const MixArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(mix_convert_kernel, dim3((unsigned)a.blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_state_init(DevState* st, const DevState& init, hipStream_t s) {
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(1), 0, s, st, init);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_zero(cx<T>* p, long long n, hipStream_t s) {
  const long long nb = update_blocks(n);
  hipLaunchKernelGGL(fill_zero_kernel<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

template hipError_t launch_row<double>(const RowArgs<double>&, hipStream_t);
template hipError_t launch_row<float>(const RowArgs<float>&, hipStream_t);
template hipError_t launch_col<double>(const ColArgs<double>&, hipStream_t);
template hipError_t launch_col<float>(const ColArgs<float>&, hipStream_t);
template hipError_t launch_update<double>(const UpdArgs<double>&, hipStream_t);
template hipError_t launch_update<float>(const UpdArgs<float>&, hipStream_t);
template hipError_t launch_fill_zero<double>(cx<double>*, long long, hipStream_t);
template hipError_t launch_fill_zero<float>(cx<float>*, long long, hipStream_t);
template long long row_blocks<double>(const RowArgs<double>&);
template long long row_blocks<float>(const RowArgs<float>&);
template long long col_blocks<double>(const ColArgs<double>&);
template long long col_blocks<float>(const ColArgs<float>&);

}  // namespace lshom
