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
// Twiddles (and, in the row pass, phase bytes and conductivities) are staged
// in LDS at block start.
//
// A general reference medium L0 (Sec. 2.1, Eqs. (3) and (7): Green operator
// k (x) k / (k . L0 . k)) keeps this structure with the coordinate scaled:
// u_hat = i khat s(k) c with s = 1 / sqrt(khat . L0n . khat), L0n = L0 / lbar,
// lbar = tr(L0) / d, and the forward projection s (-i khat) . tau_hat / lbar.
// The operator on c is then symmetric in the Euclidean product (it equals
// the operator on fields in the energy product of L0), so CG runs unchanged;
// for L0 = l0 I, s = 1 and lbar = l0.
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
__device__ __forceinline__ bool khat_axis0(const ColArgs<T>& a, int l, long long ii, double* kh,
                                           double* k2_out = nullptr) {
  int idx[kMaxDim];
  idx[0] = l;
  if (a.dims == 2) {
    idx[1] = (int)ii;
  } else {
    idx[1] = (int)fdiv((uint32_t)ii, a.fd_h);
    idx[2] = (int)(ii - (long long)idx[1] * a.h);
  }
  if (a.dims == 2) idx[2] = 0;
  double k2 = 0.0;
  double kf[kMaxDim];
#pragma unroll
  for (int t = 0; t < kMaxDim; ++t) {
    kf[t] = 0.0;
    if (t < a.dims) {
      const int n = a.nd[t];
      if ((n & 1) == 0 && idx[t] == n / 2) return false;
      // the last axis is stored as its non-negative half; xi = k / Y
      const int k = (t == a.dims - 1) ? idx[t] : freq_of(idx[t], n);
      kf[t] = (double)k * a.cinv[t];
      k2 += kf[t] * kf[t];
    }
  }
  if (k2 == 0.0) return false;
  if (k2_out) *k2_out = k2;
  const double inv = 1.0 / sqrt(k2);
#pragma unroll
  for (int t = 0; t < kMaxDim; ++t) kh[t] = kf[t] * inv;
  return true;
}

// Weight of a half-spectrum entry in a full-spectrum sum: columns k_last = 0
// (and N/2 for even N) hold their own mirror images, the others stand for two.
__device__ __forceinline__ double half_weight(long long k_last, int n_last) {
  if (k_last == 0) return 1.0;
  if ((n_last & 1) == 0 && k_last == n_last / 2) return 1.0;
  return 2.0;
}

// (L_q - S) v at one node for a symmetric tensor phase q whose entries are
// stored as its upper triangle row by row (2-D: 00 01 11; 3-D: 00 01 02 11
// 12 22), S symmetric in the same layout: the polarisation of Sec. 2.1,
// Eq. (3) with tensor phases (S = L0) or the current L v (S = 0).
template <typename T>
__device__ __forceinline__ void tensor_times(const T* tab, int q, int d, const T* S, const T* v, T* out) {
  if (d == 2) {
    const T* m = tab + q * 3;
    const T m0 = m[0] - S[0], m1 = m[1] - S[1], m2 = m[2] - S[2];
    out[0] = m0 * v[0] + m1 * v[1];
    out[1] = m1 * v[0] + m2 * v[1];
    out[2] = T(0);
  } else {
    const T* m = tab + q * 6;
    const T m0 = m[0] - S[0], m1 = m[1] - S[1], m2 = m[2] - S[2];
    const T m3 = m[3] - S[3], m4 = m[4] - S[4], m5 = m[5] - S[5];
    out[0] = m0 * v[0] + m1 * v[1] + m2 * v[2];
    out[1] = m1 * v[0] + m3 * v[1] + m4 * v[2];
    out[2] = m2 * v[0] + m4 * v[1] + m5 * v[2];
  }
}

// The shift of tensor_times for dL = L - L0: L0 of an anisotropic reference,
// else l0 on the diagonal.
template <typename T>
__device__ __forceinline__ void reference_shift(const RowArgs<T>& a, T l0, T* S) {
#pragma unroll
  for (int i = 0; i < 6; ++i) S[i] = a.aniso ? a.L0u[i] : T(0);
  if (!a.aniso) {
    if (a.d == 2) {
      S[0] = l0;
      S[2] = l0;
    } else {
      S[0] = l0;
      S[3] = l0;
      S[5] = l0;
    }
  }
}

// x . M . x for the upper triangle M (layout of tensor_times) and a vector
// with dims components.
__device__ __forceinline__ double sym_quad(const double* m, int dims, const double* x) {
  if (dims == 2) return m[0] * x[0] * x[0] + 2.0 * m[1] * x[0] * x[1] + m[2] * x[1] * x[1];
  return m[0] * x[0] * x[0] + m[3] * x[1] * x[1] + m[5] * x[2] * x[2] +
         2.0 * (m[1] * x[0] * x[1] + m[2] * x[0] * x[2] + m[4] * x[1] * x[2]);
}

// Loads in flight per thread in the staging and data loops: with few blocks
// per CU (small grids) latency, not bandwidth, bounds a pass, so every loop
// issues kBatch independent global loads before it waits.
constexpr int kBatch = 4;

// Copy n elements global -> LDS with kBatch loads in flight per thread.
template <typename V, int NT>
__device__ __forceinline__ void copy_batched(V* dst, const V* __restrict__ src, int n) {
  for (int base = 0; base < n; base += NT * kBatch) {
    V r[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = base + u * NT + (int)threadIdx.x;
      r[u] = V{};
      if (i < n) r[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = base + u * NT + (int)threadIdx.x;
      if (i < n) dst[i] = r[u];
    }
  }
}

static __host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// arr[c] for a small runtime c without dynamic indexing (which would place
// the array in scratch memory)
template <typename V>
__device__ __forceinline__ V pick3(const V (&arr)[kMaxDim], int c) {
  return c == 0 ? arr[0] : (c == 1 ? arr[1] : arr[2]);
}

// The dispatcher deals the blocks of a launch to the 8 XCDs (each with its own
// L2) in linear order, one each in turn.  Neighbouring blocks of a pass read
// the two halves (or quarters) of the same cache lines, so the linear id is
// re-mapped to give each XCD one contiguous run of (problem, block) pairs:
// the shared lines are then fetched once into one L2.  A bijection of the
// grid: XCD x owns q + (x < rem) consecutive ids.
__device__ __forceinline__ void xcd_order(unsigned& bx, unsigned& by) {
  const unsigned gx = gridDim.x, total = gx * gridDim.y;
  const unsigned lin = blockIdx.y * gx + blockIdx.x;
  const unsigned xcd = lin & 7u, slot = lin >> 3;
  const unsigned q = total >> 3, rem = total & 7u;
  const unsigned lin2 = xcd * q + (xcd < rem ? xcd : rem) + slot;
  by = lin2 / gx;
  bx = lin2 - by * gx;
}

// ---------------------------------------------------------------------------
// Row pass
// ---------------------------------------------------------------------------

template <typename T, int NT, int RS, int MODE>
__global__ __launch_bounds__(NT) void row_kernel(RowArgs<T> a) {
  // neighbouring row blocks share the cache lines at their edges in the
  // transposed layout: XCD-aware order
  unsigned bx, by;
  xcd_order(bx, by);
  const int pb = a.bt.live ? a.bt.live[by] : (int)by;
  DevState* st = a.st + pb;
  // the flags a row pass gates on are written only by earlier launches; the
  // spectral passes read them with their first data chunk (below)
  if constexpr (MODE == ROW_FWD) {
    if (gated_out_stable(st, a.gate)) return;
  }
  const ProbEntry* pe = a.bt.tab ? a.bt.tab + pb : nullptr;
  const long long vo = (long long)pb * a.bt.vstride;
  Partials parts = a.parts;
  parts.base += (long long)pb * a.bt.pstride;
  const uint8_t* phase = pe ? pe->phase : a.phase;
  const T l0 = pe ? (T)pe->l0 : a.l0;
  T Ev[kMaxDim];
#pragma unroll
  for (int c = 0; c < kMaxDim; ++c) Ev[c] = (a.flags & ROWF_STATE_E) ? (T)st->E[c] : a.E[c];
  const long long nvox = (long long)a.n * a.nrows;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = a.n, h = a.h, ss = a.ss, d = a.d, R = a.rows_per_block;
  const int half_rows = R / 2;
  // split: this block holds one component (c_fix) of row block rb
  const long long rb = a.split ? (long long)(bx / d) : (long long)bx;
  const int c_fix = a.split ? (int)(bx - rb * d) : 0;
  const int npairs = (a.split ? 1 : d) * half_rows;
  cx<T>* Z = reinterpret_cast<cx<T>*>(smem_raw);
  size_t off = align16((size_t)npairs * ss * sizeof(cx<T>));
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw + off);
  off = align16(off + (size_t)twiddle_entries(n) * sizeof(cx<T>));
  uint8_t* phs = smem_raw + off;  // phase bytes of the block's rows (fused pass)
  off = align16(off + (size_t)R * n);
  T* cond = reinterpret_cast<T*>(smem_raw + off);
  const int tid = threadIdx.x;
  const long long row0 = rb * R;
  const int rows_here = (int)((a.nrows - row0) < R ? (a.nrows - row0) : R);
  // phase bytes of this block's rows (each read once, coalesced)
  const uint8_t* ph = phase + row0 * n;

  const int ntw = twiddle_entries(n);
  const T* csrc = a.cond + (long long)pb * kCondStride;

  // pair p: component c = p / half_rows, rows 2j and 2j+1 with j = p % half_rows
  // (split: component c_fix, rows 2p and 2p + 1)
  auto pair_comp = [&](int p) -> int { return a.split ? c_fix : (int)fdiv((uint32_t)p, a.fd_half); };
  auto pair_row = [&](int p) -> int {
    return a.split ? 2 * p : 2 * (p - (int)fdiv((uint32_t)p, a.fd_half) * half_rows);
  };

  if constexpr (MODE == ROW_FWD) {
    copy_batched<cx<T>, NT>(tw, a.tw, ntw);
    copy_batched<T, NT>(cond, csrc, a.n_phases);
    __syncthreads();
    if (a.tensor && (a.flags & ROWF_DL)) {
      // every component of a node at once (the block holds all of them)
      T shift[6];
      reference_shift(a, l0, shift);
      for (int idx = tid; idx < half_rows * n; idx += NT) {
        const int j = (int)fdiv((uint32_t)idx, a.fd_n);
        const int x = idx - j * n;
        T t[2][kMaxDim];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int rl = 2 * j + u;
          T v[kMaxDim] = {T(0), T(0), T(0)};
#pragma unroll
          for (int c = 0; c < kMaxDim; ++c) {
            t[u][c] = T(0);
            if (c < d && rl < rows_here)
              v[c] = (a.flags & ROWF_CONST_E) ? pick3(Ev, c) : (T)pick3(a.real_in, c)[(row0 + rl) * n + x];
          }
          if (rl < rows_here) tensor_times(cond, ph[rl * n + x], d, shift, v, t[u]);
        }
#pragma unroll
        for (int c = 0; c < kMaxDim; ++c)
          if (c < d) Z[(c * half_rows + j) * ss + x] = cx<T>{t[0][c], t[1][c]};
      }
      __syncthreads();
    } else {
    for (int idx = tid; idx < npairs * n; idx += NT) {
      const int p = (int)fdiv((uint32_t)idx, a.fd_n);
      const int x = idx - p * n;
      const int c = pair_comp(p);
      const int ra = pair_row(p);
      T v[2] = {T(0), T(0)};
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int rl = ra + u;
        if (rl >= rows_here) continue;
        // a batched problem without a warm start projects the zero field
        const double* rin = pe ? (pe->x0 ? pe->x0 + c * nvox : nullptr) : pick3(a.real_in, c);
        T val = (a.flags & ROWF_CONST_E) ? pick3(Ev, c) : (rin ? (T)rin[(row0 + rl) * n + x] : T(0));
        if (a.flags & ROWF_DL) val *= cond[ph[rl * n + x]] - l0;
        v[u] = val;
      }
      Z[p * ss + x] = cx<T>{v[0], v[1]};
    }
    __syncthreads();
    }
  } else {
    // Hermitian half rows of two rows -> one full complex row
    const int total = npairs * h;
    for (int base = 0; base < total; base += NT * kBatch) {
      cx<T> sa[kBatch], sb[kBatch];
      int pk[kBatch], kk[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int idx = base + u * NT + tid;
        sa[u] = cx<T>{T(0), T(0)};
        sb[u] = cx<T>{T(0), T(0)};
        pk[u] = -1;
        kk[u] = 0;
        if (idx < total) {
          int p, k;
          if (a.row_fast) {
            k = (int)fdiv((uint32_t)idx, a.fd_np);
            p = idx - k * npairs;
          } else {
            p = (int)fdiv((uint32_t)idx, a.fd_h);
            k = idx - p * h;
          }
          pk[u] = p;
          kk[u] = k;
          const int c = pair_comp(p);
          const int ra = pair_row(p);
          const cx<T>* sp = pick3(a.spec, c) + vo;
          if (ra < rows_here) sa[u] = sp[(row0 + ra) * a.rs_row + k * a.rs_k];
          if (ra + 1 < rows_here) sb[u] = sp[(row0 + ra + 1) * a.rs_row + k * a.rs_k];
        }
      }
      if (base == 0) {
        // the gate, the twiddles, the conductivities and (fused pass) the
        // phase bytes, requested while the first data chunk is in flight
        if (gated_out_stable(st, a.gate)) return;
        if constexpr (MODE == ROW_FUSED) {
          const int nph = rows_here * n;
          for (int i0 = tid; i0 < nph; i0 += 8 * NT) {
            uint8_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = i0 + u * NT < nph ? ph[i0 + u * NT] : (uint8_t)0;
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (i0 + u * NT < nph) phs[i0 + u * NT] = v[u];
          }
        }
        auto ldtw = [&](int i) -> cx<T> {
          if (i < ntw) {
            const cx<T>* q = a.tw + i;
            return cx<T>{q->re, q->im};
          }
          return cx<T>{T(0), T(0)};
        };
        const cx<T> tw0 = ldtw(tid);
        const cx<T> tw1 = ldtw(tid + NT);
        const T cd0 = tid < a.n_phases ? csrc[tid] : T(0);
        if (tid < ntw) tw[tid] = tw0;
        if (tid + NT < ntw) tw[tid + NT] = tw1;
        for (int i = tid + 2 * NT; i < ntw; i += NT) tw[i] = a.tw[i];
        if (tid < a.n_phases) cond[tid] = cd0;
        for (int i = tid + NT; i < a.n_phases; i += NT) cond[i] = csrc[i];
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        if (pk[u] < 0) continue;
        const int p = pk[u], k = kk[u];
        Z[p * ss + k] = cx<T>{sa[u].re - sb[u].im, sa[u].im + sb[u].re};
        if (k >= 1 && n - k >= h) Z[p * ss + n - k] = cx<T>{sa[u].re + sb[u].im, sb[u].re - sa[u].im};
      }
    }
    __syncthreads();
    fft_lds<T, +1, NT, RS>(Z, npairs, ss, a.plan, tw, tid);

    if constexpr (MODE == ROW_INV) {
      double acc[kMaxDim] = {0.0, 0.0, 0.0};
      if (a.tensor && (a.flags & (ROWF_LEFF | ROWF_DL_OUT))) {
        T shift[6], zero6[6];
        reference_shift(a, l0, shift);
#pragma unroll
        for (int i = 0; i < 6; ++i) zero6[i] = T(0);
        for (int idx = tid; idx < half_rows * n; idx += NT) {
          const int j = (int)fdiv((uint32_t)idx, a.fd_n);
          const int x = idx - j * n;
          cx<T> z[kMaxDim];
#pragma unroll
          for (int c = 0; c < kMaxDim; ++c) z[c] = c < d ? Z[(c * half_rows + j) * ss + x] : cx<T>{T(0), T(0)};
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int rl = 2 * j + u;
            if (rl >= rows_here) continue;
            const long long g = (row0 + rl) * n + x;
            const int q = ph[rl * n + x];
            T v[kMaxDim], w[kMaxDim];
#pragma unroll
            for (int c = 0; c < kMaxDim; ++c)
              v[c] = c < d ? (T)((double)pick3(Ev, c) + (double)((u == 0 ? z[c].re : z[c].im) * a.inv_n)) : T(0);
            if (a.flags & ROWF_DL_OUT) {
              tensor_times(cond, q, d, shift, v, w);
#pragma unroll
              for (int c = 0; c < kMaxDim; ++c) v[c] = w[c];
            }
#pragma unroll
            for (int c = 0; c < kMaxDim; ++c) {
              if (c >= d) continue;
              double val = (double)v[c];
              if (a.flags & ROWF_ADD) val += pick3(a.real_add, c)[g];
              v[c] = (T)val;
              double* out = pick3(a.real_out, c);
              if (out) out[g] = val;
            }
            if (a.flags & ROWF_LEFF) {
              tensor_times(cond, q, d, zero6, v, w);
#pragma unroll
              for (int c = 0; c < kMaxDim; ++c) acc[c] += (double)w[c];
            }
          }
        }
      } else {
      for (int idx = tid; idx < npairs * n; idx += NT) {
        const int p = (int)fdiv((uint32_t)idx, a.fd_n);
        const int x = idx - p * n;
        const int c = pair_comp(p);
        const int ra = pair_row(p);
        const cx<T> z = Z[p * ss + x];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int rl = ra + u;
          if (rl >= rows_here) continue;
          const long long g = (row0 + rl) * n + x;
          double val = (double)pick3(Ev, c) + (double)((u == 0 ? z.re : z.im) * a.inv_n);
          if (a.flags & ROWF_DL_OUT) val *= (double)cond[ph[rl * n + x]] - (double)l0;
          if (a.flags & ROWF_ADD) val += pick3(a.real_add, c)[g];
          double* out = pe ? (pe->e_out ? pe->e_out + c * nvox : nullptr) : pick3(a.real_out, c);
          if (out) out[g] = val;
          if (a.flags & ROWF_LEFF) {
            const double jv = (double)cond[ph[rl * n + x]] * val;
#pragma unroll
            for (int cc = 0; cc < kMaxDim; ++cc)
              if (cc == c) acc[cc] += jv;
          }
        }
      }
      }
      if (a.flags & ROWF_LEFF) {
        double* dst = parts.region(PART_AUX) + (long long)bx * 3;
        for (int c = 0; c < 3; ++c) store_partial<NT>(acc[c], dst + c);
      }
      return;
    }

    // ROW_FUSED: polarisation dL (E + u) at the nodes (Sec. 2.2, Eq. (17))
    if (a.tensor) {
      T shift[6];
      reference_shift(a, l0, shift);
      for (int idx = tid; idx < half_rows * n; idx += NT) {
        const int j = (int)fdiv((uint32_t)idx, a.fd_n);
        const int x = idx - j * n;
        T u0[kMaxDim], u1[kMaxDim], t0[kMaxDim], t1[kMaxDim];
#pragma unroll
        for (int c = 0; c < kMaxDim; ++c) {
          const cx<T> z = c < d ? Z[(c * half_rows + j) * ss + x] : cx<T>{T(0), T(0)};
          u0[c] = c < d ? pick3(Ev, c) + z.re * a.inv_n : T(0);
          u1[c] = c < d ? pick3(Ev, c) + z.im * a.inv_n : T(0);
          t0[c] = T(0);
          t1[c] = T(0);
        }
        if (2 * j < rows_here) tensor_times(cond, phs[2 * j * n + x], d, shift, u0, t0);
        if (2 * j + 1 < rows_here) tensor_times(cond, phs[(2 * j + 1) * n + x], d, shift, u1, t1);
#pragma unroll
        for (int c = 0; c < kMaxDim; ++c)
          if (c < d) Z[(c * half_rows + j) * ss + x] = cx<T>{t0[c], t1[c]};
      }
    } else
    for (int idx = tid; idx < npairs * n; idx += NT) {
      const int p = (int)fdiv((uint32_t)idx, a.fd_n);
      const int x = idx - p * n;
      const int c = pair_comp(p);
      const int ra = pair_row(p);
      const cx<T> z = Z[p * ss + x];
      T t0 = T(0), t1 = T(0);
      const T Ec = pick3(Ev, c);
      if (ra < rows_here) t0 = (cond[phs[ra * n + x]] - l0) * (Ec + z.re * a.inv_n);
      if (ra + 1 < rows_here) t1 = (cond[phs[(ra + 1) * n + x]] - l0) * (Ec + z.im * a.inv_n);
      Z[p * ss + x] = cx<T>{t0, t1};
    }
    __syncthreads();
  }

  fft_lds<T, -1, NT, RS>(Z, npairs, ss, a.plan, tw, tid);

  // split the two rows' spectra and store the half rows
  const int total = npairs * h;
  for (int idx = tid; idx < total; idx += NT) {
    int p, k;
    if (a.row_fast) {
      k = (int)fdiv((uint32_t)idx, a.fd_np);
      p = idx - k * npairs;
    } else {
      p = (int)fdiv((uint32_t)idx, a.fd_h);
      k = idx - p * h;
    }
    const int c = pair_comp(p);
    const int ra = pair_row(p);
    const cx<T> Y = Z[p * ss + k];
    const cx<T> Ym = Z[p * ss + (k == 0 ? 0 : n - k)];
    const T half = T(0.5);
    cx<T>* sp = pick3(a.spec, c) + vo;
    if (ra < rows_here)
      sp[(row0 + ra) * a.rs_row + k * a.rs_k] = cx<T>{(Y.re + Ym.re) * half, (Y.im - Ym.im) * half};
    if (ra + 1 < rows_here)
      sp[(row0 + ra + 1) * a.rs_row + k * a.rs_k] = cx<T>{(Y.im + Ym.im) * half, (Ym.re - Y.re) * half};
  }
}

// ---------------------------------------------------------------------------
// Strided-axis pass
// ---------------------------------------------------------------------------

template <typename T, int NT, int RS, int MODE>
__global__ __launch_bounds__(NT) void col_kernel(ColArgs<T> a) {
  // in the natural layout a tile reads C consecutive elements per transform
  // index; below one 128-byte line per segment, neighbouring tiles read the
  // halves or quarters of the same lines: XCD-aware order then.  (Tiles of the
  // transposed layout read whole columns and keep the dispatch order.)
  unsigned bx = blockIdx.x, by = blockIdx.y;
  if (a.sii == 1 && a.tile * (int)sizeof(cx<T>) < 128) xcd_order(bx, by);
  const int pb = a.bt.live ? a.bt.live[by] : (int)by;
  DevState* st = a.st + pb;
  // the direction step of the inverse pass reads its gate with the (r, r)
  // sums (block 0 of the same launch may set the flags); the other modes
  // see flags that only earlier launches write
  constexpr bool kInv = MODE == COL_INV_C || MODE == COL_INV_C_GEN;
  constexpr bool kGen = MODE == COL_INV_C_GEN || MODE == COL_FWD_PROJ_GEN;
  const bool pipe = kGen && a.pipe;
  const bool aniso = kGen && a.aniso;
  if (!(kInv && (a.cg_step || pipe)) && gated_out_stable(st, a.gate)) return;
  const ProbEntry* pe = a.bt.tab ? a.bt.tab + pb : nullptr;
  Partials parts = a.parts;
  parts.base += (long long)pb * a.bt.pstride;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  const int L = a.L, C = a.tile, ss = a.ss, d = a.d;
  const int nseq = d * C;
  cx<T>* Z = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw + align16((size_t)nseq * ss * sizeof(cx<T>)));
  copy_batched<cx<T>, NT>(tw, a.tw, twiddle_entries(L));

  const long long o = bx / a.tiles_per_outer;
  const long long i0 = (long long)(bx - o * a.tiles_per_outer) * C;
  const long long rem = a.inner - i0;
  const int width = rem < C ? (int)rem : C;
  // every array of problem pb starts vstride elements after that of pb - 1
  const long long base_o = (long long)pb * a.bt.vstride + o * (long long)L * a.inner;
  const cx<T> zero = {T(0), T(0)};
  // thread order over (l, c): c fastest in the natural layout, l fastest in
  // the transposed one, so that global accesses are contiguous
  const bool l_fast = a.sl == 1;
  auto split = [&](int idx, int& l, int& c) {
    if (l_fast) {
      c = (int)fdiv((uint32_t)idx, a.fd_L);
      l = idx - c * L;
    } else {
      l = (int)fdiv((uint32_t)idx, a.fd_C);
      c = idx - l * C;
    }
  };

  if constexpr (kInv) {
    double beta = 0.0;
    if (pipe) {
      if (!pipe_direction<NT>(st, parts, a.inv_n, a.gate, bx == 0)) return;
    } else if (a.cg_step && !cg_direction<NT>(st, parts, a.inv_n, &beta, a.gate, a.eq, bx == 0)) {
      return;
    }
    const T tb = (T)beta;
    const int total = L * C;
    for (int base = 0; base < total; base += NT * kBatch) {
      cx<T> rv[kBatch], pv[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int idx = base + u * NT + tid;
        rv[u] = zero;
        pv[u] = zero;
        if (idx < total) {
          int l, c;
          split(idx, l, c);
          if (c < width) {
            const long long g = base_o + l * a.sl + (i0 + c) * a.sii;
            if (a.cg_step) {
              rv[u] = a.r_in[g];
              pv[u] = a.p_io[g];
            } else {
              rv[u] = a.c_in[g];
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int idx = base + u * NT + tid;
        if (idx >= total) continue;
        int l, c;
        split(idx, l, c);
        if (c < width) {
          const long long g = base_o + l * a.sl + (i0 + c) * a.sii;
          cx<T> cv = rv[u];
          if (a.cg_step) {
            cv = cx<T>{rv[u].re + tb * pv[u].re, rv[u].im + tb * pv[u].im};
            a.p_io[g] = cv;
          }
          double kh[kMaxDim];
          const bool nz = khat_axis0(a, l, i0 + c, kh);
          const double sk = (aniso && nz) ? 1.0 / sqrt(sym_quad(a.L0n, a.dims, kh)) : 1.0;
#pragma unroll
          for (int al = 0; al < kMaxDim; ++al) {
            if (al >= d) break;
            const T k = nz ? (T)(kh[al] * sk) : T(0);
            Z[(al * C + c) * ss + l] = cx<T>{-k * cv.im, k * cv.re};  // i khat_a c
          }
        } else {
#pragma unroll
          for (int al = 0; al < kMaxDim; ++al)
            if (al < d) Z[(al * C + c) * ss + l] = zero;
        }
      }
    }
    __syncthreads();
    fft_lds<T, +1, NT, RS>(Z, nseq, ss, a.plan, tw, tid);
    for (int idx = tid; idx < L * C; idx += NT) {
      int l, c;
      split(idx, l, c);
      if (c < width) {
        const long long g = base_o + l * a.sl + (i0 + c) * a.sii;
#pragma unroll
        for (int al = 0; al < kMaxDim; ++al)
          if (al < d) a.comp[al][g] = Z[(al * C + c) * ss + l];
      }
    }
    return;
  }

  {
    // one component at a time, four loads in flight per thread (named
    // registers: a register array indexed here ended up in scratch)
    const int total = L * C;
    for (int al = 0; al < d; ++al) {
      const cx<T>* __restrict__ src = pick3(a.comp, al);
      auto ld = [&](int idx) -> cx<T> {
        if (idx < total) {
          int l, c;
          split(idx, l, c);
          if (c < width) {
            const cx<T>* q = src + base_o + l * a.sl + (i0 + c) * a.sii;
            return cx<T>{q->re, q->im};
          }
        }
        return zero;
      };
      auto st = [&](int idx, const cx<T>& v) {
        if (idx < total) {
          int l, c;
          split(idx, l, c);
          Z[(al * C + c) * ss + l] = v;
        }
      };
      for (int base = tid; base < total; base += NT * 4) {
        const cx<T> v0 = ld(base);
        const cx<T> v1 = ld(base + NT);
        const cx<T> v2 = ld(base + 2 * NT);
        const cx<T> v3 = ld(base + 3 * NT);
        st(base, v0);
        st(base + NT, v1);
        st(base + 2 * NT, v2);
        st(base + 3 * NT, v3);
      }
    }
  }
  __syncthreads();

  if constexpr (MODE == COL_PLAIN || MODE == COL_PLAIN_FWD) {
    fft_lds<T, MODE == COL_PLAIN ? +1 : -1, NT, RS>(Z, nseq, ss, a.plan, tw, tid);
    for (int al = 0; al < d; ++al) {
      cx<T>* __restrict__ dst = pick3(a.comp, al);
      for (int idx = tid; idx < L * C; idx += NT) {
        int l, c;
        split(idx, l, c);
        if (c < width) dst[base_o + l * a.sl + (i0 + c) * a.sii] = Z[(al * C + c) * ss + l];
      }
    }
  } else {
  // COL_FWD_PROJ
  fft_lds<T, -1, NT, RS>(Z, nseq, ss, a.plan, tw, tid);
  double acc = 0.0, acc_eq = 0.0;
  const int n_last = a.nd[a.dims - 1];
  const int total = L * C;
  const T cs = a.coef_s * (a.s_inv_l0 ? (T)(1.0 / (pe ? pe->l0 : a.l0)) : T(1));
  // pipelined CG: z = A w + beta z (beta of this iteration, set by the inverse pass)
  const T pbeta = pipe ? (T)st->pipe_beta[st->iter_u & 1] : T(0);
  for (int base = 0; base < total; base += NT * kBatch) {
    cx<T> bv[kBatch], zv[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int idx = base + u * NT + tid;
      bv[u] = zero;
      zv[u] = zero;
      if (idx < total) {
        int l, c;
        split(idx, l, c);
        if (c < width) {
          const long long g = base_o + l * a.sl + (i0 + c) * a.sii;
          if (a.base) bv[u] = a.base[g];
          if (pipe) zv[u] = a.out[g];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int idx = base + u * NT + tid;
      if (idx >= total) continue;
      int l, c;
      split(idx, l, c);
      if (c >= width) continue;
      const long long g = base_o + l * a.sl + (i0 + c) * a.sii;
      double kh[kMaxDim];
      double k2 = 0.0;
      const bool nz = khat_axis0(a, l, i0 + c, kh, &k2);
      double sk = 1.0;
      if (aniso && nz) {
        // the Green operator takes 1 / sqrt(q) like the inverse pass; the
        // plain projection of a field takes the inverse scale sqrt(q); the
        // equilibrium weight |xi|^2 becomes xi . L0n . xi
        const double q = sym_quad(a.L0n, a.dims, kh);
        sk = a.s_inv_l0 ? 1.0 / sqrt(q) : sqrt(q);
        k2 *= q;
      }
      if (a.eq && l == 0 && i0 + c == 0) {
        // k = 0: the cell sum of the transformed field (dL (E + u) or dL u)
        double* dst = a.dot == 1 ? st->taup : st->jx;
#pragma unroll
        for (int al = 0; al < kMaxDim; ++al) dst[al] = al < d ? (double)Z[(al * C + c) * ss + l].re : 0.0;
      }
      cx<T> t = zero;
      if (nz) {
#pragma unroll
        for (int al = 0; al < kMaxDim; ++al) {
          if (al >= d) break;
          const cx<T> v = Z[(al * C + c) * ss + l];
          const T k = (T)(kh[al] * sk);
          t.re += k * v.re;
          t.im += k * v.im;
        }
      }
      // s = -i khat . tau_hat
      cx<T> val = {cs * t.im, -cs * t.re};
      const cx<T> b = bv[u];
      val.re += a.coef_base * b.re;
      val.im += a.coef_base * b.im;
      if (pipe) {
        val.re += pbeta * zv[u].re;
        val.im += pbeta * zv[u].im;
      }
      a.out[g] = val;
      if (a.dot) {
        const uint32_t kl = (uint32_t)(i0 + c);
        const double w = half_weight(kl - fdiv(kl, a.fd_h) * (uint32_t)a.h, n_last);
        if (a.dot == 1) {
          acc += w * ((double)b.re * (double)val.re + (double)b.im * (double)val.im);
        } else {
          // dot 2: |out|^2; dot 3: the step |out - base|^2 of the basic scheme
          const double dr = a.dot == 3 ? (double)val.re - (double)b.re : (double)val.re;
          const double di = a.dot == 3 ? (double)val.im - (double)b.im : (double)val.im;
          const double m2 = dr * dr + di * di;
          acc += w * m2;
          if (a.eq) acc_eq += w * k2 * m2;
        }
      }
    }
  }
  if (a.dot) {
    if (a.eq && a.dot != 1) {
      double v[2] = {acc, acc_eq};
      (void)block_sums_gated<NT, 2>(v, 0);
      if (tid == 0) {
        parts.region(a.dot_region)[bx] = v[0];
        parts.region(a.eq_region)[bx] = v[1];
      }
    } else {
      store_partial<NT>(acc, parts.region(a.dot_region) + bx);
    }
    if (a.dot_region == PART_RR0 && bx == 0 && tid == 0) st->nparts[0] = (int)gridDim.x;
    if (a.dot_region == PART_PQ && bx == 0 && tid == 0) st->nparts_pq = (int)gridDim.x;
  }
  }
}

// |xi|^2 (xi = k / Y) of half-spectrum entry i, or xi . L0n . xi for an
// anisotropic reference: 2-D arrays are stored [k1][k0] (kq = i / N0 is k1),
// 3-D arrays [k0][k1][k2] (kq = i).
template <typename T>
__device__ __forceinline__ double spectral_k2(const UpdArgs<T>& a, uint32_t i, uint32_t kq, uint32_t k_last) {
  int k0, k1;
  if (a.dims == 2) {
    k0 = (int)(i - kq * (uint32_t)a.nd[0]);
    k1 = 0;
  } else {
    const uint32_t rest = fdiv(kq, a.fd_h);
    const uint32_t i0 = fdiv(rest, a.fd_n1);
    k1 = freq_of((int)(rest - i0 * (uint32_t)a.nd[1]), a.nd[1]);
    k0 = (int)i0;
  }
  k0 = freq_of(k0, a.nd[0]);
  const int last = a.dims - 1;
  const double x0 = (double)k0 * a.cinv[0];
  const double x1 = a.dims == 2 ? 0.0 : (double)k1 * a.cinv[1];
  const double xl = (double)k_last * a.cinv[last];
  if (a.aniso) {
    const double xs[kMaxDim] = {x0, a.dims == 2 ? xl : x1, xl};
    return sym_quad(a.L0n, a.dims, xs);
  }
  return x0 * x0 + x1 * x1 + xl * xl;
}

// Weight of entry i of a vector in the wave-pass layout V
// (((b G + cg) 8 + cc) N0 + a; the last-axis column is c = 8 cg + cc, the
// last axis odd): 1 for c = 0, 2 below h, 0 on the padding.
__device__ __forceinline__ double w3_entry_weight(uint32_t i, const FastDiv& fd_n0, int G, int h) {
  const uint32_t col = fdiv(i, fd_n0);           // (b G + cg) 8 + cc
  const uint32_t cc = col & 7u;
  const uint32_t bg = col >> 3;                   // b G + cg
  const uint32_t cg = bg - (bg / (uint32_t)G) * (uint32_t)G;
  const uint32_t c = cg * 8u + cc;
  return c == 0 ? 1.0 : (c < (uint32_t)h ? 2.0 : 0.0);
}

// ---------------------------------------------------------------------------
// CG update: alpha = (r, r) / (p, q); x += alpha p, r -= alpha q, (r, r)
// ---------------------------------------------------------------------------

// EQ: the equilibrium sums ride along (a.eq); the plain kernel has no code for them.
// DEFER: x is neither read nor written; the lead records that the next
// direction step owes x += alpha p (alpha_log, x_pend).
// The deferred variant runs 512 threads per block: the same 512 partials,
// twice the loads in flight (FP32 at 243^3: 44 -> 35.5 us).
template <typename T, bool EQ, bool DEFER>
__global__ __launch_bounds__(DEFER ? 512 : 256) void update_kernel(UpdArgs<T> a) {
  constexpr int NT = DEFER ? 512 : 256;
  // loads in flight per thread: the deferred FP32 update (two vectors of
  // half-size entries) takes twice as many; the others would lose occupancy
  constexpr int UB = (sizeof(T) == 4 && DEFER) ? 2 * kBatch : kBatch;
  const int pb = batch_prob(a.bt);
  DevState* st = a.st + pb;
  Partials parts = a.parts;
  parts.base += (long long)pb * a.bt.pstride;
  const long long vo = (long long)pb * a.bt.vstride;
  const cx<T>* __restrict__ P = a.p + vo;
  const cx<T>* __restrict__ Q = a.q + vo;
  cx<T>* __restrict__ X = a.x + vo;
  cx<T>* __restrict__ Rv = a.r + vo;
  const long long stride = (long long)gridDim.x * NT;
  cx<T> p[UB], q[UB], x[UB], r[UB];
  auto load = [&](long long base) {
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const long long i = base + u * stride;
      if (i < a.n) {
        if constexpr (!DEFER) {
          p[u] = P[i];
          x[u] = X[i];
        }
        if constexpr (DEFER && sizeof(T) == 8) {
          // q is not read again in the iteration: streamed, it leaves the
          // cache to r, which the next pass reads (FP64 at 243^3: that pass
          // 150 -> 143 us; with the half-size FP32 vectors no gain)
          typedef T v2 __attribute__((ext_vector_type(2)));
          const v2 t = __builtin_nontemporal_load(reinterpret_cast<const v2*>(Q + i));
          q[u] = cx<T>{t.x, t.y};
        } else {
          q[u] = Q[i];
        }
        r[u] = Rv[i];
      }
    }
  };
  // a problem finished by an earlier launch returns before any load; the
  // first chunk of vectors does not depend on alpha and is requested before
  // the scalar sums, so its latency overlaps their reduction
  if (gated_out_stable(st, a.gate)) return;
  const long long first = (long long)blockIdx.x * NT + threadIdx.x;
  load(first);
  // gate, iteration index and both sums in one reduction (block 0 of this
  // launch sets the done flag on a breakdown)
  const int skip0 = gate_flags(st, a.gate);
  const int k = st->iter_u;
  double sums[2] = {partial_share<NT>(parts.region(k & 1), st->nparts[k & 1]),
                    partial_share<NT>(parts.region(PART_PQ), st->nparts_pq)};
  if (block_sums_gated<NT, 2>(sums, skip0)) return;
  const double rr = sums[0] * a.inv_n;
  const double pq = sums[1] * a.inv_n;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (lead) {
      st->pq_log = pq;
      st->status = -6;
      st->done = 1;
    }
    return;
  }
  const double alpha = rr / pq;
  const T ta = (T)alpha;
  double acc = 0.0, acc_eq = 0.0;
  for (long long i0 = first; i0 < a.n; i0 += stride * UB) {
    if (i0 != first) load(i0);
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const long long i = i0 + u * stride;
      if (i >= a.n) continue;
      if constexpr (!DEFER) {
        x[u].re += ta * p[u].re;
        x[u].im += ta * p[u].im;
        X[i] = x[u];
      }
      r[u].re -= ta * q[u].re;
      r[u].im -= ta * q[u].im;
      Rv[i] = r[u];
      const double m2 = (double)r[u].re * (double)r[u].re + (double)r[u].im * (double)r[u].im;
      if (a.w3) {
        acc += w3_entry_weight((uint32_t)i, a.fd_w3n0, a.w3g, a.h) * m2;
      } else {
        const uint32_t kq = fdiv((uint32_t)i, a.fd_kd);
        const uint32_t k_last = kq - fdiv(kq, a.fd_h) * (uint32_t)a.h;
        const double w = half_weight(k_last, a.n_last);
        acc += w * m2;
        if constexpr (EQ) acc_eq += w * spectral_k2(a, (uint32_t)i, kq, k_last) * m2;
      }
    }
  }
  const int nxt = (k + 1) & 1;
  if constexpr (EQ) {
    double v[2] = {acc, acc_eq};
    (void)block_sums_gated<NT, 2>(v, 0);
    if (threadIdx.x == 0) {
      parts.region(nxt)[blockIdx.x] = v[0];
      parts.region(PART_EQ0 + nxt)[blockIdx.x] = v[1];
    }
  } else {
    store_partial<NT>(acc, parts.region(nxt) + blockIdx.x);
  }
  if (lead) {
    st->nparts[nxt] = (int)gridDim.x;
    st->iter_a = k + 1;
    st->alpha_log = alpha;
    st->pq_log = pq;
    if constexpr (DEFER) st->x_pend = 1;
    // cell sum of dL (E + u(x)) follows x += alpha p linearly
    if constexpr (EQ)
      for (int c = 0; c < kMaxDim; ++c) st->jx[c] += alpha * st->taup[c];
  }
}

// ---------------------------------------------------------------------------
// Pipelined CG update: s = w + beta s, p = r + beta p, x += alpha p,
// r -= alpha s, w -= alpha z; (r, r) and (w, r) of the new iterate in one
// reduction (the only one of the iteration)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void pipe_update_kernel(PipeArgs<double> a) {
  constexpr int NT = 256;
  const int pb = batch_prob(a.bt);
  DevState* st = a.st + pb;
  if (gated_out(st, a.gate)) return;
  Partials parts = a.parts;
  parts.base += (long long)pb * a.bt.pstride;
  const long long vo = (long long)pb * a.bt.vstride;
  const int k = st->iter_u;
  const double alpha = st->pipe_alpha[k & 1];
  const double beta = st->pipe_beta[k & 1];
  cx<double>* __restrict__ X = a.x + vo;
  cx<double>* __restrict__ Rv = a.r + vo;
  cx<double>* __restrict__ P = a.p + vo;
  cx<double>* __restrict__ W = a.w + vo;
  cx<double>* __restrict__ S = a.s + vo;
  const cx<double>* __restrict__ Z = a.z + vo;
  double acc_rr = 0.0, acc_wr = 0.0;
  const long long stride = (long long)gridDim.x * NT;
  for (long long i0 = (long long)blockIdx.x * NT + threadIdx.x; i0 < a.n; i0 += stride * 2) {
    cx<double> x[2], r[2], p[2], w[2], sv[2], z[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const long long i = i0 + u * stride;
      if (i < a.n) {
        x[u] = X[i];
        r[u] = Rv[i];
        p[u] = P[i];
        w[u] = W[i];
        sv[u] = S[i];
        z[u] = Z[i];
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const long long i = i0 + u * stride;
      if (i >= a.n) continue;
      sv[u] = cx<double>{w[u].re + beta * sv[u].re, w[u].im + beta * sv[u].im};
      p[u] = cx<double>{r[u].re + beta * p[u].re, r[u].im + beta * p[u].im};
      x[u].re += alpha * p[u].re;
      x[u].im += alpha * p[u].im;
      r[u].re -= alpha * sv[u].re;
      r[u].im -= alpha * sv[u].im;
      w[u].re -= alpha * z[u].re;
      w[u].im -= alpha * z[u].im;
      X[i] = x[u];
      Rv[i] = r[u];
      P[i] = p[u];
      W[i] = w[u];
      S[i] = sv[u];
      const uint32_t kq = fdiv((uint32_t)i, a.fd_kd);
      const double wt = half_weight(kq - fdiv(kq, a.fd_h) * (uint32_t)a.h, a.n_last);
      acc_rr += wt * (r[u].re * r[u].re + r[u].im * r[u].im);
      acc_wr += wt * (w[u].re * r[u].re + w[u].im * r[u].im);
    }
  }
  const int nxt = (k + 1) & 1;
  double v[2] = {acc_rr, acc_wr};
  (void)block_sums_gated<NT, 2>(v, 0);
  if (threadIdx.x == 0) {
    parts.region(nxt)[blockIdx.x] = v[0];
    parts.region(PART_PQ)[blockIdx.x] = v[1];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->nparts[nxt] = (int)gridDim.x;
    st->nparts_pq = (int)gridDim.x;
    st->iter_a = k + 1;
    st->alpha_log = alpha;
  }
}

// ---------------------------------------------------------------------------
// Mixed precision helpers
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void mix_accumulate_kernel(MixArgs a) {
  const int pb = batch_prob(a.bt);
  if (gated_out(a.st + pb, a.gate)) return;
  const long long vo = (long long)pb * a.bt.vstride;
  const long long stride = (long long)gridDim.x * 256;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < a.n; i += stride) {
    const cx<float> y = a.x32[vo + i];
    cx<double> x = a.x64[vo + i];
    x.re += (double)y.re;
    x.im += (double)y.im;
    a.x64[vo + i] = x;
    a.x32[vo + i] = cx<float>{0.f, 0.f};
  }
}

__global__ __launch_bounds__(256) void mix_convert_kernel(MixArgs a) {
  const int pb = batch_prob(a.bt);
  DevState* st = a.st + pb;
  if (gated_out(st, a.gate)) return;
  Partials parts = a.parts;
  parts.base += (long long)pb * a.bt.pstride;
  const long long vo = (long long)pb * a.bt.vstride;
  const int k = st->iter_a;
  double acc = 0.0;
  const long long stride = (long long)gridDim.x * 256;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < a.n; i += stride) {
    const cx<double> r = a.r64[vo + i];
    const cx<float> f = cx<float>{(float)r.re, (float)r.im};
    a.r32[vo + i] = f;
    double w;
    if (a.w3) {
      w = w3_entry_weight((uint32_t)i, a.fd_w3n0, a.w3g, a.h);
    } else {
      const uint32_t kq = fdiv((uint32_t)i, a.fd_kd);
      w = half_weight(kq - fdiv(kq, a.fd_h) * (uint32_t)a.h, a.n_last);
    }
    acc += w * ((double)f.re * (double)f.re + (double)f.im * (double)f.im);
  }
  store_partial<256>(acc, parts.region(k & 1) + blockIdx.x);
  if (blockIdx.x == 0 && threadIdx.x == 0) st->nparts[k & 1] = (int)gridDim.x;
}

// ---------------------------------------------------------------------------
// BiCG elementwise steps (one partial per block, fixed-order sums)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void bicg_kernel(BicgArgs a) {
  constexpr int NT = 256;
  DevState* st = a.st;
  if (gated_out(st, a.gate)) return;
  const long long total = a.n * a.d;
  const long long stride = (long long)gridDim.x * NT;
  const long long i0 = (long long)blockIdx.x * NT + threadIdx.x;
  if (a.mode == BV_LEFF) {
    double acc[kMaxDim] = {0.0, 0.0, 0.0};
    if (a.tensor) {
      const double zero6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (long long j = i0; j < a.n; j += stride) {
        double v[kMaxDim], w[kMaxDim];
#pragma unroll
        for (int c = 0; c < kMaxDim; ++c) v[c] = c < a.d ? a.x[(long long)c * a.n + j] : 0.0;
        tensor_times(a.cond, a.phase[j], a.d, zero6, v, w);
#pragma unroll
        for (int c = 0; c < kMaxDim; ++c) acc[c] += w[c];
      }
    } else {
      for (int c = 0; c < a.d; ++c) {
        const double* xc = a.x + (long long)c * a.n;
        double s = 0.0;
        for (long long j = i0; j < a.n; j += stride) s += a.cond[a.phase[j]] * xc[j];
        acc[c] = s;
      }
    }
    double* dst = a.parts.region(PART_AUX) + (long long)blockIdx.x * 3;
    for (int c = 0; c < 3; ++c) store_partial<NT>(acc[c], dst + c);
    return;
  }
  double s0 = 0.0, s1 = 0.0;
  const double alpha = a.mode == BV_UPDATE ? st->bicg_alpha : 0.0;
  const double beta = a.mode == BV_DIRECTION ? st->bicg_beta : 0.0;
  for (long long i = i0; i < total; i += stride) {
    switch (a.mode) {
      case BV_FILL_E: {
        const int c = (int)fdiv((uint32_t)i, a.fd_n);
        a.x[i] = st->E[c];
        break;
      }
      case BV_START: {
        const int c = (int)fdiv((uint32_t)i, a.fd_n);
        const double r = st->E[c] - a.ap[i];
        a.r[i] = r;
        a.rs[i] = r;
        a.p[i] = r;
        a.ps[i] = r;
        s0 += r * r;
        s1 += r * r;
        break;
      }
      case BV_DOT_APP:
        s0 += a.ap[i] * a.ps[i];
        break;
      case BV_UPDATE: {
        a.x[i] += alpha * a.p[i];
        const double r = a.r[i] - alpha * a.ap[i];
        const double rs = a.rs[i] - alpha * a.atp[i];
        a.r[i] = r;
        a.rs[i] = rs;
        s0 += r * rs;
        s1 += r * r;
        break;
      }
      case BV_DIRECTION:
        a.p[i] = a.r[i] + beta * a.p[i];
        a.ps[i] = a.rs[i] + beta * a.ps[i];
        break;
      case BV_RESID: {
        const int c = (int)fdiv((uint32_t)i, a.fd_n);
        const double r = st->E[c] - a.ap[i];
        s0 += r * r;
        break;
      }
      default:
        break;
    }
  }
  if (a.mode == BV_START || a.mode == BV_UPDATE) {
    double v[2] = {s0, s1};
    (void)block_sums_gated<NT, 2>(v, 0);
    if (threadIdx.x == 0) {
      double* dst = a.parts.region(PART_AUX) + (long long)blockIdx.x * 3;
      dst[0] = v[0];
      dst[1] = v[1];
    }
  } else if (a.mode == BV_DOT_APP) {
    store_partial<NT>(s0, a.parts.region(PART_PQ) + blockIdx.x);
  } else if (a.mode == BV_RESID) {
    store_partial<NT>(s0, a.parts.region(PART_AUX) + blockIdx.x);
  }
}

// ---------------------------------------------------------------------------
// Single-block scalar steps
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void finalize_kernel(FinArgs a) {
  constexpr int NT = 256;
  const int pb = batch_prob(a.bt);
  DevState* st = a.st + pb;
  if (gated_out(st, a.gate)) return;
  Partials parts = a.parts;
  parts.base += (long long)pb * a.bt.pstride;
  const bool lead = threadIdx.x == 0;
  switch (a.mode) {
    case FZ_CHECK: {
      const int m = st->iter_a;
      const double rr = sum_partials<NT>(parts.region(m & 1), st->nparts[m & 1]) * a.inv_n;
      bool conv = rr <= st->tol2b2;
      if (a.eq) {
        const double eqs = sum_partials<NT>(parts.region(PART_EQ0 + (m & 1)), st->nparts[m & 1]);
        const bool eq_ok = equilibrium_test(st, m, rr, eqs, lead);
        if (st->norm == 1) conv = eq_ok;
      }
      if (lead) {
        st->rr_log = rr;
        if (!isfinite(rr)) {
          st->status = -6;
          st->done = 1;
        } else if (conv) {
          st->done = 1;
        } else if (m >= st->max_iter) {
          st->status = -5;
          st->done = 1;
        }
      }
      break;
    }
    case FZ_AUX: {
      const double s = sum_partials<NT>(parts.region(PART_AUX), a.n) * a.inv_n;
      if (lead) st->dot_aux = s;
      break;
    }
    case FZ_RR_TRUE: {
      const double s = sum_partials<NT>(parts.region(PART_AUX), a.n) * a.inv_n;
      if (a.eq) (void)equilibrium_test(st, -1, s, sum_partials<NT>(parts.region(PART_EQ0), a.n), lead);
      if (lead) st->rr_true = s;
      break;
    }
    case FZ_BICG_START:
    case FZ_BICG_STEP: {
      const double rho = sum_partials<NT>(parts.region(PART_AUX), a.n, 3);
      const double rr = sum_partials<NT>(parts.region(PART_AUX) + 1, a.n, 3);
      if (lead) {
        const int m = st->iter_a + (a.mode == FZ_BICG_STEP ? 1 : 0);
        st->iter_a = m;
        st->rr_log = rr;
        if (a.mode == FZ_BICG_STEP) st->bicg_beta = rho / st->bicg_rho;
        st->bicg_rho = rho;
        if (!isfinite(rr) || !isfinite(rho)) {
          st->status = -6;
          st->done = 1;
        } else if (rr <= st->tol2b2) {
          st->done = 1;
        } else if (m >= st->max_iter) {
          st->status = -5;
          st->done = 1;
        } else if (rho == 0.0) {
          st->status = -6;
          st->done = 1;
        }
      }
      break;
    }
    case FZ_BICG_ALPHA: {
      const double sigma = sum_partials<NT>(parts.region(PART_PQ), a.n);
      if (lead) {
        if (!(sigma != 0.0) || !isfinite(sigma)) {
          st->status = -6;
          st->done = 1;
        } else {
          st->bicg_alpha = st->bicg_rho / sigma;
        }
      }
      break;
    }
    case FZ_FFTH: {
      // iterate m was transformed into m + 1; the step is its residual
      const int m = st->iter_a;
      // the step's producer set nparts[0] (a wide one had its partials folded)
      const double rr = sum_partials<NT>(parts.region(PART_RR0), st->nparts[0]) * a.inv_n;
      bool conv = rr <= st->tol2b2;
      if (a.eq) {
        const bool eq_ok =
            equilibrium_test(st, m, rr, sum_partials<NT>(parts.region(PART_EQ0), st->nparts[0]), lead);
        if (st->norm == 1) conv = eq_ok;
      }
      if (lead) {
        st->rr_log = rr;
        st->iter_a = m + 1;
        st->iter_u = m;
        if (!isfinite(rr)) {
          st->status = -6;
          st->done = 1;
        } else if (conv) {
          st->done = 1;
        } else if (m + 1 >= st->max_iter) {
          st->status = -5;
          st->done = 1;
        }
      }
      break;
    }
    case FZ_LEFF: {
      for (int c = 0; c < a.d; ++c) {
        const double s = sum_partials<NT>(parts.region(PART_AUX) + c, a.n, 3) * a.inv_n;
        if (lead) st->leff[c] = s;
      }
      break;
    }
    case FZ_REFRESH:
    case FZ_REFRESH_INIT: {
      const double rr = sum_partials<NT>(parts.region(PART_AUX), a.n) * a.inv_n;
      if (lead) {
        st->rr_true = rr;
        st->rr_ref = rr;
        st->rr_log = rr;
        st->k_ref = st->iter_a;
        if (a.mode == FZ_REFRESH) st->n_refresh += 1;
        st->refresh = 0;
        if (!isfinite(rr)) {
          st->status = -6;
          st->done = 1;
        } else if (rr <= st->tol2b2) {
          st->done = 1;
        } else if (st->iter_a >= st->max_iter) {
          st->status = -5;
          st->done = 1;
        }
      }
      break;
    }
    default:
      break;
  }
}

__global__ void state_init_kernel(DevState* st, DevState init) { *st = init; }

// One block: a running count over chunks of 256 problems (ballots per wave,
// wave totals in LDS), so the list keeps index order.
__global__ __launch_bounds__(256) void compact_live_kernel(const DevState* st, int nprob, int rows, int* live) {
  __shared__ int wsum[2][4];
  __shared__ int first_done;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) first_done = nprob;
  __syncthreads();
  int base_live = 0, base_done = 0;
  for (int c0 = 0; c0 < nprob; c0 += 256) {
    const int i = c0 + tid;
    const bool in = i < nprob;
    const bool act = in && st[i].done == 0;
    const bool dn = in && !act;
    const unsigned long long ba = __ballot(act), bd = __ballot(dn);
    const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
    if (lane == 0) {
      wsum[0][w] = __popcll(ba);
      wsum[1][w] = __popcll(bd);
    }
    __syncthreads();
    int off_a = base_live, off_d = base_done, tot_a = 0, tot_d = 0;
    for (int k = 0; k < 4; ++k) {
      if (k < w) {
        off_a += wsum[0][k];
        off_d += wsum[1][k];
      }
      tot_a += wsum[0][k];
      tot_d += wsum[1][k];
    }
    if (act) {
      const int pos = off_a + __popcll(ba & below);
      if (pos < rows) live[pos] = i;
    }
    if (dn && off_d + __popcll(bd & below) == 0) first_done = i;
    base_live += tot_a;
    base_done += tot_d;
    __syncthreads();
  }
  // fill the remaining rows with a done problem (its blocks return at entry)
  const int fill = first_done < nprob ? first_done : 0;
  for (int r = base_live + tid; r < rows; r += 256) live[r] = fill;
}

__global__ __launch_bounds__(256) void state_copy_kernel(DevState* st, const DevState* src, int nprob) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < nprob) st[i] = src[i];
}

template <typename T>
__global__ __launch_bounds__(256) void fill_zero_kernel(cx<T>* p, long long n) {
  const long long stride = (long long)gridDim.x * 256;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
    p[i] = cx<T>{T(0), T(0)};
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

int lds_odd_stride(int n) { return (n & 1) ? n : n + 1; }

static int nprob_of(const Batch& b) { return b.nprob > 1 ? b.nprob : 1; }

hipError_t launch_compact_live(const DevState* st, int nprob, int rows, int* live, hipStream_t s) {
  hipLaunchKernelGGL(compact_live_kernel, dim3(1), dim3(256), 0, s, st, nprob, rows, live);
  return hipGetLastError();
}

long long bicg_blocks(const BicgArgs& a) { return update_blocks(a.n * a.d); }

hipError_t launch_bicg(const BicgArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(bicg_kernel, dim3((unsigned)bicg_blocks(a)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_state_copy(DevState* st, const DevState* src, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(state_copy_kernel, dim3((unsigned)((nprob + 255) / 256)), dim3(256), 0, s, st, src, nprob);
  return hipGetLastError();
}

size_t row_lds_bytes(int n, int rows_per_block, int comps, int elem_bytes, int n_phases, int* ss_out) {
  const int ss = lds_odd_stride(n);
  if (ss_out) *ss_out = ss;
  const int npairs = comps * (rows_per_block / 2);
  size_t off = align16((size_t)npairs * ss * elem_bytes);
  off = align16(off + (size_t)twiddle_entries(n) * elem_bytes);
  off = align16(off + (size_t)rows_per_block * n);  // phase bytes
  return off + (size_t)n_phases * (size_t)(elem_bytes / 2);
}

size_t col_lds_bytes(int L, int tile, int d, int elem_bytes, int* ss_out) {
  const int ss = lds_odd_stride(L);
  if (ss_out) *ss_out = ss;
  return align16((size_t)d * tile * ss * elem_bytes) + (size_t)twiddle_entries(L) * elem_bytes;
}

template <typename T>
long long row_blocks(const RowArgs<T>& a) {
  return (a.split ? a.d : 1) * ((a.nrows + a.rows_per_block - 1) / a.rows_per_block);
}

template <typename T>
long long col_blocks(const ColArgs<T>& a) {
  return a.outer * (long long)a.tiles_per_outer;
}

long long update_blocks(long long n) {
  long long b = (n + 255) / 256;
  return b > kUpdateBlocks ? kUpdateBlocks : (b < 1 ? 1 : b);
}

// Block size: 128 threads when the batch fits their butterfly capacity.
static int pick_threads(int points, const FftPlan& plan) {
  return points <= plan_batch_cap(plan, 128) ? 128 : 256;
}

// Largest phase index of a phase image (validation at workspace set-up).
__global__ __launch_bounds__(256) void max_phase_kernel(const uint8_t* ph, long long n, unsigned* out) {
  unsigned m = 0;
  const long long stride = (long long)gridDim.x * 256;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) m = max(m, (unsigned)ph[i]);
  for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_down((int)m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

hipError_t launch_max_phase(const uint8_t* ph, long long n, unsigned* out, hipStream_t s) {
  hipLaunchKernelGGL(max_phase_kernel, dim3((unsigned)update_blocks(n)), dim3(256), 0, s, ph, n, out);
  return hipGetLastError();
}

// Node count of every phase index (256 bins): block counts in LDS, then one
// global atomic add per bin and block.  counts must be zero on entry.
__global__ __launch_bounds__(256) void phase_histogram_kernel(const uint8_t* ph, long long n, unsigned* counts) {
  __shared__ unsigned bins[256];
  bins[threadIdx.x] = 0u;
  __syncthreads();
  const long long stride = (long long)gridDim.x * 256;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) atomicAdd(&bins[ph[i]], 1u);
  __syncthreads();
  if (bins[threadIdx.x]) atomicAdd(&counts[threadIdx.x], bins[threadIdx.x]);
}

hipError_t launch_phase_histogram(const uint8_t* ph, long long n, unsigned* counts, hipStream_t s) {
  hipLaunchKernelGGL(phase_histogram_kernel, dim3((unsigned)update_blocks(n)), dim3(256), 0, s, ph, n, counts);
  return hipGetLastError();
}

// One kernel symbol per (precision, block size, radix set, pass mode): the
// compiler specialises each mode, and profiles attribute time per pass.
template <typename T, int RS, int MODE>
static void launch_row_m(const RowArgs<T>& a, size_t lds, long long nb, int nt, hipStream_t s) {
  const dim3 grid((unsigned)nb, (unsigned)nprob_of(a.bt));
  if (nt == 128)
    hipLaunchKernelGGL((row_kernel<T, 128, RS, MODE>), grid, dim3(128), lds, s, a);
  else
    hipLaunchKernelGGL((row_kernel<T, 256, RS, MODE>), grid, dim3(256), lds, s, a);
}

template <typename T, int RS>
static void launch_row_rs(const RowArgs<T>& a, size_t lds, long long nb, int nt, hipStream_t s) {
  if (a.mode == ROW_FUSED) launch_row_m<T, RS, ROW_FUSED>(a, lds, nb, nt, s);
  else if (a.mode == ROW_INV) launch_row_m<T, RS, ROW_INV>(a, lds, nb, nt, s);
  else launch_row_m<T, RS, ROW_FWD>(a, lds, nb, nt, s);
}

template <typename T, int RS, int MODE>
static void launch_col_m(const ColArgs<T>& a, size_t lds, long long nb, int nt, hipStream_t s) {
  const dim3 grid((unsigned)nb, (unsigned)nprob_of(a.bt));
  if (nt == 128)
    hipLaunchKernelGGL((col_kernel<T, 128, RS, MODE>), grid, dim3(128), lds, s, a);
  else
    hipLaunchKernelGGL((col_kernel<T, 256, RS, MODE>), grid, dim3(256), lds, s, a);
}

template <typename T, int RS>
static void launch_col_rs(const ColArgs<T>& a, size_t lds, long long nb, int nt, hipStream_t s) {
  const bool gen = a.aniso || a.pipe;
  if (a.mode == COL_INV_C && gen) launch_col_m<T, RS, COL_INV_C_GEN>(a, lds, nb, nt, s);
  else if (a.mode == COL_INV_C) launch_col_m<T, RS, COL_INV_C>(a, lds, nb, nt, s);
  else if (a.mode == COL_PLAIN && a.dir > 0) launch_col_m<T, RS, COL_PLAIN>(a, lds, nb, nt, s);
  else if (a.mode == COL_PLAIN) launch_col_m<T, RS, COL_PLAIN_FWD>(a, lds, nb, nt, s);
  else if (gen) launch_col_m<T, RS, COL_FWD_PROJ_GEN>(a, lds, nb, nt, s);
  else launch_col_m<T, RS, COL_FWD_PROJ>(a, lds, nb, nt, s);
}

template <typename T>
hipError_t launch_row(const RowArgs<T>& a, hipStream_t s) {
  const int comps = a.split ? 1 : a.d;
  const size_t lds = row_lds_bytes(a.n, a.rows_per_block, comps, (int)sizeof(cx<T>), a.n_phases, nullptr);
  const long long nb = row_blocks(a);
  const int nt = a.nt ? a.nt : pick_threads(comps * (a.rows_per_block / 2) * a.n, a.plan);
  switch (plan_radix_set(a.plan)) {
    case RADIX_POW3: launch_row_rs<T, RADIX_POW3>(a, lds, nb, nt, s); break;
    case RADIX_POW2: launch_row_rs<T, RADIX_POW2>(a, lds, nb, nt, s); break;
    case RADIX_WIDE: launch_row_rs<T, RADIX_WIDE>(a, lds, nb, nt, s); break;
    default: launch_row_rs<T, RADIX_ALL>(a, lds, nb, nt, s); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col(const ColArgs<T>& a, hipStream_t s) {
  const size_t lds = col_lds_bytes(a.L, a.tile, a.d, (int)sizeof(cx<T>), nullptr);
  const long long nb = col_blocks(a);
  const int nt = a.nt ? a.nt : pick_threads(a.d * a.tile * a.L, a.plan);
  switch (plan_radix_set(a.plan)) {
    case RADIX_POW3: launch_col_rs<T, RADIX_POW3>(a, lds, nb, nt, s); break;
    case RADIX_POW2: launch_col_rs<T, RADIX_POW2>(a, lds, nb, nt, s); break;
    case RADIX_WIDE: launch_col_rs<T, RADIX_WIDE>(a, lds, nb, nt, s); break;
    default: launch_col_rs<T, RADIX_ALL>(a, lds, nb, nt, s); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_update(const UpdArgs<T>& a, hipStream_t s) {
  const dim3 grid((unsigned)update_blocks(a.n), (unsigned)nprob_of(a.bt));
  if (a.eq && a.defer_x) return hipErrorInvalidValue;
  if (a.eq) hipLaunchKernelGGL((update_kernel<T, true, false>), grid, dim3(256), 0, s, a);
  else if (a.defer_x) hipLaunchKernelGGL((update_kernel<T, false, true>), grid, dim3(512), 0, s, a);
  else hipLaunchKernelGGL((update_kernel<T, false, false>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// The x step an update left pending, for problems that stopped before a
// direction step applied it.  x_pend is read here and cleared by the next
// kernel, so that no block reads a flag another block of its launch writes.
template <typename T>
__global__ __launch_bounds__(256) void flush_x_kernel(UpdArgs<T> a) {
  const int pb = batch_prob(a.bt);
  const DevState* st = a.st + pb;
  if (!st->x_pend) return;
  const long long vo = (long long)pb * a.bt.vstride;
  const T ta = (T)st->alpha_log;
  const long long stride = (long long)gridDim.x * 256;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < a.n; i += stride) {
    cx<T> x = a.x[vo + i];
    const cx<T> p = a.p[vo + i];
    x.re += ta * p.re;
    x.im += ta * p.im;
    a.x[vo + i] = x;
  }
}

__global__ void clear_xpend_kernel(DevState* st, Batch bt) {
  if (threadIdx.x == 0) st[batch_prob(bt)].x_pend = 0;
}

template <typename T>
hipError_t launch_flush_x(const UpdArgs<T>& a, hipStream_t s) {
  const unsigned np = (unsigned)nprob_of(a.bt);
  hipLaunchKernelGGL((flush_x_kernel<T>), dim3((unsigned)update_blocks(a.n), np), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(clear_xpend_kernel, dim3(1, np), dim3(64), 0, s, a.st, a.bt);
  return hipGetLastError();
}

// The partials of one producer folded into their first entry, the count set
// to one.  The consumers of these regions run in every block of a launch
// (the direction step, the CG update): without the fold each of their blocks
// would read all partials of a producer with many blocks.  One block of 1024
// threads sums them in a fixed order, so the value is deterministic; thread 0
// writes after the block barrier that ends every thread's reads.
__global__ __launch_bounds__(1024) void fold_partials_kernel(FoldArgs a) {
  constexpr int NT = 1024;
  const int pb = batch_prob(a.bt);
  DevState* st = a.st + pb;
  if (gated_out(st, a.gate)) return;
  Partials parts = a.parts;
  parts.base += (long long)pb * a.bt.pstride;
  int* count = a.region == PART_PQ ? &st->nparts_pq : &st->nparts[0];
  const int n = *count;
  const double s0 = block_sum_all<NT>(partial_share<NT>(parts.region(a.region), n));
  const double s1 = a.eq_region >= 0 ? block_sum_all<NT>(partial_share<NT>(parts.region(a.eq_region), n)) : 0.0;
  if (threadIdx.x == 0) {
    parts.region(a.region)[0] = s0;
    if (a.eq_region >= 0) parts.region(a.eq_region)[0] = s1;
    *count = 1;
  }
}

hipError_t launch_fold_partials(const FoldArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(fold_partials_kernel, dim3(1, (unsigned)nprob_of(a.bt)), dim3(1024), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finalize(const FinArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1, (unsigned)nprob_of(a.bt)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pipe_update(const PipeArgs<double>& a, hipStream_t s) {
  hipLaunchKernelGGL(pipe_update_kernel, dim3((unsigned)update_blocks(a.n), (unsigned)nprob_of(a.bt)), dim3(256), 0, s,
                     a);
  return hipGetLastError();
}

hipError_t launch_mix_accumulate(const MixArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(mix_accumulate_kernel, dim3((unsigned)update_blocks(a.n), (unsigned)nprob_of(a.bt)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mix_convert(const MixArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(mix_convert_kernel, dim3((unsigned)update_blocks(a.n), (unsigned)nprob_of(a.bt)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_state_init(DevState* st, const DevState& init, hipStream_t s) {
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(1), 0, s, st, init);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_zero(cx<T>* p, long long n, hipStream_t s) {
  hipLaunchKernelGGL(fill_zero_kernel<T>, dim3((unsigned)update_blocks(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

template hipError_t launch_row<double>(const RowArgs<double>&, hipStream_t);
template hipError_t launch_row<float>(const RowArgs<float>&, hipStream_t);
template hipError_t launch_col<double>(const ColArgs<double>&, hipStream_t);
template hipError_t launch_col<float>(const ColArgs<float>&, hipStream_t);
template hipError_t launch_update<double>(const UpdArgs<double>&, hipStream_t);
template hipError_t launch_update<float>(const UpdArgs<float>&, hipStream_t);
template hipError_t launch_flush_x<double>(const UpdArgs<double>&, hipStream_t);
template hipError_t launch_flush_x<float>(const UpdArgs<float>&, hipStream_t);
template hipError_t launch_fill_zero<double>(cx<double>*, long long, hipStream_t);
template hipError_t launch_fill_zero<float>(cx<float>*, long long, hipStream_t);
template long long row_blocks<double>(const RowArgs<double>&);
template long long row_blocks<float>(const RowArgs<float>&);
template long long col_blocks<double>(const ColArgs<double>&);
template long long col_blocks<float>(const ColArgs<float>&);

}  // namespace lshom
