// Wave passes of the operator apply on 3-D grids whose axes are 27, 81 or 243
// nodes long (the layouts V, Gl, Hl are described in kernels.hpp).
//
// Same algebra as the block passes of passes.hip: the CG vectors are the
// spectral coordinate c of the admissible fields, u_hat = i khat c, and one
// apply is
//   axis-0 inverse (W3_INV0): c -> F0^-1 [i xi_0 c / |xi|], F0^-1 [i c / |xi|]   V -> Gl
//                             (CG: also p = r + beta p and the x step the
//                             last update left to it)
//   axis-1 inverse (W3_COL1): F1^-1, u_1 also times xi_1                Gl -> Hl
//   row pass       (W3_ROW):  u_2 times xi_2, F2^-1, dL (E + u), F2,
//                             tau_2 times xi_2                          Hl -> Hl
//   axis-1 forward (W3_COL1): F1 tau_0, xi_1 F1 tau_1 + F1 (xi_2 tau_2)   Hl -> Hl
//   axis-0 forward (W3_FWD0): t = xi_0 F0 [..] + F0 [..] = xi . tau_hat,
//                             s = -i t / |xi|, out, dot                 Hl -> V
// (Sec. 2.2, Eqs. (15)-(17): the Green operator k (x) k / (l0 |k|^2) of
// Sec. 2.1, Eq. (7) becomes the projection on khat and 1 / l0.)  The wave
// vector components xi_1 and xi_2 are constant along axis 0, so the axis-0
// passes carry two fields instead of three: xi_1 is applied in the axis-1
// spectrum and xi_2 in the last-axis spectrum (by linearity of the other
// transforms), which saves two of the eighteen 1-D transforms of an apply
// and a sixth of its bytes.
//
// Every 1-D transform is a wave-level FFT (wave_fft.hpp): a block is a few
// independent waves, each owning whole sequences, with one block barrier
// once the twiddle table (and the tile) are in LDS; the loads of a block's
// data go out before its tables are stored, so their latencies overlap.  A
// block owns one tile (8 columns of one cg group, all points of the
// transformed axis) and writes it as one contiguous region of its output
// layout; reads are strided in 128-byte rows (column passes) or contiguous.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "reduce.hpp"
#include "wave_fft.hpp"

namespace lshom {

namespace {

// columns of a tile transformed by one wave (the tile is 8 columns wide)
template <int N>
__host__ __device__ constexpr int w3_cpw() {
  return N == 243 ? 2 : (N == 81 ? 4 : 8);
}
template <int N>
__host__ __device__ constexpr int w3_col_threads() {
  return 64 * (kW3Group / w3_cpw<N>());
}
// rows per row-pass block: four waves, two real rows per complex sequence
template <int N>
__host__ __device__ constexpr int w3_rows_per_block() {
  return 4 * 2 * WaveGeom<N>::SPW;
}

__device__ __forceinline__ int w3_freq(int m, int n) { return (m <= n / 2) ? m : m - n; }

// Wave-vector component xi = k / Y for integer frequency k, in the precision
// of the pass (FP32 passes form it in FP32).
template <typename T>
__device__ __forceinline__ T w3_xi(int k, double cinv) {
  if constexpr (sizeof(T) == 8) return (double)k * cinv;
  else return (float)k * (float)cinv;
}

// 1 / |xi| at a point of the half spectrum; 0 at xi = 0 and in the padding
// (ok false).  FP64 passes take the correctly rounded value; FP32 passes the
// hardware reciprocal square root in FP32 (about one FP32 ulp).  Both axis-0
// passes of one precision form it here, so the factor applied on the way in
// is the one applied on the way out and the operator stays symmetric.
template <typename T>
__device__ __forceinline__ T w3_inv_norm(T x0, T x1, T x2, bool ok) {
  const T k2 = x0 * x0 + x1 * x1 + x2 * x2;
  if constexpr (sizeof(T) == 8) return (ok && k2 > 0.0) ? 1.0 / sqrt(k2) : 0.0;
  else return (ok && k2 > 0.0f) ? __builtin_amdgcn_rsqf(k2) : 0.0f;
}

// Streaming access for vectors that no later pass of the iteration reads
// again soon (x, p around the axis-0 passes): the non-temporal hint keeps them
// from displacing the pass fields the next pass reads.
template <typename T>
__device__ __forceinline__ cx<T> ld_stream(const cx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return cx<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void st_stream(cx<T>* p, cx<T> c) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 v;
  v.x = c.re;
  v.y = c.im;
  __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
}

// Weight of half-spectrum column c in a full-spectrum sum (the last axis is
// odd here: column 0 stands for itself, the others for two; padding: 0).
__device__ __forceinline__ double w3_weight(int c, int h) { return c == 0 ? 1.0 : (c < h ? 2.0 : 0.0); }

// The dispatcher deals the blocks of a launch to the 8 XCDs in turn; the
// blocks of one tile's three components (consecutive linear ids) should share
// an XCD (and its L2), so each XCD is given one contiguous run of ids.
__device__ __forceinline__ unsigned w3_xcd_block() {
  const unsigned total = gridDim.x, lin = blockIdx.x;
  const unsigned xcd = lin & 7u, slot = lin >> 3;
  const unsigned q = total >> 3, rem = total & 7u;
  return xcd * q + (xcd < rem ? xcd : rem) + slot;
}

// arr[c] for a runtime c without a dynamically indexed register array
template <typename V>
__device__ __forceinline__ V w3_pick(const V (&arr)[kMaxDim], int c) {
  return c == 0 ? arr[0] : (c == 1 ? arr[1] : arr[2]);
}

// A tile of 8 columns x L points of one field moves between global memory
// (entry (p, cc) at g + p * pstride + cc) and the block's LDS sequences
// (column cc at seq + cc * L, points in natural order) with eight
// consecutive threads on each 128-byte row.  tile_load multiplies point p by
// xi = freq(p) * ks when ks != 0.
template <typename T, int L, int NT>
struct TileRegs {
  static constexpr int TOT = kW3Group * L, PER = (TOT + NT - 1) / NT;
  cx<T> v[PER];
};

// tile_load in two halves: the global loads into registers, then the LDS
// stores (so that other loads, such as the twiddle table's, can go out
// between them)
template <typename T, int L, int NT>
__device__ __forceinline__ void tile_fetch(TileRegs<T, L, NT>& t, const cx<T>* __restrict__ g, long long pstride) {
  constexpr int TOT = TileRegs<T, L, NT>::TOT, PER = TileRegs<T, L, NT>::PER;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = (int)threadIdx.x + u * NT;
    t.v[u] = (TOT % NT == 0 || e < TOT) ? g[(long long)(e >> 3) * pstride + (e & 7)] : cx<T>{T(0), T(0)};
  }
}

template <typename T, int L, int NT>
__device__ __forceinline__ void tile_put(cx<T>* seq, const TileRegs<T, L, NT>& t, double ks) {
  constexpr int TOT = TileRegs<T, L, NT>::TOT, PER = TileRegs<T, L, NT>::PER;
  const cx<T>* v = t.v;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = (int)threadIdx.x + u * NT;
    if (TOT % NT == 0 || e < TOT) {
      const int pt = e >> 3, cc = e & 7;
      cx<T> x = v[u];
      if (ks != 0.0) {
        const T k = w3_xi<T>(w3_freq(pt, L), ks);
        x = cx<T>{k * x.re, k * x.im};
      }
      seq[cc * L + pt] = x;
    }
  }
}

template <typename T, int L, int NT>
__device__ __forceinline__ void tile_load(cx<T>* seq, const cx<T>* __restrict__ g, long long pstride, double ks) {
  TileRegs<T, L, NT> t;
  tile_fetch<T, L, NT>(t, g, pstride);
  tile_put<T, L, NT>(seq, t, ks);
}

template <typename T, int L, int NT>
__device__ __forceinline__ void tile_store(cx<T>* __restrict__ g, long long pstride, const cx<T>* seq) {
  constexpr int TOT = kW3Group * L, PER = (TOT + NT - 1) / NT;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = (int)threadIdx.x + u * NT;
    if (TOT % NT == 0 || e < TOT) g[(long long)(e >> 3) * pstride + (e & 7)] = seq[(e & 7) * L + (e >> 3)];
  }
}

// The twiddle table in two halves, one entry per thread (N <= NT): the load
// goes out with the block's other loads, the LDS store comes after them.
template <typename T, int N, int NT>
__device__ __forceinline__ cx<T> tw_fetch(const cx<T>* __restrict__ src) {
  static_assert(N <= NT, "one twiddle entry per thread");
  return (int)threadIdx.x < N ? src[threadIdx.x] : cx<T>{T(0), T(0)};
}
template <typename T, int N>
__device__ __forceinline__ void tw_put(cx<T>* tw, cx<T> v) {
  if ((int)threadIdx.x < N) tw[threadIdx.x] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// Axis-0 inverse: V -> Gl
// ---------------------------------------------------------------------------
template <typename T, int N0>
__global__ __launch_bounds__(w3_col_threads<N0>()) void w3_inv0_kernel(W3Args<T> a) {
  constexpr int NT = w3_col_threads<N0>();
  constexpr int LPS = WaveGeom<N0>::LPS, CPW = w3_cpw<N0>();
  const int pb = a.bt.live ? a.bt.live[blockIdx.y] : (int)blockIdx.y;
  DevState* st = a.st + pb;
  Partials parts = a.parts;
  parts.base += (long long)pb * a.bt.pstride;
  const unsigned bx = blockIdx.x;
  // x += alpha p owed by the last CG update (stable during this launch: set
  // by the update, cleared by the pass after this one)
  const int xp = (a.cg_step && a.x_io) ? st->x_pend : 0;
  double beta = 0.0;
  // the direction step decides beta (and the stop) from the (r, r) sums; all
  // threads take part in the block reduction before anything else
  bool go = true;
  if (a.cg_step) {
    go = cg_direction<NT>(st, parts, a.inv_nd, &beta, a.gate, 0, bx == 0);
  } else if (gated_out_stable(st, a.gate)) {
    return;
  }
  if (!go && !xp) return;
  const int G = a.G, N1 = a.N1;
  const int b = (int)(bx / (unsigned)G), cg = (int)(bx - (unsigned)b * G);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int s = lane / LPS, j = lane - s * LPS;
  const bool act = s < CPW;
  const int cc = w * CPW + (act ? s : 0);
  const int c = cg * kW3Group + cc;
  const long long vo = (long long)pb * a.bt.vstride;
  // V: ((b G + cg) 8 + cc) N0 + a;  Gl: ((b G + cg) N0 + a) 8 + cc
  const long long vcol = vo + ((long long)(b * G + cg) * kW3Group + cc) * N0;
  const T ta = xp ? (T)st->alpha_log : T(0);
  if (!go) {
    // the solve stops here: only the owed step of x
    if (act) {
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        cx<T> xv = ld_stream(a.x_io + vcol + j + LPS * r);
        const cx<T> pv = a.p_io[vcol + j + LPS * r];
        xv.re += ta * pv.re;
        xv.im += ta * pv.im;
        st_stream(a.x_io + vcol + j + LPS * r, xv);
      }
    }
    return;
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  // the table is staged first: the block barrier then comes before the
  // column's loads, and each wave runs on to its transforms on its own
  tw_put<T, N0>(tw, tw_fetch<T, N0, NT>(a.tw[0]));
  __syncthreads();
  cx<T>* buf = tw + N0 + (w * CPW + (act ? s : 0)) * N0;
  const long long gtile = vo + (long long)(b * G + cg) * N0 * kW3Group;
  cx<T> cv[9];
  const T tb = (T)beta;
  if (act) {
    if (a.cg_step) {
      cx<T> rv[9], pv[9];
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        rv[r] = a.r_in[vcol + j + LPS * r];
        pv[r] = a.p_io[vcol + j + LPS * r];
      }
      if (xp) {
#pragma unroll
        for (int r = 0; r < 9; ++r) {
          cx<T> xv = ld_stream(a.x_io + vcol + j + LPS * r);
          xv.re += ta * pv[r].re;
          xv.im += ta * pv[r].im;
          st_stream(a.x_io + vcol + j + LPS * r, xv);
        }
      }
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        cv[r] = cx<T>{rv[r].re + tb * pv[r].re, rv[r].im + tb * pv[r].im};
        st_stream(a.p_io + vcol + j + LPS * r, cv[r]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < 9; ++r) cv[r] = a.c_in[vcol + j + LPS * r];
    }
  }
  // khat at each point: xi_0 depends on a, xi_1 and xi_2 on the column
  const T x1 = w3_xi<T>(w3_freq(b, N1), a.cinv[1]);
  const T x2 = w3_xi<T>(c, a.cinv[2]);
  const bool col_ok = c < a.h;
  // c / |xi| in place: only it stays live across the two transforms (the
  // kernel then holds three waves per SIMD instead of two)
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const T inv = w3_inv_norm<T>(w3_xi<T>(w3_freq(j + LPS * r, N0), a.cinv[0]), x1, x2, col_ok);
    cv[r] = cx<T>{inv * cv[r].re, inv * cv[r].im};
  }
  // field 0: i xi_0 c / |xi|; field 1: i c / |xi| (xi_1, xi_2 come later)
#pragma unroll 1
  for (int al = 0; al < 2; ++al) {
    cx<T> v[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const T k = al == 0 ? w3_xi<T>(w3_freq(j + LPS * r, N0), a.cinv[0]) : T(1);
      v[r] = cx<T>{-k * cv[r].im, k * cv[r].re};
    }
    wave_fft<T, N0, +1>(v, buf, tw, j, act);
    __syncthreads();
    tile_store<T, N0, NT>((al == 0 ? a.gl[0] : a.gl[1]) + gtile, kW3Group, tw + N0);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Axis-1 transform: Gl -> Hl (inverse, dir > 0) or Hl -> Hl (forward)
// ---------------------------------------------------------------------------
template <typename T, int N1, int DIR>
__global__ __launch_bounds__(w3_col_threads<N1>()) void w3_col1_kernel(W3Args<T> a) {
  constexpr int NT = w3_col_threads<N1>();
  constexpr int LPS = WaveGeom<N1>::LPS, CPW = w3_cpw<N1>();
  const int pb = a.bt.live ? a.bt.live[blockIdx.y] : (int)blockIdx.y;
  DevState* st = a.st + pb;
  // after a direction step: the x step it owed has been applied (also when
  // this launch is gated out)
  if (DIR > 0 && a.clear_xpend && blockIdx.x == 0 && threadIdx.x == 0) st->x_pend = 0;
  if (gated_out_stable(st, a.gate)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* seq = tw + N1;
  const int G = a.G, N0 = a.N0;
  // block = (tile, output), the output fastest.  Forward: the two fields the
  // axis-0 pass takes.  Inverse FP64: u_0, u_1, u_2, one transform per block;
  // inverse FP32: u_0, and u_1 with u_2 from one fetch of field 1 (the FP32
  // passes are bound by instruction issue, the FP64 ones by memory: measured
  // at 243^3, FP32 70 -> 66 us, FP64 133 -> 139 us)
  constexpr bool kU12 = DIR > 0 && sizeof(T) == 4;
  constexpr unsigned NF = (DIR > 0 && !kU12) ? 3u : 2u;
  const unsigned lin = w3_xcd_block();
  const int al = (int)(lin % NF);
  const unsigned bx = lin / NF;
  const int ai = (int)(bx / (unsigned)G), cg = (int)(bx - (unsigned)ai * G);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int s = lane / LPS, j = lane - s * LPS;
  const bool act = s < CPW;
  cx<T>* buf = seq + (w * CPW + (act ? s : 0)) * N1;
  const long long vo = (long long)pb * a.bt.vstride;
  // Gl: ((b G + cg) N0 + a) 8 + cc (stride in b: G N0 8);  Hl: ((a G + cg) N1 + b) 8 + cc
  const long long htile = vo + (long long)(ai * G + cg) * N1 * kW3Group;
  const long long gtile = vo + ((long long)cg * N0 + ai) * kW3Group;
  const long long gstep = (long long)G * N0 * kW3Group;
  if constexpr (DIR > 0) {
    // u_0 from field 0; u_1 (times xi_1 of the input index) and u_2 from field
    // 1 (FP32: fetched once, transformed twice); the tile's loads go out
    // before the twiddle table is staged
    TileRegs<T, N1, NT> t;
    tile_fetch<T, N1, NT>(t, (al == 0 ? a.gl[0] : a.gl[1]) + gtile, gstep);
    tw_put<T, N1>(tw, tw_fetch<T, N1, NT>(a.tw[1]));
    tile_put<T, N1, NT>(seq, t, al == 1 ? a.cinv[1] : 0.0);
    __syncthreads();
    wave_fft_lds<T, N1, DIR>(buf, tw, j, act);
    __syncthreads();
    tile_store<T, N1, NT>(w3_pick(a.hl, al) + htile, kW3Group, seq);
    if (kU12 && al == 1) {
      __syncthreads();
      tile_put<T, N1, NT>(seq, t, 0.0);
      __syncthreads();
      wave_fft_lds<T, N1, DIR>(buf, tw, j, act);
      __syncthreads();
      tile_store<T, N1, NT>(a.hl[2] + htile, kW3Group, seq);
    }
  } else {
    // field 0: F1 tau_0; field 1: xi_1 F1 tau_1 + F1 (xi_2 tau_2), written over tau_1
    TileRegs<T, N1, NT> t;
    tile_fetch<T, N1, NT>(t, (al == 0 ? a.hl[0] : a.hl[1]) + htile, kW3Group);
    tw_put<T, N1>(tw, tw_fetch<T, N1, NT>(a.tw[1]));
    tile_put<T, N1, NT>(seq, t, 0.0);
    __syncthreads();
    wave_fft_lds<T, N1, DIR>(buf, tw, j, act);
    if (al == 1) {
      cx<T> acc[9];
      if (act) {
#pragma unroll
        for (int r = 0; r < 9; ++r) {
          const T k1 = w3_xi<T>(w3_freq(j + LPS * r, N1), a.cinv[1]);
          const cx<T> z = buf[j + LPS * r];
          acc[r] = cx<T>{k1 * z.re, k1 * z.im};
        }
      }
      __syncthreads();
      tile_load<T, N1, NT>(seq, a.hl[2] + htile, kW3Group, 0.0);
      __syncthreads();
      wave_fft_lds<T, N1, DIR>(buf, tw, j, act);
      if (act) {
#pragma unroll
        for (int r = 0; r < 9; ++r) {
          const cx<T> z = buf[j + LPS * r];
          buf[j + LPS * r] = cx<T>{acc[r].re + z.re, acc[r].im + z.im};
        }
      }
    }
    __syncthreads();
    tile_store<T, N1, NT>((al == 0 ? a.hl[0] : a.hl[1]) + htile, kW3Group, seq);
  }
}

// ---------------------------------------------------------------------------
// Row pass (last axis), Hl in place: rows rho = a N1 + b, two real rows per
// complex sequence (rho even: first, rho + 1: second).
// ---------------------------------------------------------------------------
template <typename T, int N2, int MODE>
__global__ __launch_bounds__(256) void w3_row_kernel(W3Args<T> a) {
  constexpr int LPS = WaveGeom<N2>::LPS, SPW = WaveGeom<N2>::SPW;
  constexpr int RB = w3_rows_per_block<N2>();
  const int pb = a.bt.live ? a.bt.live[blockIdx.y] : (int)blockIdx.y;
  DevState* st = a.st + pb;
  if (gated_out_stable(st, a.gate)) return;
  const ProbEntry* pe = a.bt.tab ? a.bt.tab + pb : nullptr;
  Partials parts = a.parts;
  parts.base += (long long)pb * a.bt.pstride;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  T* cond = reinterpret_cast<T*>(tw + N2 + 4 * SPW * N2);
  // phase bytes of the block's rows, after the conductivity table (16-byte aligned)
  uint8_t* phs = reinterpret_cast<uint8_t*>(cond) + ((size_t)a.n_phases * sizeof(T) + 15) / 16 * 16;
  // block = (row block, component), the component fastest
  const unsigned lin = w3_xcd_block();
  const int al = (int)(lin % 3u);
  const unsigned rb = lin / 3u;
  const int G = a.G, N1 = a.N1, h = a.h;
  const long long nrows = (long long)a.N0 * N1;
  const long long nvox = nrows * N2;
  const uint8_t* phase = pe ? pe->phase : a.phase;
  const long long row0 = (long long)rb * RB;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int s = lane / LPS, j = lane - s * LPS;
  const bool lane_ok = s < SPW;
  const long long rhoA = (long long)rb * RB + (long long)(w * SPW + (lane_ok ? s : 0)) * 2;
  const bool hasA = lane_ok && rhoA < nrows;
  const bool hasB = lane_ok && rhoA + 1 < nrows;
  cx<T>* buf = tw + N2 + (w * SPW + (lane_ok ? s : 0)) * N2;
  const long long vo = (long long)pb * a.bt.vstride;
  // Hl entry (rho, c): a = rho / N1, b = rho % N1 -> ((a G + cg) N1 + b) 8 + cc
  // Hl entry 0 of the wave's row wrow + t (t < 2 SPW), without a division per
  // row: b wraps at most once when 2 SPW <= 27 <= N1, else at most twice
  const int wrow32 = (int)rb * RB + w * SPW * 2;
  const int wa0 = wrow32 / N1, wb0 = wrow32 - wa0 * N1;
  auto wbase = [&](int t) -> long long {
    int ai = wa0, bi = wb0 + t;
    const bool w1 = bi >= N1;
    bi = w1 ? bi - N1 : bi;
    ai += w1 ? 1 : 0;
    if constexpr (2 * SPW > 27) {
      const bool w2 = bi >= N1;
      bi = w2 ? bi - N1 : bi;
      ai += w2 ? 1 : 0;
    }
    return vo + ((long long)ai * G * N1 + bi) * kW3Group;
  };
  // The wave's half-spectrum entries e = lane + 64 it, in groups of eight
  // (one 128-byte group of a row each): group g = e / 8 is entry group
  // mg = g / SPW of the wave's row pair qq = g % SPW.  When SPW divides 8 the
  // pair does not depend on it and mg grows by 8 / SPW per it: the row bases
  // and the entry offset are formed once.
  constexpr bool kPairFixed = 8 % SPW == 0;
  auto pair_of = [&](int e) -> int { return kPairFixed ? (lane >> 3) % SPW : (e >> 3) % SPW; };
  auto group_of = [&](int e, int it) -> int {
    return kPairFixed ? (lane >> 3) / SPW + (8 / SPW) * it : (e >> 3) / SPW;
  };
  // entry offset of half index mg 8 + (e & 7) within its row
  auto hoff_g = [&](int mg, int e) -> long long { return (long long)mg * N1 * kW3Group + (e & 7); };
  // the wave's half-spectrum entries (not in the forward-from-real mode) are
  // requested before the block stages its tables, so both latencies overlap
  constexpr int HP = w3_groups(N2 / 2 + 1) * kW3Group;  // padded half length
  constexpr int TOT = SPW * HP;                          // entries of the wave's rows
  constexpr int IT = (TOT + 63) / 64;
  const long long wrow = (long long)rb * RB + (long long)w * SPW * 2;  // the wave's first row
  cx<T> A[IT], B[IT];
  if constexpr (MODE != ROW_FWD) {
    const cx<T>* src = w3_pick(a.hl, al);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = lane + 64 * it;
      const int qq = pair_of(e), mg = group_of(e, it), m = mg * kW3Group + (e & 7);
      const long long ra = wrow + 2 * qq;
      const bool ok = e < TOT && m < h;
      const long long ho = hoff_g(mg, e);
      A[it] = (ok && ra < nrows) ? src[wbase(2 * qq) + ho] : cx<T>{T(0), T(0)};
      B[it] = (ok && ra + 1 < nrows) ? src[wbase(2 * qq + 1) + ho] : cx<T>{T(0), T(0)};
    }
  }
  // the block's tables: twiddles, conductivities, the phase bytes of its rows
  // (as words when aligned); every load is issued before the LDS stores
  const cx<T> twv = tw_fetch<T, N2, 256>(a.tw[2]);
  const T* csrc = a.cond + (long long)pb * kCondStride;
  {
    const long long rows_here = nrows - row0 < RB ? nrows - row0 : RB;
    const int nb = (int)(rows_here * N2);
    const uint8_t* src = phase + row0 * N2;
    if ((reinterpret_cast<uintptr_t>(src) & 3u) == 0) {
      constexpr int PW = (RB * N2 / 4 + 255) / 256;  // phase words per thread
      const uint32_t* s4 = reinterpret_cast<const uint32_t*>(src);
      uint32_t* d4 = reinterpret_cast<uint32_t*>(phs);
      uint32_t pw[PW];
#pragma unroll
      for (int u = 0; u < PW; ++u) {
        const int i = (int)threadIdx.x + 256 * u;
        pw[u] = i < nb / 4 ? s4[i] : 0u;
      }
#pragma unroll
      for (int u = 0; u < PW; ++u) {
        const int i = (int)threadIdx.x + 256 * u;
        if (i < nb / 4) d4[i] = pw[u];
      }
      for (int i = (nb / 4) * 4 + threadIdx.x; i < nb; i += 256) phs[i] = src[i];
    } else {
      for (int i = threadIdx.x; i < nb; i += 256) phs[i] = src[i];
    }
  }
  for (int i = threadIdx.x; i < a.n_phases; i += 256) cond[i] = csrc[i];
  tw_put<T, N2>(tw, twv);
  __syncthreads();
  const T l0 = pe ? (T)pe->l0 : a.l0;
  const T Ea = (a.flags & ROWF_STATE_E) ? (T)st->E[al] : w3_pick(a.E, al);
  cx<T> v[9];
  if constexpr (MODE == ROW_FWD) {
    // real rows in (or the constant E), times dL when asked
    const double* rin = pe ? (pe->x0 ? pe->x0 + al * nvox : nullptr) : w3_pick(a.real_in, al);
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const int x = j + LPS * r;
      T t[2] = {T(0), T(0)};
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const bool has = u == 0 ? hasA : hasB;
        if (!has) continue;
        const long long g = (rhoA + u) * N2 + x;
        T val = (a.flags & ROWF_CONST_E) ? Ea : (rin ? (T)rin[g] : T(0));
        if (a.flags & ROWF_DL) val *= cond[phs[(int)(g - row0 * N2)]] - l0;
        t[u] = val;
      }
      v[r] = cx<T>{t[0], t[1]};
    }
  } else {
    // two Hermitian half rows -> one full complex row, inverse transform
    // each stored half-spectrum entry m < h of the wave's rows is read once
    // (eight consecutive lanes on one 128-byte group of a row) and placed at
    // m and (its Hermitian image) N2 - m of the packed sequence
    cx<T>* wseq = tw + N2 + w * SPW * N2;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = lane + 64 * it;
      const int qq = pair_of(e), m = group_of(e, it) * kW3Group + (e & 7);
      if (e >= TOT || m >= h) continue;
      cx<T> Am = A[it], Bm = B[it];
      if (al == 2) {
        // u_2: the field carries i c / |xi| here; xi_2 of the stored half index
        const T k2 = w3_xi<T>(m, a.cinv[2]);
        Am = cx<T>{k2 * Am.re, k2 * Am.im};
        Bm = cx<T>{k2 * Bm.re, k2 * Bm.im};
      }
      cx<T>* sq = wseq + qq * N2;
      sq[m] = cx<T>{Am.re - Bm.im, Am.im + Bm.re};
      if (m > 0) sq[N2 - m] = cx<T>{Am.re + Bm.im, Bm.re - Am.im};
    }
    // the inverse transform stays in registers: z[r] = node j + LPS r
    cx<T> z[9];
    wave_fft_lds_regs<T, N2, +1>(buf, tw, j, lane_ok, z);
    if constexpr (MODE == ROW_INV) {
      double* out = pe ? (pe->e_out ? pe->e_out + al * nvox : nullptr) : w3_pick(a.real_out, al);
      const double* add = w3_pick(a.real_add, al);
      double acc = 0.0;
      if (lane_ok) {
#pragma unroll
        for (int r = 0; r < 9; ++r) {
          const int x = j + LPS * r;
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const bool has = u == 0 ? hasA : hasB;
            if (!has) continue;
            const long long g = (rhoA + u) * N2 + x;
            const int q = phs[(int)(g - row0 * N2)];
            double val = (double)Ea + (double)((u == 0 ? z[r].re : z[r].im) * a.inv_n);
            if (a.flags & ROWF_DL_OUT) val *= (double)cond[q] - (double)l0;
            if (a.flags & ROWF_ADD) val += add[g];
            if (out) out[g] = val;
            if (a.flags & ROWF_LEFF) acc += (double)cond[q] * val;
          }
        }
      }
      if (a.flags & ROWF_LEFF) store_partial<256>(acc, parts.region(PART_AUX) + (long long)rb * 3 + al);
      return;
    } else {
      // polarisation dL (E + u) at the nodes (Sec. 2.2, Eq. (17))
      if (lane_ok) {
#pragma unroll
        for (int r = 0; r < 9; ++r) {
          const int x = j + LPS * r;
          T t0 = T(0), t1 = T(0);
          const int pa = (int)(rhoA - row0) * N2 + x;
          if (hasA) t0 = (cond[phs[pa]] - l0) * (Ea + z[r].re * a.inv_n);
          if (hasB) t1 = (cond[phs[pa + N2]] - l0) * (Ea + z[r].im * a.inv_n);
          v[r] = cx<T>{t0, t1};
        }
      }
    }
  }
  if constexpr (MODE != ROW_INV) {
    wave_fft<T, N2, -1>(v, buf, tw, j, lane_ok);
    __builtin_amdgcn_wave_barrier();
    // split the two rows' spectra (tau_2 times xi_2: the axis-1 pass adds it
    // to xi_1 tau_1); eight consecutive lanes write one 128-byte group of a
    // row; the padding of the half rows gets zeros
    cx<T>* dst = w3_pick(a.hl, al);
    constexpr int HP = w3_groups(N2 / 2 + 1) * kW3Group;
    constexpr int TOT = SPW * HP;
    const long long wrow = (long long)rb * RB + (long long)w * SPW * 2;
    const cx<T>* wseq = tw + N2 + w * SPW * N2;
#pragma unroll
    for (int e0 = 0; e0 < TOT; e0 += 64) {
      const int e = e0 + lane;
      if (TOT % 64 != 0 && e >= TOT) break;
      const int qq = pair_of(e), mg = group_of(e, e0 / 64), k = mg * kW3Group + (e & 7);
      const long long ra = wrow + 2 * qq;
      const long long ho = hoff_g(mg, e);
      cx<T> oa = {T(0), T(0)}, ob = {T(0), T(0)};
      if (k < h) {
        const cx<T>* sq = wseq + qq * N2;
        const cx<T> Y = sq[k];
        const cx<T> Ym = sq[k == 0 ? 0 : N2 - k];
        const T half = al == 2 ? T(0.5) * w3_xi<T>(k, a.cinv[2]) : T(0.5);
        oa = cx<T>{(Y.re + Ym.re) * half, (Y.im - Ym.im) * half};
        ob = cx<T>{(Y.im + Ym.im) * half, (Ym.re - Y.re) * half};
      }
      if (ra < nrows) dst[wbase(2 * qq) + ho] = oa;
      if (ra + 1 < nrows) dst[wbase(2 * qq + 1) + ho] = ob;
    }
  }
}

// ---------------------------------------------------------------------------
// Axis-0 forward + projection: Hl -> V
// ---------------------------------------------------------------------------
template <typename T, int N0>
__global__ __launch_bounds__(w3_col_threads<N0>()) void w3_fwd0_kernel(W3Args<T> a) {
  constexpr int NT = w3_col_threads<N0>();
  constexpr int LPS = WaveGeom<N0>::LPS, CPW = w3_cpw<N0>();
  const int pb = a.bt.live ? a.bt.live[blockIdx.y] : (int)blockIdx.y;
  DevState* st = a.st + pb;
  if (gated_out_stable(st, a.gate)) return;
  const ProbEntry* pe = a.bt.tab ? a.bt.tab + pb : nullptr;
  Partials parts = a.parts;
  parts.base += (long long)pb * a.bt.pstride;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  const cx<T> twv = tw_fetch<T, N0, NT>(a.tw[0]);
  __syncthreads();
  const int G = a.G, N1 = a.N1;
  const unsigned bx = blockIdx.x;
  const int b = (int)(bx / (unsigned)G), cg = (int)(bx - (unsigned)b * G);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int s = lane / LPS, j = lane - s * LPS;
  const bool act = s < CPW;
  const int cc = w * CPW + (act ? s : 0);
  const int c = cg * kW3Group + cc;
  cx<T>* buf = tw + N0 + (w * CPW + (act ? s : 0)) * N0;
  const long long vo = (long long)pb * a.bt.vstride;
  // Hl: ((a G + cg) N1 + b) 8 + cc (stride in a: G N1 8);  V: ((b G + cg) 8 + cc) N0 + a
  const long long htile = vo + ((long long)cg * N1 + b) * kW3Group;
  const long long hstep = (long long)G * N1 * kW3Group;
  const long long vcol = vo + ((long long)(b * G + cg) * kW3Group + cc) * N0;
  const T x1 = w3_xi<T>(w3_freq(b, N1), a.cinv[1]);
  const T x2 = w3_xi<T>(c, a.cinv[2]);
  const bool col_ok = c < a.h;
  // t = xi . tau_hat over the components; the factor 1 / |xi| of khat is
  // applied once at the end (fewer registers live across the transforms)
  cx<T> t[9];
#pragma unroll
  for (int r = 0; r < 9; ++r) t[r] = cx<T>{T(0), T(0)};
#pragma unroll 1
  for (int al = 0; al < 2; ++al) {
    __syncthreads();
    TileRegs<T, N0, NT> tr;
    tile_fetch<T, N0, NT>(tr, (al == 0 ? a.hl[0] : a.hl[1]) + htile, hstep);
    if (al == 0) tw_put<T, N0>(tw, twv);
    tile_put<T, N0, NT>(tw + N0, tr, 0.0);
    __syncthreads();
    cx<T> z[9];
    wave_fft_lds_regs<T, N0, -1>(buf, tw, j, act, z);
    if (act) {
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        // field 0 carries tau_0 (times xi_0 here), field 1 xi_1 tau_1 + xi_2 tau_2
        const T k = al == 0 ? w3_xi<T>(w3_freq(j + LPS * r, N0), a.cinv[0]) : T(1);
        t[r].re += k * z[r].re;
        t[r].im += k * z[r].im;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  const T cs = a.coef_s * (a.s_inv_l0 ? (T)(1.0 / (pe ? pe->l0 : a.l0d)) : T(1));
  const double wgt = w3_weight(c, a.h);
  double acc = 0.0;
  if (act) {
    cx<T> bv[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) bv[r] = a.base ? ld_stream(a.base + vcol + j + LPS * r) : cx<T>{T(0), T(0)};
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const T csk = cs * w3_inv_norm<T>(w3_xi<T>(w3_freq(j + LPS * r, N0), a.cinv[0]), x1, x2, col_ok);
      // s = -i khat . tau_hat
      cx<T> val = {csk * t[r].im, -csk * t[r].re};
      val.re += a.coef_base * bv[r].re;
      val.im += a.coef_base * bv[r].im;
      a.out[vcol + j + LPS * r] = val;
      if (a.dot == 1) {
        acc += wgt * ((double)bv[r].re * (double)val.re + (double)bv[r].im * (double)val.im);
      } else if (a.dot == 2) {
        acc += wgt * ((double)val.re * (double)val.re + (double)val.im * (double)val.im);
      } else if (a.dot == 3) {
        // the step |out - base|^2 of the basic scheme
        const double dr = (double)val.re - (double)bv[r].re, di = (double)val.im - (double)bv[r].im;
        acc += wgt * (dr * dr + di * di);
      }
    }
  }
  if (a.dot) {
    store_partial<NT>(acc, parts.region(a.dot_region) + bx);
    if (a.dot_region == PART_RR0 && bx == 0 && threadIdx.x == 0) st->nparts[0] = (int)gridDim.x;
    if (a.dot_region == PART_PQ && bx == 0 && threadIdx.x == 0) st->nparts_pq = (int)gridDim.x;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

namespace {

template <int N>
size_t w3_col_lds(int elem) {
  return (size_t)(N + kW3Group * N) * elem;
}

template <int N>
size_t w3_row_lds(int elem, int n_phases) {
  return (size_t)(N + 4 * WaveGeom<N>::SPW * N) * elem + ((size_t)n_phases * (elem / 2) + 15) / 16 * 16 +
         (size_t)w3_rows_per_block<N>() * N;
}

template <typename T, int N>
hipError_t launch_w3_n(int pass, const W3Args<T>& a, hipStream_t s) {
  const unsigned rows = (unsigned)(a.bt.nprob > 0 ? a.bt.nprob : 1);
  const int elem = (int)sizeof(cx<T>);
  switch (pass) {
    case W3_INV0:
      hipLaunchKernelGGL((w3_inv0_kernel<T, N>), dim3((unsigned)(a.N1 * a.G), rows), dim3(w3_col_threads<N>()),
                         w3_col_lds<N>(elem), s, a);
      break;
    case W3_COL1:
      if (a.dir > 0)
        hipLaunchKernelGGL((w3_col1_kernel<T, N, +1>), dim3((unsigned)((sizeof(T) == 4 ? 2 : 3) * a.N0 * a.G), rows),
                           dim3(w3_col_threads<N>()), w3_col_lds<N>(elem), s, a);
      else
        hipLaunchKernelGGL((w3_col1_kernel<T, N, -1>), dim3((unsigned)(2 * a.N0 * a.G), rows),
                           dim3(w3_col_threads<N>()), w3_col_lds<N>(elem), s, a);
      break;
    case W3_ROW: {
      const long long nrows = (long long)a.N0 * a.N1;
      const unsigned nb = 3u * (unsigned)((nrows + w3_rows_per_block<N>() - 1) / w3_rows_per_block<N>());
      const size_t lds = w3_row_lds<N>(elem, a.n_phases);
      if (a.mode == ROW_FUSED) hipLaunchKernelGGL((w3_row_kernel<T, N, ROW_FUSED>), dim3(nb, rows), dim3(256), lds, s, a);
      else if (a.mode == ROW_INV) hipLaunchKernelGGL((w3_row_kernel<T, N, ROW_INV>), dim3(nb, rows), dim3(256), lds, s, a);
      else hipLaunchKernelGGL((w3_row_kernel<T, N, ROW_FWD>), dim3(nb, rows), dim3(256), lds, s, a);
      break;
    }
    default:
      hipLaunchKernelGGL((w3_fwd0_kernel<T, N>), dim3((unsigned)(a.N1 * a.G), rows), dim3(w3_col_threads<N>()),
                         w3_col_lds<N>(elem), s, a);
      break;
  }
  return hipGetLastError();
}

}  // namespace

long long w3_blocks(int pass, int N0, int N1, int N2) {
  const int G = w3_groups(N2 / 2 + 1);
  switch (pass) {
    case W3_INV0:
    case W3_FWD0:
      return (long long)N1 * G;
    case W3_COL1:
      return (long long)N0 * G;
    default: {
      const long long rb = N2 == 243 ? w3_rows_per_block<243>() : (N2 == 81 ? w3_rows_per_block<81>()
                                                                            : w3_rows_per_block<27>());
      return ((long long)N0 * N1 + rb - 1) / rb;
    }
  }
}

template <typename T>
hipError_t launch_w3(int pass, const W3Args<T>& a, hipStream_t s) {
  // the transformed axis decides the kernel
  const int n = pass == W3_COL1 ? a.N1 : (pass == W3_ROW ? a.N2 : a.N0);
  if (n == 243) return launch_w3_n<T, 243>(pass, a, s);
  if (n == 81) return launch_w3_n<T, 81>(pass, a, s);
  if (n == 27) return launch_w3_n<T, 27>(pass, a, s);
  return hipErrorInvalidValue;
}

template hipError_t launch_w3<double>(int, const W3Args<double>&, hipStream_t);
template hipError_t launch_w3<float>(int, const W3Args<float>&, hipStream_t);

}  // namespace lshom
