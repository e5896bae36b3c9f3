// Internal interface between the host driver (lshom_api.cpp) and the HIP pass
// kernels.  Nothing here crosses the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_engine.hpp"

namespace lshom {

constexpr int kThreads = 256;   // every pass kernel runs 4 wave64s per block
constexpr int kMaxDim = 3;

// Device-resident CG scalars.  Written only by the last block of a reduction
// (fixed summation order), read by every kernel at entry.
struct DevState {
  double rr;            // (r, r) of the recursive residual
  double pq;            // (p, A p)
  double alpha, beta;
  double tol2b2;        // (tol * ||b||)^2
  double b2;            // ||b||^2 = |E|^2 |N|
  double rr0;           // (r0, r0)
  double rr_true;       // last FP64 true residual squared
  double leff[3];       // <lambda e>
  double dot_aux;       // scratch result of a plain reduction
  double rr_ref;        // mixed: (r, r) at the last refresh
  double drop2;         // mixed: refresh when rr < drop2 * rr_ref
  int iter;             // CG iterations done (operator applies in the loop)
  int max_iter;
  int done;             // nonzero: every iteration kernel returns at entry
  int status;           // 0 ok, -5 not converged, -6 breakdown
  int refresh;          // mixed: the refresh sequence runs when nonzero
  int since_refresh;
  int refresh_every;
  int n_refresh;
  int applies32, applies64;
  unsigned counter;     // arrival counter of the last-block reductions
  int pad[5];
};

// When a kernel returns at entry (it reads the device state first).
enum Gate : int {
  GATE_ALWAYS = 0,      // set-up and output kernels
  GATE_ACTIVE = 1,      // CG iteration kernels: skip once done
  GATE_REFRESH = 2,     // mixed refresh kernels: run only when a refresh is due
  GATE_NO_REFRESH = 3,  // skip when done or a refresh is due
};

// What the last block of a reducing kernel does with the grid-wide sum(s).
enum Finalize : int {
  FIN_NONE = 0,
  FIN_ALPHA = 1,      // pq -> alpha; breakdown if pq <= 0 or not finite
  FIN_RR_INIT = 2,    // rr0 = rr = sum; done if converged at the start
  FIN_UPDATE = 3,     // rr_new -> beta, iter++, convergence / iteration limit
  FIN_RR_TRUE = 4,    // rr_true = sum
  FIN_LEFF = 5,       // leff[0..d) = sums / |N|
  FIN_AUX = 6,        // dot_aux = sum
  FIN_REFRESH = 7,    // mixed: true residual of the refresh -> rr, rr_ref, done
  FIN_CLEAR_REFRESH = 8,  // mixed: the refresh sequence has finished
};

// ---------------------------------------------------------------------------
// Row pass: FFTs along the contiguous (last) axis, on rows of the half
// spectrum.  Pairs of real signals share one complex transform.
// ---------------------------------------------------------------------------
enum RowMode : int {
  ROW_FUSED = 0,   // spectrum A -> real u -> dL (E + u) -> spectrum T
  ROW_INV = 1,     // spectrum A -> real out = add + E + u (FP64); optional <lambda out>
  ROW_FWD = 2,     // real in (FP64, or constant E) -> [dL] in -> spectrum T
};
enum RowFlags : int {
  ROWF_DL = 1,        // ROW_FWD: multiply the input by dL = lambda - l0
  ROWF_CONST_E = 2,   // ROW_FWD: the input is the constant field E
  ROWF_ADD = 4,       // ROW_INV: add real_add to the output
  ROWF_LEFF = 8,      // ROW_INV: reduce <lambda out> into leff
};

template <typename T>
struct RowArgs {
  int n;                 // row length (last axis)
  int h;                 // n / 2 + 1
  long long nrows;       // product of the other axes
  int rows_per_block;
  int d;
  int mode, flags;
  int ss;                // LDS stride between sequences (odd, >= n)
  cx<T>* spec[kMaxDim];          // half-spectrum components [nrows][h]
  const double* real_in[kMaxDim];
  double* real_out[kMaxDim];
  const double* real_add[kMaxDim];
  const uint8_t* phase;          // [nrows][n]
  const T* cond;                 // conductivity per phase
  T l0;
  T E[kMaxDim];
  T inv_n;                       // 1 / |N|
  FftPlan plan;
  const cx<T>* tw;               // exp(-2 pi i m / n)
  DevState* st;
  double* partials;
  int fin;
  int gate;
};

// ---------------------------------------------------------------------------
// Strided-axis pass: FFTs along a non-contiguous axis of the half spectrum.
// The array is [outer][L][inner]; a block owns `tile` consecutive inner
// indices of one outer slice for all d components.
// ---------------------------------------------------------------------------
enum ColMode : int {
  COL_INV_C = 0,    // scalar c -> i khat_a c (a < d) -> inverse FFT -> comp[a]
  COL_PLAIN = 1,    // comp[a] -> FFT (direction dir) -> comp[a]
  COL_FWD_PROJ = 2, // comp[a] -> forward FFT -> s = -i khat . tau_hat -> out
};

template <typename T>
struct ColArgs {
  int L;                 // axis length
  long long inner;       // contiguous extent after the axis (in elements)
  long long outer;       // slices before the axis
  int tile;              // inner elements per block
  int tiles_per_outer;
  int d;
  int mode, dir;
  int ss;
  cx<T>* comp[kMaxDim];
  // spectral frequency data (axis-0 passes: L = N[0])
  int nd[kMaxDim];       // full grid sizes
  int dims;
  int h;                 // half length of the last axis
  // COL_INV_C
  const cx<T>* c_in;     // used when fuse_p == 0
  cx<T>* p_io;           // fuse_p: p = r + beta p (written back)
  const cx<T>* r_in;
  int fuse_p;
  // COL_FWD_PROJ: out = coef_base * base + coef_s * s
  cx<T>* out;
  const cx<T>* base;
  T coef_base, coef_s;
  int dot;               // 0 none, 1 (base, out), 2 (out, out)
  FftPlan plan;
  const cx<T>* tw;
  DevState* st;
  double* partials;
  int fin;
  int gate;
  double inv_n;          // scales the dot to real-space inner products
};

// ---------------------------------------------------------------------------
// Elementwise CG update on the half spectrum
// ---------------------------------------------------------------------------
template <typename T>
struct UpdArgs {
  long long n;           // elements
  int h;                 // half length of the last axis
  int n_last;            // full length of the last axis
  cx<T>* x;
  cx<T>* r;
  const cx<T>* p;
  const cx<T>* q;
  DevState* st;
  double* partials;
  double inv_n;
  int blocks;
  int gate;
};

// ---------------------------------------------------------------------------
// Mixed precision: fold the FP32 correction into the FP64 iterate and hand
// the FP64 true residual back to the FP32 recursion.
// ---------------------------------------------------------------------------
struct MixArgs {
  long long n;
  cx<double>* x64;
  cx<float>* x32;
  const cx<double>* r64;
  cx<float>* r32;
  DevState* st;
  double* partials;
  int gate;
  int clear_refresh;     // convert: the last block clears the refresh flag
  int blocks;
};

// Host launchers (defined in passes.hip).
template <typename T> hipError_t launch_row(const RowArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_col(const ColArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_update(const UpdArgs<T>& a, hipStream_t s);
hipError_t launch_state_init(DevState* st, const DevState& init, hipStream_t s);
hipError_t launch_mix_accumulate(const MixArgs& a, hipStream_t s);   // x64 += x32, x32 = 0
hipError_t launch_mix_convert(const MixArgs& a, hipStream_t s);      // r32 = r64
template <typename T> hipError_t launch_fill_zero(cx<T>* p, long long n, hipStream_t s);

// Number of blocks a launch uses (so the host can size partials).
template <typename T> long long row_blocks(const RowArgs<T>& a);
template <typename T> long long col_blocks(const ColArgs<T>& a);
long long update_blocks(long long n);

size_t row_lds_bytes(int n, int rows_per_block, int d, int elem_bytes, int* ss_out);
size_t col_lds_bytes(int L, int tile, int d, int elem_bytes, int* ss_out);

}  // namespace lshom
