// Internal interface between the host driver (lshom_api.cpp) and the HIP pass
// kernels.  Nothing here crosses the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_engine.hpp"

namespace lshom {

constexpr int kMaxDim = 3;
constexpr int kUpdateBlocks = 512;   // grid of the elementwise kernels (one partial each)
constexpr int kCondStride = 256;     // conductivity-table entries per problem

// Device-resident CG scalars.
//
// Inner products are reduced without atomics or fences: every block of a
// producing kernel stores one partial sum, and the consuming kernel (which
// starts after the producer has finished) sums the partials in block order in
// each of its blocks, so all blocks obtain the same value.  Each field below
// is written by one thread of a launch (block 0's first thread, or for jx and
// taup the thread that holds the k = 0 mode) and read only by later launches
// or by that same thread, so blocks of one kernel do not race on it.
struct DevState {
  double tol2b2;        // (tol * ||b||)^2
  double b2;            // ||b||^2 = |E|^2 |N|
  double rr_log;        // (r_k, r_k) seen by the last direction kernel / check
  double pq_log;        // (p_k, A p_k)
  double alpha_log;
  double rr_true;       // FP64 true residual squared (refresh / final check)
  double dot_aux;       // a plain reduction result
  double rr_ref;        // mixed: (r, r) at the last refresh
  double drop2;         // mixed: refresh when rr < drop2 * rr_ref
  double leff[3];       // <lambda e>
  double E[3];          // macroscopic field of the solve (set with the initial state)
  double l0;            // reference conductivity (the norms of Sec. 3, Eqs. (21)-(22));
                        // tr(L0) / d for an anisotropic reference
  double l0E[3];        // L0 E: the current of the reference medium under E
  double nvox;          // |N|
  double tol2;          // tol^2 (equilibrium test)
  double jx[3];         // DFT at k = 0 of dL (E + u(x)) for the iterate being tested
  double taup[3];       // DFT at k = 0 of dL u(p) for the last CG direction
  double eta_e_log;     // eta_e of the last test (-1: not formed)
  double eta_e_true;    // eta_e of the final field (-1: not formed)
  double bicg_rho;      // BiCG: (r, r*) of the current iterate
  double bicg_alpha;    // BiCG: step of the current iteration
  double bicg_beta;     // BiCG: direction update of the current iteration
  double pipe_alpha[2]; // pipelined CG: step of iteration k at [k & 1]
  double pipe_beta[2];  // pipelined CG: direction update of iteration k at [k & 1]
  double* hist;         // (eta_r, eta_e) of iterate m at [2m], [2m + 1], m < hist_len (or null)
  int hist_len;
  int norm;             // 0: ||r|| <= tol ||b||; 1: eta_e <= tol
  int iter_a;           // iterations completed (written by the update kernel)
  int iter_u;           // iteration in progress (written by the direction kernel)
  int max_iter;
  int done;             // nonzero: iteration kernels return at entry
  int status;           // 0 ok, -5 not converged, -6 breakdown
  int refresh;          // mixed: the refresh sequence runs when nonzero
  int refresh_every;    // mixed: > 0 selects the mixed-precision decisions
  int k_ref;            // mixed: iteration count at the last refresh
  int n_refresh;
  int nparts[2];        // number of partials in the two (r, r) buffers
  int nparts_pq;        // number of partials in the PQ region (set by its producer)
  int x_pend;           // the update left x += alpha_log p to the next direction step
                        // (set by the update, cleared by the pass after that step)
  int pad;
};

// When a kernel returns at entry.
enum Gate : int {
  GATE_ALWAYS = 0,      // set-up and output kernels
  GATE_ACTIVE = 1,      // FP64 CG kernels: skip once done
  GATE_REFRESH = 2,     // mixed refresh kernels: run only when a refresh is due
  GATE_NO_REFRESH = 3,  // mixed FP32 kernels: skip when done or a refresh is due
};

// Regions of the partial-sum array (each `stride` doubles; AUX holds 3 per
// block).  EQ0 / EQ1 hold the |k|^2-weighted residual sums of the
// equilibrium norm beside RR0 / RR1 (same producer, same count).
enum PartRegion : int { PART_RR0 = 0, PART_RR1 = 1, PART_PQ = 2, PART_AUX = 3, PART_EQ0 = 4, PART_EQ1 = 5 };
constexpr int kPartRegions = 6;

struct Partials {
  double* base;
  long long stride;     // doubles per region
  __host__ __device__ double* region(int r) const { return base + (long long)r * stride; }
};

// Per-problem data of a batched launch (device memory).
struct ProbEntry {
  const uint8_t* phase;   // [nrows][n] phase image
  double* e_out;          // FP64 field output d x |N| (may be null)
  const double* x0;       // FP64 warm start d x |N| (may be null)
  double l0;
};

// Problem dimension of a launch: block row blockIdx.y is problem p; its
// vectors start p * vstride elements, its partial sums p * pstride doubles
// and its state p entries after the launch's base pointers.  tab == nullptr
// means a single problem whose data are the fields of the argument struct.
struct Batch {
  int nprob;              // grid rows of the launch
  long long vstride;
  long long pstride;
  const ProbEntry* tab;
  const int* live;        // grid row -> problem; null: row y is problem y
};

// Problem of this block (see Batch::live).
__device__ __forceinline__ int batch_prob(const Batch& b) {
  return b.live ? b.live[blockIdx.y] : (int)blockIdx.y;
}

// Scalar steps of the single-block finalize kernel.
enum FinMode : int {
  FZ_CHECK = 0,         // FP64: convergence / limit test on (r_m, r_m), m = iter_a
  FZ_AUX = 1,           // dot_aux = sum(AUX)
  FZ_RR_TRUE = 2,       // rr_true = sum(AUX)
  FZ_LEFF = 3,          // leff[c] = sum(AUX[3 b + c]) / |N|
  FZ_REFRESH = 4,       // mixed: rr_true = sum(AUX); new reference; done tests
  FZ_REFRESH_INIT = 5,  // mixed: as FZ_REFRESH without counting a refresh
  FZ_FFTH = 6,          // basic scheme: norms of the step sum(RR0), sum(EQ0); count; done tests
  FZ_BICG_START = 7,    // BiCG: rho = sum(AUX[3b]), (r, r) = sum(AUX[3b + 1]); done tests
  FZ_BICG_ALPHA = 8,    // BiCG: alpha = rho / sum(PQ) (breakdown when zero or not finite)
  FZ_BICG_STEP = 9,     // BiCG: rho' and (r, r) of the new iterate; beta; count; done tests
};

// ---------------------------------------------------------------------------
// Row pass: FFTs along the contiguous (last) real-space axis.  A block owns
// rows_per_block consecutive rows (an even number) of every component, or of
// one component (split: block b handles component b % d of row block b / d),
// and pairs row 2j with row 2j+1 of the same component into one complex
// transform.
// Spectral element (row, k) of a component lives at row * rs_row + k * rs_k:
// natural layout rs_row = h, rs_k = 1; transposed (2-D) rs_row = 1, rs_k = nrows.
// ---------------------------------------------------------------------------
enum RowMode : int {
  ROW_FUSED = 0,   // spectrum -> real u -> dL (E + u) -> spectrum
  ROW_INV = 1,     // spectrum -> real out = add + E + u (FP64); optional <lambda out>
  ROW_FWD = 2,     // real in (FP64, or constant E) -> [dL] in -> spectrum
};
enum RowFlags : int {
  ROWF_DL = 1,        // ROW_FWD: multiply the input by dL = lambda - l0
  ROWF_CONST_E = 2,   // ROW_FWD: the input is the constant field E
  ROWF_ADD = 4,       // ROW_INV: add real_add to the output
  ROWF_LEFF = 8,      // ROW_INV: partial sums of <lambda out> into AUX
  ROWF_STATE_E = 16,  // E of each problem from its device state (not the argument)
  ROWF_DL_OUT = 32,   // ROW_INV: multiply E + u by dL = L - L0 before adding real_add
};

template <typename T>
struct RowArgs {
  int n;                 // row length (last axis)
  int h;                 // n / 2 + 1
  long long nrows;       // product of the other axes
  int rows_per_block;    // even
  int d;
  int split;             // one component per block
  int nt;                // block size (0: chosen by the launcher)
  int mode, flags;
  int ss;                // LDS stride between sequences (odd, >= n)
  long long rs_row, rs_k;
  int row_fast;          // thread order for global spectral access: rows fastest
  cx<T>* spec[kMaxDim];
  const double* real_in[kMaxDim];
  double* real_out[kMaxDim];
  const double* real_add[kMaxDim];
  const uint8_t* phase;          // [nrows][n]
  const T* cond;                 // conductivity table (n_phases entries)
  int n_phases;                  // table entries (phases x entries per phase)
  int tensor;                    // symmetric tensor phases: d (d + 1) / 2 entries each (needs !split)
  int aniso;                     // anisotropic reference (needs tensor): dL = L - L0 with L0 below
  T L0u[6];                      // L0, upper triangle row by row (2-D: 00 01 11)
  T l0;
  T E[kMaxDim];
  T inv_n;                       // 1 / |N|
  FftPlan plan;
  const cx<T>* tw;               // exp(-2 pi i m / n)
  DevState* st;
  Partials parts;
  int gate;
  Batch bt;
  FastDiv fd_n, fd_np, fd_h, fd_half;  // n, pairs per block, h, rows_per_block / 2
};

// ---------------------------------------------------------------------------
// Strided-axis pass: FFTs along a non-contiguous axis of the half spectrum.
// Element (o, l, ii) lives at o * L * inner + l * sl + ii * sii (natural:
// sl = inner, sii = 1; transposed 2-D: sl = 1, sii = L).  A block owns `tile`
// consecutive ii of one outer slice for all d components.
// ---------------------------------------------------------------------------
enum ColMode : int {
  COL_INV_C = 0,    // scalar c -> i khat_a c (a < d) -> inverse FFT -> comp[a]
  COL_PLAIN = 1,    // comp[a] -> FFT (direction dir) -> comp[a]
  COL_FWD_PROJ = 2, // comp[a] -> forward FFT -> s = -i khat . tau_hat -> out
  COL_PLAIN_FWD = 3, // kernel specialisation of COL_PLAIN with dir < 0 (launcher-internal)
  // launcher-internal specialisations of COL_INV_C / COL_FWD_PROJ that carry
  // the anisotropic-reference scale and the pipelined-CG steps (the plain
  // ones stay free of that code)
  COL_INV_C_GEN = 4,
  COL_FWD_PROJ_GEN = 5,
};

template <typename T>
struct ColArgs {
  int L;
  long long inner;
  long long outer;
  long long sl, sii;
  int tile;
  int tiles_per_outer;
  int nt;                // block size (0: chosen by the launcher)
  int d;
  int mode, dir;
  int ss;
  cx<T>* comp[kMaxDim];
  int nd[kMaxDim];       // full grid sizes
  int dims;
  int h;                 // half length of the last axis
  double cinv[kMaxDim];  // 1 / cell side length per axis: wave vector xi = k / Y
  // anisotropic reference: upper triangle of L0 / (tr(L0) / d); the spectral
  // coordinate then carries the factor 1 / sqrt(khat . L0n . khat)
  int aniso;
  double L0n[6];
  // COL_INV_C
  const cx<T>* c_in;     // used when cg_step == 0
  cx<T>* p_io;           // cg_step: p = r + beta p (written back)
  const cx<T>* r_in;
  int cg_step;           // this launch is the CG direction step (decides beta, stop)
  int pipe;              // pipelined CG: COL_INV_C takes the scalar step (alpha, beta,
                         // stop) from (r, r), (w, r); COL_FWD_PROJ adds beta * out
  // COL_FWD_PROJ: out = coef_base * base + coef_s * [1 / l0 if s_inv_l0] * s
  // (+ beta out for pipelined CG: z = A w + beta z)
  cx<T>* out;
  const cx<T>* base;
  T coef_base, coef_s;
  int s_inv_l0;
  double l0;             // single problem (batched: the problem table)
  int dot;               // 0 none, 1 (base, out), 2 (out, out), 3 (out - base, out - base)
  int dot_region;        // partial region; PART_RR0 also sets nparts[0]
  // equilibrium norm: record the DFT at k = 0 of the transformed field (taup
  // for dot 1, jx otherwise); dots 2 and 3 also store the |k|^2-weighted sum
  // into eq_region.  COL_INV_C with cg_step: the direction step reads it.
  int eq;
  int eq_region;
  FftPlan plan;
  const cx<T>* tw;
  DevState* st;
  Partials parts;
  int gate;
  double inv_n;          // scales spectral sums to real-space inner products
  Batch bt;
  FastDiv fd_L, fd_C, fd_h;  // L, tile, h
};

// ---------------------------------------------------------------------------
// Elementwise CG update on the half spectrum: x += alpha p, r -= alpha q
// ---------------------------------------------------------------------------
template <typename T>
struct UpdArgs {
  long long n;
  int h, n_last;
  long long klast_div;   // k_last = (i / klast_div) % h
  cx<T>* x;
  cx<T>* r;
  const cx<T>* p;
  const cx<T>* q;
  DevState* st;
  Partials parts;
  double inv_n;
  int gate;
  Batch bt;
  FastDiv fd_kd, fd_h;   // klast_div, h (n < 2^31)
  // equilibrium norm: |k|^2-weighted (r, r) beside (r, r), jx += alpha taup
  int eq;
  int dims;
  int nd[kMaxDim];
  FastDiv fd_n1;         // nd[1] (3-D index split)
  double cinv[kMaxDim];  // 1 / cell side length per axis
  int aniso;             // equilibrium weight xi . L0n . xi in place of |xi|^2
  double L0n[6];
  int w3;                // vectors in the wave-pass layout V (k_last from (cg, cc))
  FastDiv fd_w3n0;       // N0
  int w3g;               // G
  // x is not touched: x += alpha p waits for the next direction step, which
  // reads p anyway (x_pend, alpha_log)
  int defer_x;
};

// Pipelined CG update (spectral coordinate): s = w + beta s, p = r + beta p,
// x += alpha p, r -= alpha s, w -= alpha z; partials of (r, r) and (w, r).
template <typename T>
struct PipeArgs {
  long long n;
  int h, n_last;
  long long klast_div;
  cx<T>* x;
  cx<T>* r;
  cx<T>* p;
  cx<T>* w;
  cx<T>* s;
  const cx<T>* z;
  DevState* st;
  Partials parts;
  int gate;
  Batch bt;
  FastDiv fd_kd, fd_h;
};

// BiCG on real d-component nodal fields ([d][n] FP64, components contiguous):
// the elementwise steps around the two operator applies of an iteration.
enum BicgMode : int {
  BV_FILL_E = 0,     // x = E
  BV_START = 1,      // r = E - ap, r* = p = p* = r; AUX: (r, r*), (r, r)
  BV_DOT_APP = 2,    // PQ: (A p, p*)
  BV_UPDATE = 3,     // x += alpha p, r -= alpha A p, r* -= alpha A^T p*; AUX: (r, r*), (r, r)
  BV_DIRECTION = 4,  // p = r + beta p, p* = r* + beta p*
  BV_LEFF = 5,       // AUX[3b + c]: sum of lambda x_c
  BV_RESID = 6,      // AUX[b]: sum of (E - ap)^2
};

struct BicgArgs {
  long long n;           // nodes per component
  int d;
  int mode;
  double* x;
  double* r;
  double* rs;
  double* p;
  double* ps;
  const double* ap;
  const double* atp;
  const uint8_t* phase;  // BV_LEFF
  const double* cond;
  int tensor;            // cond holds symmetric tensors (upper triangles)
  DevState* st;
  Partials parts;
  int gate;
  FastDiv fd_n;
};

// Mixed precision: x64 += x32, x32 = 0 (accumulate); r32 = r64 and the
// partials of (r32, r32) into the (r, r) buffer of the current iteration
// (convert).
struct MixArgs {
  long long n;
  int h, n_last;
  long long klast_div;
  cx<double>* x64;
  cx<float>* x32;
  const cx<double>* r64;
  cx<float>* r32;
  DevState* st;
  Partials parts;
  double inv_n;
  int gate;
  Batch bt;
  FastDiv fd_kd, fd_h;
  int w3;                // vectors in the wave-pass layout V
  FastDiv fd_w3n0;
  int w3g;
};

// Folding of a wide producer's partials (see fold_partials_kernel).
struct FoldArgs {
  DevState* st;
  Partials parts;
  int region;            // PART_RR0 (count nparts[0]) or PART_PQ (count nparts_pq)
  int eq_region;         // region sharing the count (PART_EQ0), or -1
  int gate;
  Batch bt;
};
// Producers with more blocks than this have their partials folded.
constexpr long long kFoldAbove = 4096;

struct FinArgs {
  DevState* st;
  Partials parts;
  int mode;
  int n;                 // partials to sum (AUX modes)
  int d;
  double inv_n;
  int gate;
  Batch bt;
  int eq;                // the equilibrium sums beside the (r, r) sums are present
};

// ---------------------------------------------------------------------------
// Wave passes of 3-D grids whose axes are 27, 81 or 243 long (wave3d.hip).
// The last-axis half spectrum (h = N2 / 2 + 1 entries) is padded to
// G = ceil(h / 8) groups of 8 (cg, cc), c = 8 cg + cc; padded entries hold
// zeros.  Per problem, with (a, b) the indices of axes 0 and 1:
//   V  (CG vectors x, r, p, q): ((b G + cg) 8 + cc) N0 + a   (axis 0 fastest)
//   Gl (axis-0 inverse -> axis-1 inverse): ((b G + cg) N0 + a) 8 + cc
//   Hl (axis-1 inverse -> row pass -> axis-1 forward -> axis-0 forward,
//       in place): ((a G + cg) N1 + b) 8 + cc
// so that every pass writes whole tiles contiguously.
// ---------------------------------------------------------------------------
constexpr int kW3Group = 8;

__host__ __device__ constexpr int w3_groups(int h) { return (h + kW3Group - 1) / kW3Group; }
// axis lengths the wave FFTs take (nine points per lane, whole sequences per wave)
__host__ __device__ constexpr bool wave_fft_length(long long n) { return n == 27 || n == 81 || n == 243; }

enum W3Pass : int {
  W3_INV0 = 0,    // axis-0 inverse from the scalar c (or the CG direction step)
  W3_COL1 = 1,    // axis-1 transform Gl -> Hl (inverse) or Hl -> Hl (forward)
  W3_ROW = 2,     // row pass (modes of RowMode, flags of RowFlags)
  W3_FWD0 = 3,    // axis-0 forward + projection
};

template <typename T>
struct W3Args {
  int N0, N1, N2, h, G;
  long long nhp;                 // padded entries per problem (N0 N1 G 8)
  cx<T>* gl[kMaxDim];
  cx<T>* hl[kMaxDim];
  const cx<T>* tw[kMaxDim];      // exp(-2 pi i m / N_a), per axis
  double cinv[kMaxDim];          // 1 / cell side lengths: wave vector xi = k / Y
  // W3_INV0
  const cx<T>* c_in;
  cx<T>* p_io;
  const cx<T>* r_in;
  int cg_step;
  cx<T>* x_io;                   // CG step: applies a pending x += alpha_log p (x_pend)
  // W3_COL1
  int dir;
  int clear_xpend;               // the lead block clears x_pend (after the direction step)
  // W3_ROW
  int mode, flags;
  const double* real_in[kMaxDim];
  double* real_out[kMaxDim];
  const double* real_add[kMaxDim];
  const uint8_t* phase;
  const T* cond;
  int n_phases;
  T l0;
  T E[kMaxDim];
  T inv_n;
  // W3_FWD0: out = coef_base base + coef_s [1 / l0] (-i khat) . tau_hat
  cx<T>* out;
  const cx<T>* base;
  T coef_base, coef_s;
  int s_inv_l0;
  double l0d;
  int dot, dot_region;
  DevState* st;
  Partials parts;
  int gate;
  double inv_nd;
  Batch bt;
};

// Blocks of one problem of each wave pass, and their launchers.
long long w3_blocks(int pass, int N0, int N1, int N2);
template <typename T> hipError_t launch_w3(int pass, const W3Args<T>& a, hipStream_t s);
// Entries of the padded spectral layout per problem.
__host__ __device__ inline long long w3_entries(long long N0, long long N1, long long N2) {
  return N0 * N1 * (long long)w3_groups((int)(N2 / 2 + 1)) * kW3Group;
}

// Host launchers (passes.hip).
template <typename T> hipError_t launch_row(const RowArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_col(const ColArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_update(const UpdArgs<T>& a, hipStream_t s);
// x += alpha_log p for every problem whose update was deferred and not yet
// applied (the end of a CG loop), then x_pend cleared.
template <typename T> hipError_t launch_flush_x(const UpdArgs<T>& a, hipStream_t s);
hipError_t launch_pipe_update(const PipeArgs<double>& a, hipStream_t s);
hipError_t launch_finalize(const FinArgs& a, hipStream_t s);
hipError_t launch_fold_partials(const FoldArgs& a, hipStream_t s);
hipError_t launch_mix_accumulate(const MixArgs& a, hipStream_t s);
hipError_t launch_mix_convert(const MixArgs& a, hipStream_t s);
hipError_t launch_bicg(const BicgArgs& a, hipStream_t s);
long long bicg_blocks(const BicgArgs& a);
hipError_t launch_state_init(DevState* st, const DevState& init, hipStream_t s);
// copy nprob initial states from device memory src into st
hipError_t launch_state_copy(DevState* st, const DevState* src, int nprob, hipStream_t s);
// live[0..rows): the problems whose state is not done, in index order, then
// done problems to fill the rows (the host picks rows >= the count not done).
hipError_t launch_compact_live(const DevState* st, int nprob, int rows, int* live, hipStream_t s);
template <typename T> hipError_t launch_fill_zero(cx<T>* p, long long n, hipStream_t s);
hipError_t launch_max_phase(const uint8_t* ph, long long n, unsigned* out, hipStream_t s);
// counts[0..256): nodes of each phase index (counts zero on entry)
hipError_t launch_phase_histogram(const uint8_t* ph, long long n, unsigned* counts, hipStream_t s);

template <typename T> long long row_blocks(const RowArgs<T>& a);
template <typename T> long long col_blocks(const ColArgs<T>& a);
long long update_blocks(long long n);

// Dynamic LDS of a launch (sequence data + twiddles + phase bytes).
// comps: components per row-pass block (1 when split, else d)
size_t row_lds_bytes(int n, int rows_per_block, int comps, int elem_bytes, int n_phases, int* ss_out);
size_t col_lds_bytes(int L, int tile, int d, int elem_bytes, int* ss_out);
int lds_odd_stride(int n);

}  // namespace lshom
