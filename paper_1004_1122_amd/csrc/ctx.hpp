// Library context, problem groups, workspace layout and the solve drivers
// (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "lshom.h"
#include "plan.hpp"

struct lshom_ctx;

namespace lshom {

constexpr size_t kAlign = 256;
constexpr int kMaxPhases = kCondStride;
// Dynamic LDS per block.  gfx950 gives a workgroup up to 160 KiB; the pass
// kernels' static LDS (reduction scratch) stays under 1 KiB.  The default
// shapes aim at kLdsPreferred so that two or more blocks of a pass share a
// CU; shapes up to the device's limit (wider tiles found by the autotuner,
// grids whose smallest shape needs more) are accepted as well.
constexpr size_t kLdsStaticReserve = 1024;
constexpr size_t kLdsLimit = 160 * 1024 - kLdsStaticReserve;
constexpr size_t kLdsPreferred = 63 * 1024;
constexpr long long kMinBlocks = 128;

// Offsets (bytes from the workspace base) of everything a group of nprob
// problems of one grid needs.  Per-problem arrays are consecutive.
struct Layout {
  size_t total = 0;
  size_t off_state = 0, off_partials = 0, off_cond64 = 0, off_cond32 = 0, off_scratch = 0;
  size_t off_tab = 0, off_live = 0;
  size_t off_tw64[3] = {0, 0, 0}, off_tw32[3] = {0, 0, 0};
  size_t off_v64[4] = {0, 0, 0, 0}, off_w64[3] = {0, 0, 0};
  size_t off_v32[4] = {0, 0, 0, 0}, off_w32[3] = {0, 0, 0};
  // wave passes (3-D grids of 27/81/243): the axis-0 inverse output Gl
  size_t off_g64[3] = {0, 0, 0}, off_g32[3] = {0, 0, 0};
  // BiCG: real d x |N| FP64 fields x, r, r*, p, p*, A p, A^T p* (single problems)
  size_t off_bicg[7] = {0, 0, 0, 0, 0, 0, 0};
  long long part_stride = 0;  // doubles per partial region
  long long pstride = 0;      // doubles per problem (all regions)
  bool has32 = false;
  bool has_bicg = false;
};

template <typename T>
struct Bufs {
  cx<T>* v[4];   // x, r, p, q (half spectrum) of problem 0
  cx<T>* w[3];   // per-component pass buffers of problem 0
  cx<T>* gl[3];  // wave passes: axis-0 inverse output (layout Gl)
  const T* cond;
  const cx<T>* tw[3];
  PassShape shape;
  FftPlan plan[3];
};

// Launch schedule of one grid at one precision: radix order per axis and
// pass shapes (chosen by default heuristics or by the autotuner).
struct Schedule {
  FftPlan plan[3];
  PassShape shape;
  double ms_per_iter = 0.0;   // autotuned cost of one CG iteration's passes
  int tail_rows = 0;          // > 0: for batched launches of at most this many unfinished problems
};

using SchedKey = std::tuple<int, int64_t, int64_t, int64_t, int>;  // d, N0, N1, N2, precision

// HIP-event timing of the CG-loop pass launches of real solves.
struct PassTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;   // start/end event of pending launch i at 2i, 2i+1
  std::vector<int> kinds;         // pass class of each pending launch
  double ms[LSHOM_PASS_COUNT] = {};
  double bytes[LSHOM_PASS_COUNT] = {};
  long long launches[LSHOM_PASS_COUNT] = {};
  double unit_bytes[LSHOM_PASS_COUNT] = {};  // per problem-iteration, current solve
  void reset() {
    kinds.clear();
    for (int k = 0; k < LSHOM_PASS_COUNT; ++k) ms[k] = bytes[k] = 0.0, launches[k] = 0;
  }
};

// Problems that share one grid (d, N) and are advanced by the same launches.
struct Group {
  lshom_ctx* ctx = nullptr;     // errors and the context stream
  hipStream_t stream = nullptr; // the group's own stream (batched groups run concurrently), else the context's
  int d = 0;
  int64_t N[3] = {1, 1, 1};
  long long nvox = 0, nrows = 0, nhalf = 0;
  // wave passes: the grid qualifies (3-D, axes of 27, 81 or 243 nodes,
  // isotropic phases), they are in use for the current solve, the padded
  // spectral entries per problem, and the entries allocated per problem and
  // vector (the larger of nhalf and nhp where the grid qualifies)
  bool w3ok = false;
  bool w3 = false;
  long long nhp = 0, nvec = 0;
  int h = 0;
  bool transposed = false;      // 2-D spectral arrays stored [k1][k0]
  FftPlan plan64[3], plan32[3];
  PassShape shape64{2, 1, 1, 0, 0, 0}, shape32{2, 1, 1, 0, 0, 0};
  int n_phases = 1;             // conductivity-table entries staged per problem
  int n_phase_ids = 1;          // phases (table entries per phase: 1, or d (d + 1) / 2 for tensors)
  bool tensor = false;          // symmetric tensor phases (row pass keeps all components together)
  double cell_inv[3] = {1.0, 1.0, 1.0};  // 1 / cell side lengths (wave vector xi = k / Y)
  // single problem (nprob == 1, batched == false)
  const uint8_t* phase = nullptr;
  double l0 = 0.0;              // l0, or tr(L0) / d for an anisotropic reference
  bool aniso = false;           // anisotropic reference L0 (needs tensor)
  double L0u[6] = {0, 0, 0, 0, 0, 0};  // L0, upper triangle row by row
  double L0n[6] = {0, 0, 0, 0, 0, 0};  // L0 / l0
  // batch
  int nprob = 1;
  bool batched = false;         // per-problem data come from the device table
  // grid rows of the iteration launches once finished problems are dropped
  // (0: one row per problem, no indirection)
  int live_rows = 0;
  // schedules for launches of at most tail_rows unfinished problems (per precision)
  Schedule tail_sched[2];
  bool has_tail[2] = {false, false};
  int tail_rows = 0;
  // device memory
  char* ws = nullptr;
  Layout lay;
  std::vector<DevState> host_states;
  int warm_used = 0;
  std::vector<int> warm_flags;  // warm start taken, per problem
  bool warm_any = false;        // batched: some problem brings a warm start
  std::vector<int> warm_has;    // batched: problem p brings one
  std::map<std::pair<int, int>, hipGraphExec_t>* graph_cache = nullptr;
  bool in_cg = false;           // the CG-loop passes are being queued (timed when enabled)
  bool eq = false;              // the iteration loop forms the equilibrium norm (FP64)
  PassTimer* timer = nullptr;   // event timing of the CG-loop passes (null: off)
};

// Fills the geometry, plans and shapes of g (from the context's schedule
// registry when it has an entry for the grid); UNSUPPORTED if a pass cannot
// hold its FFT batch in LDS.
lshom_status group_setup(Group& g, int d, const int64_t* N, int n_phases, bool tensor = false);
// Default pass shape: the one for kLdsPreferred when it fits, else the one for
// the limit; *fits tells whether the result fits within `limit`.
PassShape default_shape_within(int d, const int64_t* N, const FftPlan* plans, int elem_bytes, size_t limit,
                               bool transposed, int n_phases, bool allow_split, bool* fits);
size_t lds_limit_of(const Group& g);
bool schedule_fits(const Group& g, const Schedule& s, int precision);
void apply_schedule(Group& g, const Schedule& s, int precision);
Schedule current_schedule(const Group& g, int precision);

// Times the passes of one CG iteration for candidate schedules on the group's
// current data and returns the fastest (per pass, independently).
lshom_status autotune_group(Group& g, int precision, int reps, Schedule* best);
// The same with the launches restricted to the first `rows` problems of the
// group (the tail of a batch); best->tail_rows = rows.
constexpr int kTailRows = 2;
lshom_status autotune_tail(Group& g, int precision, int reps, int rows, Schedule* best);
Layout compute_layout(const Group& g, bool with32, bool with_bicg = false);

// Uploads twiddles, conductivity tables (cond[p * n_phases + i]) and the
// problem table; checks every phase index.
lshom_status prepare_workspace(Group& g, const std::vector<double>& cond, const std::vector<ProbEntry>* tab,
                               const std::vector<const uint8_t*>& phases);

// Solve every problem of the group.  init[p]: initial scalars (b2, tol2b2,
// max_iter, mixed controls).  x0 (single problem only) may be null.
lshom_status solve_group(Group& g, const std::vector<DevState>& init, const lshom_solve_opts& o,
                         const double* E_single, const double* x0, double* e_single);
lshom_status apply_real(Group& g, const double* p, double* q);
// BiCG (single problem, FP64, workspace with the BiCG fields): e_out may be null.
lshom_status solve_bicg(Group& g, const DevState& init, const lshom_solve_opts& o, double* e_out);
lshom_status solve_pipecg(Group& g, const DevState& init, const lshom_solve_opts& o, double* e_out);
lshom_status time_passes(Group& g, int precision, int reps, double* ms_out, double* bytes_out);
// Algorithmic HBM bytes of each pass class for one problem and one CG iteration.
void pass_model_bytes(const Group& g, int precision, double* out, bool basic_scheme = false);

lshom_status fail(lshom_ctx* c, lshom_status s, const std::string& msg);
// Serialises graph captures against host-staged uploads and events on the
// caller's stream across contexts (concurrent solves on several threads).
std::mutex& setup_mutex();
void drop_graphs(std::map<std::pair<int, int>, hipGraphExec_t>& cache);
void drop_batch_graphs(lshom_ctx* c);

}  // namespace lshom

struct lshom_ctx {
  int device = 0;
  // dynamic LDS a block may use on this device (hipDeviceAttributeMaxSharedMemoryPerBlock
  // less the static reserve, at most kLdsLimit)
  size_t lds_limit = lshom::kLdsLimit;
  hipStream_t user_stream = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  std::string err;
  bool have_problem = false;
  bool ws_ready = false;
  std::vector<double> cond;
  lshom::Group g;               // the single problem of set_microstructure
  size_t ws_bytes = 0;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  // iteration graphs of batched groups, per (workspace address, grid, problem
  // count, phase count, layout); valid while the schedules stay unchanged
  std::map<std::vector<long long>, std::map<std::pair<int, int>, hipGraphExec_t>> batch_graphs;
  std::map<lshom::SchedKey, lshom::Schedule> schedules;  // autotuned or set by the caller
  lshom::PassTimer timer;
  // streams of the grid groups of a batched solve (one host thread each)
  std::vector<hipStream_t> group_streams;
  std::mutex err_mutex;  // fail() from those threads
};

#define HIP_TRY(ctx, expr)                                                                       \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return ::lshom::fail((ctx), LSHOM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
