// Library context, workspace layout and the solve drivers (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "lshom.h"
#include "plan.hpp"

namespace lshom {

constexpr size_t kAlign = 256;
constexpr int kMaxPhases = 256;
// dynamic LDS per block; the rest of the 64 KiB holds the reductions' statics
constexpr size_t kLdsBudget = 63 * 1024;
constexpr long long kMinBlocks = 128;

struct Layout {
  size_t total = 0;
  size_t off_state = 0, off_partials = 0, off_cond64 = 0, off_cond32 = 0, off_scratch = 0;
  size_t off_tw64[3] = {0, 0, 0}, off_tw32[3] = {0, 0, 0};
  size_t off_v64[4] = {0, 0, 0, 0}, off_w64[3] = {0, 0, 0};
  size_t off_v32[4] = {0, 0, 0, 0}, off_w32[3] = {0, 0, 0};
  long long part_stride = 0;  // doubles per partial region
  bool has32 = false;
};

template <typename T>
struct Bufs {
  cx<T>* v[4];   // x, r, p, q (half spectrum)
  cx<T>* w[3];   // per-component pass buffers
  const T* cond;
  const cx<T>* tw[3];
  PassShape shape;
};

}  // namespace lshom

struct lshom_ctx {
  int device = 0;
  hipStream_t user_stream = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  std::string err;
  // problem
  bool have_problem = false;
  int d = 0;
  int64_t N[3] = {0, 0, 0};
  long long nvox = 0, nrows = 0, nhalf = 0;
  int h = 0;
  bool transposed = false;     // 2-D spectral arrays stored [k1][k0]
  const uint8_t* phase = nullptr;
  std::vector<double> cond;
  double l0 = 0.0;
  lshom::FftPlan plan[3];
  lshom::PassShape shape64{2, 1, 1}, shape32{2, 1, 1};
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_ready = false;
  lshom::Layout lay;
  lshom::DevState* host_state = nullptr;  // pinned host copy of the device scalars
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
};

namespace lshom {

lshom_status fail(lshom_ctx* c, lshom_status s, const std::string& msg);
void drop_graphs(lshom_ctx* c);
Layout compute_layout(const lshom_ctx* c, bool with32);
lshom_status prepare_workspace(lshom_ctx* c);  // tables, phase check

lshom_status solve_fp64(lshom_ctx* c, const double* E, double tol, const lshom_solve_opts& o,
                        const double* x0, double* e_out, double* leff, lshom_solve_info* info);
lshom_status solve_mixed(lshom_ctx* c, const double* E, double tol, const lshom_solve_opts& o,
                         const double* x0, double* e_out, double* leff, lshom_solve_info* info);
lshom_status apply_real(lshom_ctx* c, const double* p, double* q);
lshom_status time_passes(lshom_ctx* c, int precision, int reps, double* ms_out, double* bytes_out);

}  // namespace lshom

#define HIP_TRY(ctx, expr)                                                                       \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return ::lshom::fail((ctx), LSHOM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
