// C ABI of the lshom library: validation, context, workspace carving and the
// CG drivers that queue the pass kernels.  See include/lshom.h.
#include "lshom.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"

using namespace lshom;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxPhases = 256;
// dynamic LDS per block; the rest of the 64 KiB holds the reductions' statics
constexpr size_t kLdsBudget = 63 * 1024;
constexpr long long kMinBlocks = 512;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t total = 0;
  size_t off_state = 0, off_partials = 0, off_cond64 = 0, off_cond32 = 0;
  size_t off_tw64[3] = {0, 0, 0}, off_tw32[3] = {0, 0, 0};
  size_t off_v64[4] = {0, 0, 0, 0}, off_w64[3] = {0, 0, 0};
  size_t off_v32[4] = {0, 0, 0, 0}, off_w32[3] = {0, 0, 0};
  size_t partials_len = 0;
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

}  // namespace

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
  const uint8_t* phase = nullptr;
  std::vector<double> cond;
  double l0 = 0.0;
  FftPlan plan[3];
  PassShape shape64{1, 1, 1}, shape32{1, 1, 1};
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_ready = false;
  Layout lay;
  DevState* host_state = nullptr;  // pinned host copy of the device scalars
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
};

namespace {

lshom_status fail(lshom_ctx* c, lshom_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIP_TRY(ctx, expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail((ctx), LSHOM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

void drop_graphs(lshom_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

Layout compute_layout(const lshom_ctx* c, bool with32) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.off_state = take(sizeof(DevState));
  // partial sums: one slot of up to 4 doubles per block of the widest launch
  long long maxb = 1;
  for (int prec = 0; prec < (with32 ? 2 : 1); ++prec) {
    const PassShape& s = prec == 0 ? c->shape64 : c->shape32;
    maxb = std::max(maxb, ceil_div(c->nrows, s.rows_per_block));
    long long inner0 = c->h;
    for (int a = 1; a < c->d - 1; ++a) inner0 *= c->N[a];
    maxb = std::max(maxb, ceil_div(inner0, s.tile0));
    if (c->d == 3) maxb = std::max(maxb, c->N[0] * ceil_div(c->h, s.tile1));
  }
  maxb = std::max(maxb, update_blocks(c->nhalf));
  L.partials_len = (size_t)maxb * 4;
  L.off_partials = take(L.partials_len * sizeof(double));
  L.off_cond64 = take(kMaxPhases * sizeof(double));
  L.off_cond32 = take(kMaxPhases * sizeof(float));
  for (int a = 0; a < c->d; ++a) {
    L.off_tw64[a] = take((size_t)c->N[a] * sizeof(cx<double>));
    L.off_tw32[a] = take((size_t)c->N[a] * sizeof(cx<float>));
  }
  for (int i = 0; i < 4; ++i) L.off_v64[i] = take((size_t)c->nhalf * sizeof(cx<double>));
  for (int a = 0; a < c->d; ++a) L.off_w64[a] = take((size_t)c->nhalf * sizeof(cx<double>));
  L.has32 = with32;
  if (with32) {
    for (int i = 0; i < 4; ++i) L.off_v32[i] = take((size_t)c->nhalf * sizeof(cx<float>));
    for (int a = 0; a < c->d; ++a) L.off_w32[a] = take((size_t)c->nhalf * sizeof(cx<float>));
  }
  L.total = off;
  return L;
}

template <typename T>
Bufs<T> get_bufs(lshom_ctx* c);

template <>
Bufs<double> get_bufs<double>(lshom_ctx* c) {
  Bufs<double> b{};
  for (int i = 0; i < 4; ++i) b.v[i] = reinterpret_cast<cx<double>*>(c->ws + c->lay.off_v64[i]);
  for (int a = 0; a < c->d; ++a) {
    b.w[a] = reinterpret_cast<cx<double>*>(c->ws + c->lay.off_w64[a]);
    b.tw[a] = reinterpret_cast<const cx<double>*>(c->ws + c->lay.off_tw64[a]);
  }
  b.cond = reinterpret_cast<const double*>(c->ws + c->lay.off_cond64);
  b.shape = c->shape64;
  return b;
}

template <>
Bufs<float> get_bufs<float>(lshom_ctx* c) {
  Bufs<float> b{};
  for (int i = 0; i < 4; ++i) b.v[i] = reinterpret_cast<cx<float>*>(c->ws + c->lay.off_v32[i]);
  for (int a = 0; a < c->d; ++a) {
    b.w[a] = reinterpret_cast<cx<float>*>(c->ws + c->lay.off_w32[a]);
    b.tw[a] = reinterpret_cast<const cx<float>*>(c->ws + c->lay.off_tw32[a]);
  }
  b.cond = reinterpret_cast<const float*>(c->ws + c->lay.off_cond32);
  b.shape = c->shape32;
  return b;
}

DevState* dev_state(lshom_ctx* c) { return reinterpret_cast<DevState*>(c->ws + c->lay.off_state); }
double* dev_partials(lshom_ctx* c) { return reinterpret_cast<double*>(c->ws + c->lay.off_partials); }

// ---------------------------------------------------------------------------
// Pass argument builders
// ---------------------------------------------------------------------------

template <typename T>
ColArgs<T> col0_args(lshom_ctx* c, const Bufs<T>& b) {
  ColArgs<T> a{};
  a.L = (int)c->N[0];
  a.inner = c->h;
  for (int t = 1; t < c->d - 1; ++t) a.inner *= c->N[t];
  a.outer = 1;
  a.tile = b.shape.tile0;
  a.tiles_per_outer = (int)ceil_div(a.inner, a.tile);
  a.d = c->d;
  col_lds_bytes(a.L, a.tile, a.d, (int)sizeof(cx<T>), &a.ss);
  for (int t = 0; t < c->d; ++t) {
    a.comp[t] = b.w[t];
    a.nd[t] = (int)c->N[t];
  }
  a.dims = c->d;
  a.h = c->h;
  a.plan = c->plan[0];
  a.tw = b.tw[0];
  a.st = dev_state(c);
  a.partials = dev_partials(c);
  a.inv_n = 1.0 / (double)c->nvox;
  a.gate = GATE_ACTIVE;
  a.fin = FIN_NONE;
  return a;
}

template <typename T>
ColArgs<T> col1_args(lshom_ctx* c, const Bufs<T>& b, int dir) {
  ColArgs<T> a{};
  a.L = (int)c->N[1];
  a.inner = c->h;
  a.outer = c->N[0];
  a.tile = b.shape.tile1;
  a.tiles_per_outer = (int)ceil_div(a.inner, a.tile);
  a.d = c->d;
  col_lds_bytes(a.L, a.tile, a.d, (int)sizeof(cx<T>), &a.ss);
  for (int t = 0; t < c->d; ++t) {
    a.comp[t] = b.w[t];
    a.nd[t] = (int)c->N[t];
  }
  a.dims = c->d;
  a.h = c->h;
  a.mode = COL_PLAIN;
  a.dir = dir;
  a.plan = c->plan[1];
  a.tw = b.tw[1];
  a.st = dev_state(c);
  a.partials = dev_partials(c);
  a.inv_n = 1.0 / (double)c->nvox;
  a.gate = GATE_ACTIVE;
  a.fin = FIN_NONE;
  return a;
}

template <typename T>
RowArgs<T> row_args(lshom_ctx* c, const Bufs<T>& b) {
  RowArgs<T> a{};
  const int last = c->d - 1;
  a.n = (int)c->N[last];
  a.h = c->h;
  a.nrows = c->nrows;
  a.rows_per_block = b.shape.rows_per_block;
  a.d = c->d;
  row_lds_bytes(a.n, a.rows_per_block, a.d, (int)sizeof(cx<T>), &a.ss);
  for (int t = 0; t < c->d; ++t) a.spec[t] = b.w[t];
  a.phase = c->phase;
  a.cond = b.cond;
  a.l0 = (T)c->l0;
  a.inv_n = (T)(1.0 / (double)c->nvox);
  a.plan = c->plan[last];
  a.tw = b.tw[last];
  a.st = dev_state(c);
  a.partials = dev_partials(c);
  a.gate = GATE_ACTIVE;
  a.fin = FIN_NONE;
  return a;
}

// ---------------------------------------------------------------------------
// Operator sequences (see the pass kernels for the algebra)
// ---------------------------------------------------------------------------

// Forward half: [3-D axis-1 forward], axis-0 forward + projection.
template <typename T>
hipError_t enq_forward_project(lshom_ctx* c, const Bufs<T>& b, cx<T>* out, const cx<T>* base,
                               T coef_base, T coef_s, int dot, int fin, int gate) {
  hipError_t e;
  if (c->d == 3) {
    ColArgs<T> m = col1_args(c, b, -1);
    m.gate = gate;
    if ((e = launch_col(m, c->stream)) != hipSuccess) return e;
  }
  ColArgs<T> a = col0_args(c, b);
  a.mode = COL_FWD_PROJ;
  a.out = out;
  a.base = base;
  a.coef_base = coef_base;
  a.coef_s = coef_s;
  a.dot = dot;
  a.fin = fin;
  a.gate = gate;
  return launch_col(a, c->stream);
}

// Inverse half: axis-0 inverse from the scalar c (or p = r + beta p), [axis-1].
template <typename T>
hipError_t enq_inverse_from_c(lshom_ctx* c, const Bufs<T>& b, const cx<T>* c_in, cx<T>* p_io,
                              const cx<T>* r_in, int gate) {
  hipError_t e;
  ColArgs<T> a = col0_args(c, b);
  a.mode = COL_INV_C;
  a.c_in = c_in;
  a.p_io = p_io;
  a.r_in = r_in;
  a.fuse_p = p_io != nullptr;
  a.gate = gate;
  if ((e = launch_col(a, c->stream)) != hipSuccess) return e;
  if (c->d == 3) {
    ColArgs<T> m = col1_args(c, b, +1);
    m.gate = gate;
    if ((e = launch_col(m, c->stream)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// out = coef_base * base + coef_s * (-i khat) . F[dL (E + u(c_in))]
template <typename T>
hipError_t enq_apply_spec(lshom_ctx* c, const Bufs<T>& b, const cx<T>* c_in, cx<T>* p_io,
                          const cx<T>* r_in, const double* E, cx<T>* out, const cx<T>* base,
                          T coef_base, T coef_s, int dot, int fin, int gate) {
  hipError_t e;
  if ((e = enq_inverse_from_c(c, b, c_in, p_io, r_in, gate)) != hipSuccess) return e;
  RowArgs<T> r = row_args(c, b);
  r.mode = ROW_FUSED;
  for (int t = 0; t < c->d; ++t) r.E[t] = E ? (T)E[t] : T(0);
  r.gate = gate;
  if ((e = launch_row(r, c->stream)) != hipSuccess) return e;
  return enq_forward_project(c, b, out, base, coef_base, coef_s, dot, fin, gate);
}

// One CG iteration (Saad's Algorithm 6.18 in the spectral coordinate).
template <typename T>
hipError_t enq_cg_iteration(lshom_ctx* c, const Bufs<T>& b, int gate) {
  hipError_t e;
  cx<T>* x = b.v[0];
  cx<T>* r = b.v[1];
  cx<T>* p = b.v[2];
  cx<T>* q = b.v[3];
  // p = r + beta p;  q = p + (1/l0) P dL u(p);  alpha = (r,r)/(p,q)
  if ((e = enq_apply_spec<T>(c, b, nullptr, p, r, nullptr, q, p, T(1), T(1.0 / c->l0), 1, FIN_ALPHA,
                             gate)) != hipSuccess)
    return e;
  UpdArgs<T> u{};
  u.n = c->nhalf;
  u.h = c->h;
  u.n_last = (int)c->N[c->d - 1];
  u.x = x;
  u.r = r;
  u.p = p;
  u.q = q;
  u.st = dev_state(c);
  u.partials = dev_partials(c);
  u.inv_n = 1.0 / (double)c->nvox;
  u.blocks = (int)update_blocks(c->nhalf);
  u.gate = gate;
  return launch_update(u, c->stream);
}

// Residual of the iterate x (spectral) for the load E: r = -(x + (1/l0) P dL (E + u(x))).
template <typename T>
hipError_t enq_true_residual(lshom_ctx* c, const Bufs<T>& b, const cx<T>* x, const double* E,
                             cx<T>* out, int fin, int gate) {
  return enq_apply_spec<T>(c, b, x, nullptr, nullptr, E, out, x, T(-1), T(-1.0 / c->l0), 2, fin,
                           gate);
}

// r0 for x0 = E: r0 = -(1/l0) P dL E.
template <typename T>
hipError_t enq_residual_of_E(lshom_ctx* c, const Bufs<T>& b, const double* E, cx<T>* out,
                             int fin) {
  hipError_t e;
  RowArgs<T> r = row_args(c, b);
  r.mode = ROW_FWD;
  r.flags = ROWF_DL | ROWF_CONST_E;
  for (int t = 0; t < c->d; ++t) r.E[t] = (T)E[t];
  r.gate = GATE_ALWAYS;
  if ((e = launch_row(r, c->stream)) != hipSuccess) return e;
  return enq_forward_project<T>(c, b, out, nullptr, T(0), T(-1.0 / c->l0), 2, fin, GATE_ALWAYS);
}

// Real FP64 field v (d x |N|) -> spectral coordinate of P v (optionally of P dL v / l0).
hipError_t enq_project_real(lshom_ctx* c, const Bufs<double>& b, const double* v, bool with_dl,
                            cx<double>* out) {
  hipError_t e;
  RowArgs<double> r = row_args(c, b);
  r.mode = ROW_FWD;
  r.flags = with_dl ? ROWF_DL : 0;
  for (int t = 0; t < c->d; ++t) r.real_in[t] = v + (size_t)t * c->nvox;
  r.gate = GATE_ALWAYS;
  if ((e = launch_row(r, c->stream)) != hipSuccess) return e;
  return enq_forward_project<double>(c, b, out, nullptr, 0.0, with_dl ? 1.0 / c->l0 : 1.0, 0,
                                     FIN_NONE, GATE_ALWAYS);
}

// Real field out = add + E + u(x), with <lambda out> reduced into leff.
hipError_t enq_field_out(lshom_ctx* c, const Bufs<double>& b, const cx<double>* x, const double* E,
                         const double* add, double* out, bool leff) {
  hipError_t e;
  if ((e = enq_inverse_from_c<double>(c, b, x, nullptr, nullptr, GATE_ALWAYS)) != hipSuccess) return e;
  RowArgs<double> r = row_args(c, b);
  r.mode = ROW_INV;
  r.flags = (add ? ROWF_ADD : 0) | (leff ? ROWF_LEFF : 0);
  for (int t = 0; t < c->d; ++t) {
    r.E[t] = E ? E[t] : 0.0;
    r.real_out[t] = out ? out + (size_t)t * c->nvox : nullptr;
    r.real_add[t] = add ? add + (size_t)t * c->nvox : nullptr;
  }
  r.fin = leff ? FIN_LEFF : FIN_NONE;
  r.gate = GATE_ALWAYS;
  return launch_row(r, c->stream);
}

lshom_status check_ready(lshom_ctx* c, int precision) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return fail(c, LSHOM_ERR_STATE, "set_microstructure has not been called");
  if (!c->ws_ready) return fail(c, LSHOM_ERR_WORKSPACE, "no workspace attached for this problem");
  if (precision == LSHOM_PRECISION_MIXED && !c->lay.has32)
    return fail(c, LSHOM_ERR_WORKSPACE, "workspace was sized for FP64 only");
  return LSHOM_OK;
}

hipError_t sync_state(lshom_ctx* c) {
  hipError_t e = hipMemcpyAsync(c->host_state, dev_state(c), sizeof(DevState),
                                hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(c->stream);
}

hipError_t order_after_user(lshom_ctx* c) {
  hipError_t e = hipEventRecord(c->ev, c->user_stream);
  if (e != hipSuccess) return e;
  return hipStreamWaitEvent(c->stream, c->ev, 0);
}

// Mixed precision refresh (reliable update): x64 += x32, x32 = 0;
// r64 = b - A64 x64 in FP64 (convergence is decided on it); r32 = r64.
hipError_t enq_mix_refresh(lshom_ctx* c, const Bufs<double>& b64, const Bufs<float>& b32,
                           const double* E, int gate) {
  hipError_t e;
  MixArgs m{};
  m.n = c->nhalf;
  m.x64 = b64.v[0];
  m.x32 = b32.v[0];
  m.r64 = b64.v[1];
  m.r32 = b32.v[1];
  m.st = dev_state(c);
  m.partials = dev_partials(c);
  m.gate = gate;
  m.blocks = (int)update_blocks(c->nhalf);
  if ((e = launch_mix_accumulate(m, c->stream)) != hipSuccess) return e;
  if ((e = enq_true_residual<double>(c, b64, b64.v[0], E, b64.v[1], FIN_REFRESH, gate)) != hipSuccess)
    return e;
  m.clear_refresh = 1;
  return launch_mix_convert(m, c->stream);
}

// Run blocks of work until the device reports done.  A block is captured
// once into a HIP graph (key) and replayed; with K == 0 it is queued eagerly.
template <typename F>
lshom_status run_blocks(lshom_ctx* c, int key, int K, long long max_blocks, F&& enqueue_block) {
  HIP_TRY(c, sync_state(c));
  hipGraphExec_t ex = nullptr;
  if (K > 0) {
    auto gk = std::make_pair(key, K);
    auto it = c->graphs.find(gk);
    if (it == c->graphs.end()) {
      hipGraph_t g = nullptr;
      HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue_block();
      hipError_t e2 = hipStreamEndCapture(c->stream, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(c, LSHOM_ERR_HIP, std::string("graph capture failed: ") +
                                          hipGetErrorString(e != hipSuccess ? e : e2));
      }
      hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e3 != hipSuccess)
        return fail(c, LSHOM_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e3));
      c->graphs.emplace(gk, ex);
    } else {
      ex = it->second;
    }
  }
  // the device sets `done` at the latest after max_iter iterations; the
  // block bound only guards against a state that stopped advancing
  for (long long blocks = 0;; ++blocks) {
    if (c->host_state->done) break;
    if (blocks > max_blocks) return fail(c, LSHOM_ERR_HIP, "device CG state stopped advancing");
    if (ex) {
      HIP_TRY(c, hipGraphLaunch(ex, c->stream));
    } else {
      HIP_TRY(c, enqueue_block());
    }
    HIP_TRY(c, sync_state(c));
  }
  return LSHOM_OK;
}

template <typename T>
lshom_status run_iterations(lshom_ctx* c, const Bufs<T>& b, int K) {
  const int per = K > 0 ? K : 8;
  const long long max_blocks = c->host_state->max_iter / per + 4;
  return run_blocks(c, 0, K, max_blocks, [&]() -> hipError_t {
    for (int k = 0; k < per; ++k) {
      hipError_t e = enq_cg_iteration<T>(c, b, GATE_ACTIVE);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  });
}

DevState initial_state(const lshom_ctx* c, const double* E, double tol, int max_iter) {
  DevState s{};
  double e2 = 0.0;
  for (int t = 0; t < c->d; ++t) e2 += E[t] * E[t];
  s.b2 = e2 * (double)c->nvox;
  s.tol2b2 = tol * tol * s.b2;
  s.max_iter = max_iter;
  s.leff[0] = s.leff[1] = s.leff[2] = 0.0;
  return s;
}

lshom_status validate_opts(lshom_ctx* c, const lshom_solve_opts* o) {
  if (o->max_iter < 0) return fail(c, LSHOM_ERR_INVALID_ARG, "max_iter must be >= 0");
  if (o->precision != LSHOM_PRECISION_FP64 && o->precision != LSHOM_PRECISION_MIXED)
    return fail(c, LSHOM_ERR_INVALID_ARG, "precision must be FP64 (0) or MIXED (1)");
  if (o->graph_block < 0 || o->graph_block > 1024)
    return fail(c, LSHOM_ERR_INVALID_ARG, "graph_block must be in [0, 1024]");
  if (o->precision == LSHOM_PRECISION_MIXED) {
    if (o->refresh_every < 1) return fail(c, LSHOM_ERR_INVALID_ARG, "refresh_every must be >= 1");
    if (!(o->refresh_drop > 0.0 && o->refresh_drop < 1.0))
      return fail(c, LSHOM_ERR_INVALID_ARG, "refresh_drop must be in (0, 1)");
  }
  return LSHOM_OK;
}

// FP64 solve: the plain method.
lshom_status solve_fp64(lshom_ctx* c, const double* E, double tol, const lshom_solve_opts& o,
                        const double* x0, double* e_out, double* leff, lshom_solve_info* info) {
  Bufs<double> b = get_bufs<double>(c);
  cx<double>* x = b.v[0];
  cx<double>* r = b.v[1];
  cx<double>* p = b.v[2];
  cx<double>* q = b.v[3];
  DevState init = initial_state(c, E, tol, o.max_iter);
  HIP_TRY(c, launch_state_init(dev_state(c), init, c->stream));
  HIP_TRY(c, launch_fill_zero(x, c->nhalf, c->stream));
  HIP_TRY(c, launch_fill_zero(p, c->nhalf, c->stream));
  int warm_used = 0;
  if (x0) {
    // residual of E for the admissibility test, then of E + P x0
    HIP_TRY(c, (enq_residual_of_E<double>(c, b, E, r, FIN_AUX)));
    HIP_TRY(c, enq_project_real(c, b, x0, false, x));
    HIP_TRY(c, (enq_true_residual<double>(c, b, x, E, r, FIN_RR_INIT, GATE_ALWAYS)));
    HIP_TRY(c, sync_state(c));
    const DevState& hs = *c->host_state;
    if (std::isfinite(hs.rr) && hs.rr < hs.dot_aux) {
      warm_used = 1;
    } else {
      HIP_TRY(c, launch_state_init(dev_state(c), init, c->stream));
      HIP_TRY(c, launch_fill_zero(x, c->nhalf, c->stream));
    }
  }
  if (!warm_used) HIP_TRY(c, (enq_residual_of_E<double>(c, b, E, r, FIN_RR_INIT)));
  HIP_TRY(c, sync_state(c));
  lshom_status s = run_iterations<double>(c, b, o.graph_block);
  if (s != LSHOM_OK) return s;
  if (o.true_residual) HIP_TRY(c, (enq_true_residual<double>(c, b, x, E, q, FIN_RR_TRUE, GATE_ALWAYS)));
  HIP_TRY(c, enq_field_out(c, b, x, E, nullptr, e_out, true));
  HIP_TRY(c, sync_state(c));
  const DevState& hs = *c->host_state;
  if (leff)
    for (int t = 0; t < c->d; ++t) leff[t] = hs.leff[t];
  if (info) {
    info->iterations = hs.iter;
    info->applies_fp32 = 0;
    info->applies_fp64 = hs.applies64;
    info->status = hs.status;
    info->warm_start_used = warm_used;
    info->refreshes = 0;
    info->rel_res = std::sqrt(hs.rr / hs.b2);
    info->rel_res_true = o.true_residual ? std::sqrt(hs.rr_true / hs.b2) : -1.0;
    info->eta_r = c->l0 * std::sqrt(hs.rr / hs.b2);
  }
  return hs.status;
}

// Per-kernel timing of one CG iteration's launches (state set so that the
// vectors stay bounded: alpha = 0, beta = 0).
template <typename T>
lshom_status time_passes(lshom_ctx* c, const Bufs<T>& b, int reps, double* ms_out, double* bytes_out) {
  cx<T>* x = b.v[0];
  cx<T>* r = b.v[1];
  cx<T>* p = b.v[2];
  cx<T>* q = b.v[3];
  DevState init{};
  init.max_iter = 1 << 30;
  init.b2 = 1.0;
  HIP_TRY(c, launch_state_init(dev_state(c), init, c->stream));
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  const double cs = (double)sizeof(cx<T>);
  const double nh = (double)c->nhalf;
  const int d = c->d;
  for (int k = 0; k < LSHOM_PASS_COUNT; ++k) {
    ms_out[k] = 0.0;
    if (bytes_out) bytes_out[k] = 0.0;
  }
  auto timed = [&](int cls, double bytes, auto&& launch) -> hipError_t {
    hipError_t e = launch();  // warm-up
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) return e;
    for (int i = 0; i < reps; ++i)
      if ((e = launch()) != hipSuccess) return e;
    if ((e = hipEventRecord(e1, c->stream)) != hipSuccess) return e;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
    ms_out[cls] = (double)ms / reps;
    if (bytes_out) bytes_out[cls] = bytes;
    return hipSuccess;
  };
  hipError_t err = hipSuccess;
  {
    ColArgs<T> a = col0_args(c, b);
    a.mode = COL_INV_C;
    a.p_io = p;
    a.r_in = r;
    a.fuse_p = 1;
    a.gate = GATE_ALWAYS;
    err = timed(LSHOM_PASS_AXIS0_INVERSE, (3.0 + d) * nh * cs, [&] { return launch_col(a, c->stream); });
  }
  if (err == hipSuccess && d == 3) {
    ColArgs<T> m = col1_args(c, b, +1);
    m.gate = GATE_ALWAYS;
    err = timed(LSHOM_PASS_AXIS1_INVERSE, 2.0 * d * nh * cs, [&] { return launch_col(m, c->stream); });
    if (err == hipSuccess) {
      ColArgs<T> f = col1_args(c, b, -1);
      f.gate = GATE_ALWAYS;
      err = timed(LSHOM_PASS_AXIS1_FORWARD, 2.0 * d * nh * cs, [&] { return launch_col(f, c->stream); });
    }
  }
  if (err == hipSuccess) {
    RowArgs<T> r_ = row_args(c, b);
    r_.mode = ROW_FUSED;
    r_.gate = GATE_ALWAYS;
    err = timed(LSHOM_PASS_ROW, 2.0 * d * nh * cs + (double)c->nvox, [&] { return launch_row(r_, c->stream); });
  }
  if (err == hipSuccess) {
    ColArgs<T> a = col0_args(c, b);
    a.mode = COL_FWD_PROJ;
    a.out = q;
    a.base = p;
    a.coef_base = T(1);
    a.coef_s = T(1.0 / c->l0);
    a.dot = 1;
    a.fin = FIN_AUX;
    a.gate = GATE_ALWAYS;
    err = timed(LSHOM_PASS_AXIS0_FORWARD, (d + 2.0) * nh * cs, [&] { return launch_col(a, c->stream); });
  }
  if (err == hipSuccess) {
    UpdArgs<T> u{};
    u.n = c->nhalf;
    u.h = c->h;
    u.n_last = (int)c->N[c->d - 1];
    u.x = x;
    u.r = r;
    u.p = p;
    u.q = q;
    u.st = dev_state(c);
    u.partials = dev_partials(c);
    u.inv_n = 1.0 / (double)c->nvox;
    u.blocks = (int)update_blocks(c->nhalf);
    u.gate = GATE_ALWAYS;
    err = timed(LSHOM_PASS_UPDATE, 6.0 * nh * cs, [&] { return launch_update(u, c->stream); });
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(c, LSHOM_ERR_HIP, std::string("time_passes: ") + hipGetErrorString(err));
  c->err.clear();
  return LSHOM_OK;
}

// Mixed precision: FP32 operator, FP32 vectors, FP64 dots; FP64 iterate and
// FP64 true residual at every refresh (reliable update; p is kept).
lshom_status solve_mixed(lshom_ctx* c, const double* E, double tol, const lshom_solve_opts& o,
                         const double* x0, double* e_out, double* leff, lshom_solve_info* info) {
  Bufs<double> b64 = get_bufs<double>(c);
  Bufs<float> b32 = get_bufs<float>(c);
  cx<double>* x64 = b64.v[0];
  cx<double>* r64 = b64.v[1];
  DevState init = initial_state(c, E, tol, o.max_iter);
  init.refresh_every = o.refresh_every;
  init.drop2 = o.refresh_drop * o.refresh_drop;
  HIP_TRY(c, launch_state_init(dev_state(c), init, c->stream));
  HIP_TRY(c, launch_fill_zero(x64, c->nhalf, c->stream));
  for (int i : {0, 2}) HIP_TRY(c, launch_fill_zero(b32.v[i], c->nhalf, c->stream));
  int warm_used = 0;
  if (x0) {
    HIP_TRY(c, (enq_residual_of_E<double>(c, b64, E, r64, FIN_AUX)));
    HIP_TRY(c, enq_project_real(c, b64, x0, false, x64));
    HIP_TRY(c, (enq_true_residual<double>(c, b64, x64, E, r64, FIN_RR_INIT, GATE_ALWAYS)));
    HIP_TRY(c, sync_state(c));
    const DevState& hs = *c->host_state;
    if (std::isfinite(hs.rr) && hs.rr < hs.dot_aux) {
      warm_used = 1;
    } else {
      HIP_TRY(c, launch_state_init(dev_state(c), init, c->stream));
      HIP_TRY(c, launch_fill_zero(x64, c->nhalf, c->stream));
    }
  }
  if (!warm_used) HIP_TRY(c, (enq_residual_of_E<double>(c, b64, E, r64, FIN_RR_INIT)));
  {
    MixArgs m{};
    m.n = c->nhalf;
    m.r64 = r64;
    m.r32 = b32.v[1];
    m.st = dev_state(c);
    m.partials = dev_partials(c);
    m.gate = GATE_ALWAYS;
    m.blocks = (int)update_blocks(c->nhalf);
    HIP_TRY(c, launch_mix_convert(m, c->stream));
  }
  HIP_TRY(c, sync_state(c));
  const int K = o.graph_block;
  const int per = K > 0 ? K : 8;
  // a refresh may cut a block short, so at most one iteration per block is certain
  const long long max_blocks = (long long)c->host_state->max_iter + 4;
  lshom_status s = run_blocks(c, 1, K, max_blocks, [&]() -> hipError_t {
    for (int k = 0; k < per; ++k) {
      hipError_t e = enq_cg_iteration<float>(c, b32, GATE_NO_REFRESH);
      if (e != hipSuccess) return e;
    }
    return enq_mix_refresh(c, b64, b32, E, GATE_REFRESH);
  });
  if (s != LSHOM_OK) return s;
  {
    // fold what a breakdown left in the FP32 correction (no-op after a refresh)
    MixArgs m{};
    m.n = c->nhalf;
    m.x64 = x64;
    m.x32 = b32.v[0];
    m.st = dev_state(c);
    m.gate = GATE_ALWAYS;
    m.blocks = (int)update_blocks(c->nhalf);
    HIP_TRY(c, launch_mix_accumulate(m, c->stream));
  }
  if (o.true_residual) HIP_TRY(c, (enq_true_residual<double>(c, b64, x64, E, b64.v[3], FIN_RR_TRUE, GATE_ALWAYS)));
  HIP_TRY(c, enq_field_out(c, b64, x64, E, nullptr, e_out, true));
  HIP_TRY(c, sync_state(c));
  const DevState& hs = *c->host_state;
  if (leff)
    for (int t = 0; t < c->d; ++t) leff[t] = hs.leff[t];
  if (info) {
    info->iterations = hs.iter;
    info->applies_fp32 = hs.applies32;
    info->applies_fp64 = hs.n_refresh;
    info->status = hs.status;
    info->warm_start_used = warm_used;
    info->refreshes = hs.n_refresh;
    info->rel_res = std::sqrt(hs.rr / hs.b2);
    info->rel_res_true = o.true_residual ? std::sqrt(hs.rr_true / hs.b2) : -1.0;
    info->eta_r = c->l0 * std::sqrt(hs.rr / hs.b2);
  }
  return hs.status;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

const char* lshom_status_string(lshom_status s) {
  switch (s) {
    case LSHOM_OK: return "ok";
    case LSHOM_ERR_INVALID_ARG: return "invalid argument";
    case LSHOM_ERR_STATE: return "call order (state) error";
    case LSHOM_ERR_WORKSPACE: return "workspace missing or too small";
    case LSHOM_ERR_HIP: return "HIP runtime error";
    case LSHOM_ERR_NOT_CONVERGED: return "not converged within max_iter";
    case LSHOM_ERR_BREAKDOWN: return "CG breakdown ((p, Ap) <= 0 or not finite)";
    case LSHOM_ERR_UNSUPPORTED: return "unsupported input";
    default: return "unknown status";
  }
}

const char* lshom_last_error(const lshom_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

void lshom_default_opts(lshom_solve_opts* o) {
  if (!o) return;
  o->max_iter = 10000;
  o->precision = LSHOM_PRECISION_FP64;
  o->refresh_every = 50;
  o->refresh_drop = 0.1;
  o->graph_block = 16;
  o->true_residual = 1;
}

lshom_status lshom_check_problem(int d, const int64_t* N, int n_phases, const double* cond,
                                 double l0, const double* E, double tol) {
  if (d != 2 && d != 3) return LSHOM_ERR_INVALID_ARG;
  if (!N) return LSHOM_ERR_INVALID_ARG;
  for (int a = 0; a < d; ++a) {
    if (N[a] < 3) return LSHOM_ERR_INVALID_ARG;
    if (N[a] > 4096 || !fft_size_ok(N[a])) return LSHOM_ERR_UNSUPPORTED;
  }
  if (n_phases < 1 || n_phases > kMaxPhases || !cond) return LSHOM_ERR_INVALID_ARG;
  for (int i = 0; i < n_phases; ++i)
    if (!std::isfinite(cond[i]) || !(cond[i] > 0.0)) return LSHOM_ERR_INVALID_ARG;
  if (!std::isfinite(l0) || l0 < 0.0) return LSHOM_ERR_INVALID_ARG;
  if (E)
    for (int a = 0; a < d; ++a)
      if (!std::isfinite(E[a])) return LSHOM_ERR_INVALID_ARG;
  if (tol >= 0.0 && !std::isfinite(tol)) return LSHOM_ERR_INVALID_ARG;
  if (std::isnan(tol)) return LSHOM_ERR_INVALID_ARG;
  return LSHOM_OK;
}

lshom_status lshom_create(lshom_ctx** out, int device, void* hip_stream) {
  if (!out) return LSHOM_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return LSHOM_ERR_HIP;
  if (device < 0 || device >= count) return LSHOM_ERR_INVALID_ARG;
  DeviceGuard g(device);
  lshom_ctx* c = new lshom_ctx();
  c->device = device;
  c->user_stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->host_state), sizeof(DevState), hipHostMallocDefault) !=
          hipSuccess) {
    if (c->stream) (void)hipStreamDestroy(c->stream);
    if (c->ev) (void)hipEventDestroy(c->ev);
    delete c;
    return LSHOM_ERR_HIP;
  }
  std::memset(c->host_state, 0, sizeof(DevState));
  *out = c;
  return LSHOM_OK;
}

void lshom_destroy(lshom_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  if (c->host_state) (void)hipHostFree(c->host_state);
  if (c->ev) (void)hipEventDestroy(c->ev);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

lshom_status lshom_set_microstructure(lshom_ctx* c, int d, const int64_t* N,
                                      const uint8_t* phase_dev, int n_phases,
                                      const double* cond_host) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  lshom_status s = lshom_check_problem(d, N, n_phases, cond_host, 0.0, nullptr, -1.0);
  if (s != LSHOM_OK) return fail(c, s, "invalid microstructure (d, N, n_phases or cond)");
  if (!phase_dev) return fail(c, LSHOM_ERR_INVALID_ARG, "phase_dev is NULL");
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  c->ws_ready = false;
  c->d = d;
  c->nvox = 1;
  for (int a = 0; a < 3; ++a) c->N[a] = a < d ? N[a] : 1;
  for (int a = 0; a < d; ++a) c->nvox *= N[a];
  c->h = (int)(N[d - 1] / 2 + 1);
  c->nrows = c->nvox / N[d - 1];
  c->nhalf = c->nrows * c->h;
  c->phase = phase_dev;
  c->cond.assign(cond_host, cond_host + n_phases);
  double lo = cond_host[0], hi = cond_host[0];
  for (int i = 1; i < n_phases; ++i) {
    lo = std::min(lo, cond_host[i]);
    hi = std::max(hi, cond_host[i]);
  }
  c->l0 = 0.5 * (lo + hi);
  for (int a = 0; a < d; ++a) c->plan[a] = default_plan((int)N[a]);
  c->shape64 = default_shape(d, c->N, c->plan, (int)sizeof(cx<double>), kLdsBudget, kMinBlocks);
  c->shape32 = default_shape(d, c->N, c->plan, (int)sizeof(cx<float>), kLdsBudget, kMinBlocks);
  if (!shape_fits(d, c->N, c->plan, c->shape64, (int)sizeof(cx<double>), kLdsBudget) ||
      !shape_fits(d, c->N, c->plan, c->shape32, (int)sizeof(cx<float>), kLdsBudget)) {
    c->have_problem = false;
    return fail(c, LSHOM_ERR_UNSUPPORTED, "grid too long for one LDS-resident FFT batch");
  }
  c->have_problem = true;
  c->err.clear();
  return LSHOM_OK;
}

lshom_status lshom_set_reference(lshom_ctx* c, double l0) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return fail(c, LSHOM_ERR_STATE, "set_microstructure has not been called");
  if (!std::isfinite(l0) || !(l0 > 0.0)) return fail(c, LSHOM_ERR_INVALID_ARG, "l0 must be finite and > 0");
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);  // l0 is baked into captured launches
  c->l0 = l0;
  return LSHOM_OK;
}

lshom_status lshom_workspace_size(const lshom_ctx* c, int precision, size_t* bytes) {
  if (!c || !bytes) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return LSHOM_ERR_STATE;
  if (precision != LSHOM_PRECISION_FP64 && precision != LSHOM_PRECISION_MIXED)
    return LSHOM_ERR_INVALID_ARG;
  *bytes = compute_layout(c, precision == LSHOM_PRECISION_MIXED).total;
  return LSHOM_OK;
}

lshom_status lshom_set_workspace(lshom_ctx* c, void* dev, size_t bytes) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return fail(c, LSHOM_ERR_STATE, "set_microstructure has not been called");
  if (!dev || (reinterpret_cast<uintptr_t>(dev) % kAlign) != 0)
    return fail(c, LSHOM_ERR_WORKSPACE, "workspace must be non-NULL and 256-byte aligned");
  Layout l64 = compute_layout(c, false);
  Layout lmx = compute_layout(c, true);
  Layout use;
  if (bytes >= lmx.total) use = lmx;
  else if (bytes >= l64.total) use = l64;
  else return fail(c, LSHOM_ERR_WORKSPACE, "workspace smaller than lshom_workspace_size()");
  DeviceGuard g(c->device);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  drop_graphs(c);
  c->ws = static_cast<char*>(dev);
  c->ws_bytes = bytes;
  c->lay = use;
  // per-phase conductivity (unused slots NaN so that an out-of-range phase
  // poisons the solve instead of reading a stale value) and twiddles
  std::vector<double> c64(kMaxPhases, std::nan(""));
  std::vector<float> c32(kMaxPhases, std::nanf(""));
  for (size_t i = 0; i < c->cond.size(); ++i) {
    c64[i] = c->cond[i];
    c32[i] = (float)c->cond[i];
  }
  HIP_TRY(c, hipMemcpy(c->ws + use.off_cond64, c64.data(), kMaxPhases * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->ws + use.off_cond32, c32.data(), kMaxPhases * sizeof(float), hipMemcpyHostToDevice));
  for (int a = 0; a < c->d; ++a) {
    std::vector<double> tw;
    twiddles((int)c->N[a], &tw);
    std::vector<float> tw32(tw.size());
    for (size_t i = 0; i < tw.size(); ++i) tw32[i] = (float)tw[i];
    HIP_TRY(c, hipMemcpy(c->ws + use.off_tw64[a], tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->ws + use.off_tw32[a], tw32.data(), tw32.size() * sizeof(float), hipMemcpyHostToDevice));
  }
  DevState zero{};
  HIP_TRY(c, hipMemcpy(c->ws + use.off_state, &zero, sizeof(DevState), hipMemcpyHostToDevice));
  c->ws_ready = true;
  c->err.clear();
  return LSHOM_OK;
}

lshom_status lshom_solve(lshom_ctx* c, const double* E_host, double tol, const lshom_solve_opts* opts,
                         const double* x0_dev, double* e_dev, double* leff_host,
                         lshom_solve_info* info) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  lshom_solve_opts o;
  lshom_default_opts(&o);
  if (opts) o = *opts;
  lshom_status s = validate_opts(c, &o);
  if (s != LSHOM_OK) return s;
  if ((s = check_ready(c, o.precision)) != LSHOM_OK) return s;
  if (!E_host) return fail(c, LSHOM_ERR_INVALID_ARG, "E_host is NULL");
  if (!std::isfinite(tol) || tol < 0.0) return fail(c, LSHOM_ERR_INVALID_ARG, "tol must be finite and >= 0");
  for (int a = 0; a < c->d; ++a)
    if (!std::isfinite(E_host[a])) return fail(c, LSHOM_ERR_INVALID_ARG, "E must be finite");
  DeviceGuard g(c->device);
  HIP_TRY(c, order_after_user(c));
  double e2 = 0.0;
  for (int a = 0; a < c->d; ++a) e2 += E_host[a] * E_host[a];
  if (e2 == 0.0) {
    // b = 0: the solution is e = 0 (Sec. 2.2, Eq. (15) is linear)
    if (e_dev) HIP_TRY(c, hipMemsetAsync(e_dev, 0, sizeof(double) * c->d * c->nvox, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (leff_host)
      for (int a = 0; a < c->d; ++a) leff_host[a] = 0.0;
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->rel_res_true = 0.0;
    }
    return LSHOM_OK;
  }
  if (o.precision == LSHOM_PRECISION_FP64)
    s = solve_fp64(c, E_host, tol, o, x0_dev, e_dev, leff_host, info);
  else
    s = solve_mixed(c, E_host, tol, o, x0_dev, e_dev, leff_host, info);
  if (s == LSHOM_OK) c->err.clear();
  else if (s == LSHOM_ERR_NOT_CONVERGED) c->err = "not converged within max_iter";
  else if (s == LSHOM_ERR_BREAKDOWN) c->err = "CG breakdown";
  return s;
}

lshom_status lshom_homogenize(lshom_ctx* c, double tol, const lshom_solve_opts* opts,
                              double* leff_host, lshom_solve_info* infos) {
  if (!c || !leff_host) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return fail(c, LSHOM_ERR_STATE, "set_microstructure has not been called");
  const int d = c->d;
  lshom_status worst = LSHOM_OK;
  for (int b = 0; b < d; ++b) {
    double E[3] = {0.0, 0.0, 0.0};
    E[b] = 1.0;
    double col[3] = {0.0, 0.0, 0.0};
    lshom_status s = lshom_solve(c, E, tol, opts, nullptr, nullptr, col, infos ? &infos[b] : nullptr);
    if (s != LSHOM_OK && s != LSHOM_ERR_NOT_CONVERGED && s != LSHOM_ERR_BREAKDOWN) return s;
    if (s != LSHOM_OK) worst = s;
    for (int a = 0; a < d; ++a) leff_host[a * d + b] = col[a];
  }
  return worst;
}

lshom_status lshom_apply(lshom_ctx* c, const double* p_dev, double* q_dev) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  lshom_status s = check_ready(c, LSHOM_PRECISION_FP64);
  if (s != LSHOM_OK) return s;
  if (!p_dev || !q_dev || p_dev == q_dev) return fail(c, LSHOM_ERR_INVALID_ARG, "p_dev/q_dev NULL or aliased");
  DeviceGuard g(c->device);
  HIP_TRY(c, order_after_user(c));
  Bufs<double> b = get_bufs<double>(c);
  cx<double>* q = b.v[3];
  HIP_TRY(c, enq_project_real(c, b, p_dev, true, q));
  HIP_TRY(c, enq_field_out(c, b, q, nullptr, p_dev, q_dev, false));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->err.clear();
  return LSHOM_OK;
}

lshom_status lshom_time_passes(lshom_ctx* c, int precision, int reps, double* ms_out,
                               double* bytes_out) {
  if (!c || !ms_out || reps < 1) return LSHOM_ERR_INVALID_ARG;
  if (precision != LSHOM_PRECISION_FP64 && precision != LSHOM_PRECISION_MIXED)
    return fail(c, LSHOM_ERR_INVALID_ARG, "precision must be FP64 (0) or MIXED (1)");
  lshom_status s = check_ready(c, precision);
  if (s != LSHOM_OK) return s;
  DeviceGuard g(c->device);
  HIP_TRY(c, order_after_user(c));
  if (precision == LSHOM_PRECISION_FP64) return time_passes<double>(c, get_bufs<double>(c), reps, ms_out, bytes_out);
  return time_passes<float>(c, get_bufs<float>(c), reps, ms_out, bytes_out);
}

}  // extern "C"
