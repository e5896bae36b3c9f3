// C ABI of the lshom library: validation, context and workspace management.
// The solve drivers live in driver.cpp.  See include/lshom.h.
#include "lshom.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "ctx.hpp"

using namespace lshom;

namespace {

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

lshom_status check_ready(lshom_ctx* c, int precision) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return fail(c, LSHOM_ERR_STATE, "set_microstructure has not been called");
  if (!c->ws_ready) return fail(c, LSHOM_ERR_WORKSPACE, "no workspace attached for this problem");
  if (precision == LSHOM_PRECISION_MIXED && !c->lay.has32)
    return fail(c, LSHOM_ERR_WORKSPACE, "workspace was sized for FP64 only");
  return LSHOM_OK;
}

hipError_t order_after_user(lshom_ctx* c) {
  hipError_t e = hipEventRecord(c->ev, c->user_stream);
  if (e != hipSuccess) return e;
  return hipStreamWaitEvent(c->stream, c->ev, 0);
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

}  // namespace

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
  if (std::isnan(tol) || (tol >= 0.0 && !std::isfinite(tol))) return LSHOM_ERR_INVALID_ARG;
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
  c->have_problem = false;
  c->d = d;
  c->nvox = 1;
  for (int a = 0; a < 3; ++a) c->N[a] = a < d ? N[a] : 1;
  for (int a = 0; a < d; ++a) c->nvox *= N[a];
  c->h = (int)(N[d - 1] / 2 + 1);
  c->nrows = c->nvox / N[d - 1];
  c->nhalf = c->nrows * c->h;
  c->transposed = (d == 2);
  c->phase = phase_dev;
  c->cond.assign(cond_host, cond_host + n_phases);
  double lo = cond_host[0], hi = cond_host[0];
  for (int i = 1; i < n_phases; ++i) {
    lo = std::min(lo, cond_host[i]);
    hi = std::max(hi, cond_host[i]);
  }
  c->l0 = 0.5 * (lo + hi);
  for (int a = 0; a < d; ++a) c->plan[a] = default_plan((int)N[a]);
  c->shape64 = default_shape(d, c->N, c->plan, (int)sizeof(cx<double>), kLdsBudget, kMinBlocks,
                             c->transposed, n_phases);
  c->shape32 = default_shape(d, c->N, c->plan, (int)sizeof(cx<float>), kLdsBudget, kMinBlocks,
                             c->transposed, n_phases);
  if (!shape_fits(d, c->N, c->plan, c->shape64, (int)sizeof(cx<double>), kLdsBudget, n_phases) ||
      !shape_fits(d, c->N, c->plan, c->shape32, (int)sizeof(cx<float>), kLdsBudget, n_phases))
    return fail(c, LSHOM_ERR_UNSUPPORTED, "grid too long for one LDS-resident FFT batch");
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
  c->ws_ready = false;
  c->ws = static_cast<char*>(dev);
  c->ws_bytes = bytes;
  c->lay = use;
  lshom_status s = prepare_workspace(c);
  if (s != LSHOM_OK) return s;
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
  s = apply_real(c, p_dev, q_dev);
  if (s == LSHOM_OK) c->err.clear();
  return s;
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
  s = time_passes(c, precision, reps, ms_out, bytes_out);
  if (s == LSHOM_OK) c->err.clear();
  return s;
}

}  // extern "C"
