// C ABI of the lshom library: validation, context and workspace management.
// The solve drivers live in driver.cpp.  See include/lshom.h.
#include "lshom.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

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
  if (precision == LSHOM_PRECISION_MIXED && !c->g.lay.has32)
    return fail(c, LSHOM_ERR_WORKSPACE, "workspace was sized for FP64 only");
  return LSHOM_OK;
}

// x . M . y for the upper triangle M of a symmetric d x d matrix (row by row).
double sym_form(const double* m, int d, const double* x, const double* y) {
  double full[9];
  int k = 0;
  for (int i = 0; i < d; ++i)
    for (int j = i; j < d; ++j) full[i * d + j] = full[j * d + i] = m[k++];
  double s = 0.0;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) s += x[i] * full[i * d + j] * y[j];
  return s;
}

// Initial device scalars of one problem.  With an anisotropic reference
// (L0n = L0 / l0, upper triangle; not for BiCG, which iterates on the nodal
// fields in the Euclidean product) the norms are those of the scaled
// spectral coordinate: ||b||^2 = |N| E . L0n . E.
DevState initial_state(int d, long long nvox, const double* E, double tol, double l0, const lshom_solve_opts& o,
                       bool with_history, const double* L0n = nullptr) {
  DevState s{};
  double e2 = 0.0;
  for (int t = 0; t < d; ++t) e2 += E[t] * E[t];
  const bool aniso = L0n && o.method != LSHOM_METHOD_BICG;
  if (aniso) e2 = sym_form(L0n, d, E, E);
  s.b2 = e2 * (double)nvox;
  for (int t = 0; t < 3; ++t) s.E[t] = t < d ? E[t] : 0.0;
  for (int t = 0; t < 3; ++t) {
    double v = 0.0;
    if (t < d && L0n) {
      double et[3] = {0.0, 0.0, 0.0};
      et[t] = 1.0;
      v = l0 * sym_form(L0n, d, et, E);
    } else if (t < d) {
      v = l0 * E[t];
    }
    s.l0E[t] = v;
  }
  s.tol2b2 = tol * tol * s.b2;
  s.tol2 = tol * tol;
  s.l0 = l0;
  s.nvox = (double)nvox;
  s.norm = o.norm;
  s.eta_e_log = -1.0;
  s.eta_e_true = -1.0;
  if (with_history) {
    s.hist = o.history_dev;
    s.hist_len = o.history_len;
  }
  s.max_iter = o.max_iter;
  if (o.precision == LSHOM_PRECISION_MIXED) {
    s.refresh_every = o.refresh_every;
    s.drop2 = o.refresh_drop * o.refresh_drop;
  }
  return s;
}

void fill_info(const DevState& hs, double l0, const lshom_solve_opts& o, int warm_used, lshom_solve_info* info) {
  if (!info) return;
  const bool mixed = o.precision == LSHOM_PRECISION_MIXED;
  info->iterations = hs.iter_a;
  info->applies_fp32 = mixed ? hs.iter_a : 0;
  info->applies_fp64 = mixed ? hs.n_refresh : hs.iter_a;
  info->status = hs.status;
  info->warm_start_used = warm_used;
  info->refreshes = mixed ? hs.n_refresh : 0;
  const double rr = mixed ? hs.rr_true : hs.rr_log;
  const double b2 = hs.b2 > 0.0 ? hs.b2 : 1.0;
  info->rel_res = std::sqrt(rr / b2);
  info->rel_res_true = o.true_residual ? std::sqrt(hs.rr_true / b2) : -1.0;
  info->eta_r = l0 * std::sqrt(rr / b2);
  info->eta_e = o.true_residual ? hs.eta_e_true : -1.0;
  if (o.method == LSHOM_METHOD_BICG) {
    info->applies_fp64 = 2 * hs.iter_a;
    info->eta_e = -1.0;
  }
}

hipError_t order_after_user(lshom_ctx* c) {
  std::lock_guard<std::mutex> lock(setup_mutex());
  hipError_t e = hipEventRecord(c->ev, c->user_stream);
  if (e != hipSuccess) return e;
  return hipStreamWaitEvent(c->stream, c->ev, 0);
}

// Eigenvalues of a symmetric d x d matrix (d <= 3) by cyclic Jacobi
// rotations; a[] is row-major and is overwritten.
void sym_eigenvalues(double* a, int d, double* w) {
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < d; ++p)
      for (int q = p + 1; q < d; ++q) off += a[p * d + q] * a[p * d + q];
    if (off < 1e-30) break;
    for (int p = 0; p < d; ++p)
      for (int q = p + 1; q < d; ++q) {
        const double apq = a[p * d + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = 0.5 * (a[q * d + q] - a[p * d + p]) / apq;
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < d; ++k) {  // columns p, q
          const double akp = a[k * d + p], akq = a[k * d + q];
          a[k * d + p] = cs * akp - sn * akq;
          a[k * d + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < d; ++k) {  // rows p, q
          const double apk = a[p * d + k], aqk = a[q * d + k];
          a[p * d + k] = cs * apk - sn * aqk;
          a[q * d + k] = sn * apk + cs * aqk;
        }
      }
  }
  for (int i = 0; i < d; ++i) w[i] = a[i * d + i];
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
  if (o->method != LSHOM_METHOD_CG && o->method != LSHOM_METHOD_FFTH && o->method != LSHOM_METHOD_BICG &&
      o->method != LSHOM_METHOD_PIPECG)
    return fail(c, LSHOM_ERR_INVALID_ARG, "method must be CG (0), FFTH (1), BICG (2) or PIPECG (3)");
  if (o->norm != LSHOM_NORM_RESIDUAL && o->norm != LSHOM_NORM_EQUILIBRIUM)
    return fail(c, LSHOM_ERR_INVALID_ARG, "norm must be RESIDUAL (0) or EQUILIBRIUM (1)");
  if (o->history_len < 0) return fail(c, LSHOM_ERR_INVALID_ARG, "history_len must be >= 0");
  const bool mixed = o->precision == LSHOM_PRECISION_MIXED;
  if (mixed && o->method != LSHOM_METHOD_CG)
    return fail(c, LSHOM_ERR_UNSUPPORTED, "the basic scheme, BiCG and pipelined CG run in FP64 only");
  if ((o->method == LSHOM_METHOD_BICG || o->method == LSHOM_METHOD_PIPECG) &&
      (o->norm != LSHOM_NORM_RESIDUAL || o->history_dev))
    return fail(c, LSHOM_ERR_UNSUPPORTED, "BiCG and pipelined CG stop on the residual norm and keep no history");
  if (mixed && (o->norm == LSHOM_NORM_EQUILIBRIUM || o->history_dev))
    return fail(c, LSHOM_ERR_UNSUPPORTED, "the equilibrium norm and the history are FP64 only");
  return LSHOM_OK;
}

// The equilibrium norm is formed from the residual (no transform of the
// current), which needs grids without Nyquist modes.
lshom_status check_equilibrium_grid(lshom_ctx* c, const lshom_solve_opts& o, const int64_t* N, int d) {
  if (o.norm != LSHOM_NORM_EQUILIBRIUM && !o.history_dev) return LSHOM_OK;
  for (int a = 0; a < d; ++a)
    if ((N[a] & 1) == 0)
      return fail(c, LSHOM_ERR_UNSUPPORTED, "the equilibrium norm and the history need odd N");
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
  o->refresh_drop = 0.01;
  o->graph_block = 16;
  o->true_residual = 1;
  o->method = LSHOM_METHOD_CG;
  o->norm = LSHOM_NORM_RESIDUAL;
  o->history_dev = nullptr;
  o->history_len = 0;
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
  {
    // the same limits the device set-up applies: index range, and the LDS
    // footprint of the default pass shapes of both precisions
    long long nvox = 1;
    FftPlan plans[3];
    for (int a = 0; a < d; ++a) {
      nvox *= N[a];
      plans[a] = default_plan((int)N[a]);
    }
    if (nvox >= (1ll << 31)) return LSHOM_ERR_UNSUPPORTED;
    for (int es : {(int)sizeof(cx<double>), (int)sizeof(cx<float>)}) {
      bool fits = false;
      (void)default_shape_within(d, N, plans, es, kLdsLimit, d == 2, n_phases, true, &fits);
      if (!fits) return LSHOM_ERR_UNSUPPORTED;
    }
  }
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
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess ||
      lds <= (int)kLdsStaticReserve) {
    delete c;
    return LSHOM_ERR_HIP;
  }
  c->lds_limit = std::min(kLdsLimit, (size_t)lds - kLdsStaticReserve);
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev, hipEventDisableTiming) != hipSuccess) {
    if (c->stream) (void)hipStreamDestroy(c->stream);
    if (c->ev) (void)hipEventDestroy(c->ev);
    delete c;
    return LSHOM_ERR_HIP;
  }
  *out = c;
  return LSHOM_OK;
}

void lshom_destroy(lshom_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c->graphs);
  drop_batch_graphs(c);
  for (hipEvent_t ev : c->timer.pool) (void)hipEventDestroy(ev);
  if (c->ev) (void)hipEventDestroy(c->ev);
  for (hipStream_t st : c->group_streams) (void)hipStreamDestroy(st);
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
  drop_graphs(c->graphs);
  drop_batch_graphs(c);
  c->ws_ready = false;
  c->have_problem = false;
  c->g = Group{};
  c->g.ctx = c;
  c->g.graph_cache = &c->graphs;
  if (group_setup(c->g, d, N, n_phases) != LSHOM_OK)
    return fail(c, LSHOM_ERR_UNSUPPORTED, "grid too long for one LDS-resident FFT batch");
  c->g.phase = phase_dev;
  c->cond.assign(cond_host, cond_host + n_phases);
  double lo = cond_host[0], hi = cond_host[0];
  for (int i = 1; i < n_phases; ++i) {
    lo = std::min(lo, cond_host[i]);
    hi = std::max(hi, cond_host[i]);
  }
  c->g.l0 = 0.5 * (lo + hi);
  c->have_problem = true;
  c->err.clear();
  return LSHOM_OK;
}


lshom_status lshom_set_microstructure_tensor(lshom_ctx* c, int d, const int64_t* N, const uint8_t* phase_dev,
                                             int n_phases, const double* cond_tensor_host) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  if (d != 2 && d != 3) return fail(c, LSHOM_ERR_INVALID_ARG, "d must be 2 or 3");
  const int ncomp = d * (d + 1) / 2;
  if (n_phases < 1 || n_phases * ncomp > kMaxPhases || !cond_tensor_host)
    return fail(c, LSHOM_ERR_INVALID_ARG, "n_phases out of range (at most 256 / (d (d + 1) / 2)) or cond NULL");
  // the scalar check covers d and N (a unit table stands in for the tensors)
  std::vector<double> ones(n_phases, 1.0);
  lshom_status s = lshom_check_problem(d, N, n_phases, ones.data(), 0.0, nullptr, -1.0);
  if (s != LSHOM_OK) return fail(c, s, "invalid microstructure (d, N or n_phases)");
  if (!phase_dev) return fail(c, LSHOM_ERR_INVALID_ARG, "phase_dev is NULL");
  std::vector<double> table;
  double lo = 1e300, hi = -1e300;
  for (int q = 0; q < n_phases; ++q) {
    const double* m = cond_tensor_host + (size_t)q * d * d;
    double scale = 0.0;
    for (int i = 0; i < d * d; ++i) {
      if (!std::isfinite(m[i])) return fail(c, LSHOM_ERR_INVALID_ARG, "tensor entries must be finite");
      scale = std::max(scale, std::fabs(m[i]));
    }
    for (int i = 0; i < d; ++i)
      for (int j = i + 1; j < d; ++j)
        if (std::fabs(m[i * d + j] - m[j * d + i]) > 1e-12 * scale)
          return fail(c, LSHOM_ERR_INVALID_ARG, "phase tensors must be symmetric");
    double a[9], w[3];
    for (int i = 0; i < d * d; ++i) a[i] = m[i];
    sym_eigenvalues(a, d, w);
    for (int i = 0; i < d; ++i) {
      if (!(w[i] > 0.0)) return fail(c, LSHOM_ERR_INVALID_ARG, "phase tensors must be positive definite");
      lo = std::min(lo, w[i]);
      hi = std::max(hi, w[i]);
    }
    for (int i = 0; i < d; ++i)
      for (int j = i; j < d; ++j) table.push_back(0.5 * (m[i * d + j] + m[j * d + i]));
  }
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c->graphs);
  drop_batch_graphs(c);
  c->ws_ready = false;
  c->have_problem = false;
  c->g = Group{};
  c->g.ctx = c;
  c->g.graph_cache = &c->graphs;
  if (group_setup(c->g, d, N, n_phases, true) != LSHOM_OK)
    return fail(c, LSHOM_ERR_UNSUPPORTED, "grid too long for one LDS-resident FFT batch");
  c->g.phase = phase_dev;
  c->cond = table;
  // Sec. 2.3, Eq. (19): the extreme eigenvalues of L over the cell
  c->g.l0 = 0.5 * (lo + hi);
  c->have_problem = true;
  c->err.clear();
  return LSHOM_OK;
}

lshom_status lshom_set_cell(lshom_ctx* c, const double* lengths) {
  if (!c || !lengths) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return fail(c, LSHOM_ERR_STATE, "set_microstructure has not been called");
  for (int a = 0; a < c->g.d; ++a)
    if (!std::isfinite(lengths[a]) || !(lengths[a] > 0.0))
      return fail(c, LSHOM_ERR_INVALID_ARG, "cell lengths must be finite and > 0");
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c->graphs);
  drop_batch_graphs(c);  // the wave vectors are baked into captured launches
  for (int a = 0; a < 3; ++a) c->g.cell_inv[a] = a < c->g.d ? 1.0 / lengths[a] : 1.0;
  return LSHOM_OK;
}

lshom_status lshom_set_reference(lshom_ctx* c, double l0) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return fail(c, LSHOM_ERR_STATE, "set_microstructure has not been called");
  if (!std::isfinite(l0) || !(l0 > 0.0)) return fail(c, LSHOM_ERR_INVALID_ARG, "l0 must be finite and > 0");
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c->graphs);
  drop_batch_graphs(c);  // l0 is baked into captured launches
  c->g.l0 = l0;
  c->g.aniso = false;
  return LSHOM_OK;
}

lshom_status lshom_set_reference_mean(lshom_ctx* c) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return fail(c, LSHOM_ERR_STATE, "set_microstructure has not been called");
  if (!c->ws_ready) return fail(c, LSHOM_ERR_WORKSPACE, "attach a workspace first (it holds the phase counts)");
  Group& gr = c->g;
  DeviceGuard g(c->device);
  HIP_TRY(c, order_after_user(c));
  // the partial-sum area is free between solves
  unsigned* counts = reinterpret_cast<unsigned*>(gr.ws + gr.lay.off_partials);
  std::vector<unsigned> h(256, 0u);
  HIP_TRY(c, hipMemsetAsync(counts, 0, 256 * sizeof(unsigned), c->stream));
  HIP_TRY(c, launch_phase_histogram(gr.phase, gr.nvox, counts, c->stream));
  HIP_TRY(c, hipMemcpyAsync(h.data(), counts, 256 * sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int d = gr.d;
  const int ncomp = gr.tensor ? d * (d + 1) / 2 : 1;
  double M[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int q = 0; q < gr.n_phase_ids; ++q) {
    const double f = (double)h[q] / (double)gr.nvox;
    if (f == 0.0) continue;
    if (!gr.tensor) {
      for (int i = 0; i < d; ++i) M[i * d + i] += f * c->cond[q];
      continue;
    }
    int k = 0;
    for (int i = 0; i < d; ++i)
      for (int j = i; j < d; ++j, ++k) {
        const double v = f * c->cond[(size_t)q * ncomp + k];
        M[i * d + j] += v;
        if (j != i) M[j * d + i] += v;
      }
  }
  if (!gr.tensor) return lshom_set_reference(c, M[0]);
  return lshom_set_reference_tensor(c, M);
}

lshom_status lshom_set_reference_tensor(lshom_ctx* c, const double* L0) {
  if (!c || !L0) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return fail(c, LSHOM_ERR_STATE, "set_microstructure has not been called");
  Group& gr = c->g;
  const int d = gr.d;
  double scale = 0.0;
  for (int i = 0; i < d * d; ++i) {
    if (!std::isfinite(L0[i])) return fail(c, LSHOM_ERR_INVALID_ARG, "L0 entries must be finite");
    scale = std::max(scale, std::fabs(L0[i]));
  }
  for (int i = 0; i < d; ++i)
    for (int j = i + 1; j < d; ++j)
      if (std::fabs(L0[i * d + j] - L0[j * d + i]) > 1e-12 * scale)
        return fail(c, LSHOM_ERR_INVALID_ARG, "L0 must be symmetric");
  double a[9], w[3];
  for (int i = 0; i < d * d; ++i) a[i] = L0[i];
  sym_eigenvalues(a, d, w);
  for (int i = 0; i < d; ++i)
    if (!(w[i] > 0.0)) return fail(c, LSHOM_ERR_INVALID_ARG, "L0 must be positive definite");
  bool iso = true;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j)
      if (L0[i * d + j] != (i == j ? L0[0] : 0.0)) iso = false;
  if (iso) return lshom_set_reference(c, L0[0]);
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c->graphs);
  drop_batch_graphs(c);
  if (!gr.tensor) {
    // dL = L - L0 couples the components of a node: scalar phases become
    // the tensors lambda I (the row pass then keeps every component of a
    // node in one block)
    const int nph = gr.n_phase_ids;
    if (nph * d * (d + 1) / 2 > kMaxPhases)
      return fail(c, LSHOM_ERR_UNSUPPORTED, "too many phases for tensor tables (at most 256 / (d (d + 1) / 2))");
    std::vector<double> table;
    for (int q = 0; q < nph; ++q)
      for (int i = 0; i < d; ++i)
        for (int j = i; j < d; ++j) table.push_back(i == j ? c->cond[q] : 0.0);
    int64_t N[3] = {gr.N[0], gr.N[1], gr.N[2]};
    if (group_setup(gr, d, N, nph, true) != LSHOM_OK)
      return fail(c, LSHOM_ERR_UNSUPPORTED, "grid too long for one LDS-resident FFT batch with tensor phases");
    c->cond = table;
    if (c->ws_ready) {
      c->ws_ready = false;
      lshom_status s = prepare_workspace(gr, c->cond, nullptr, {gr.phase});
      if (s != LSHOM_OK) return s;
      c->ws_ready = true;
    }
  }
  double tr = 0.0;
  for (int i = 0; i < d; ++i) tr += L0[i * d + i];
  gr.l0 = tr / d;
  int k = 0;
  for (int i = 0; i < d; ++i)
    for (int j = i; j < d; ++j, ++k) {
      gr.L0u[k] = 0.5 * (L0[i * d + j] + L0[j * d + i]);
      gr.L0n[k] = gr.L0u[k] / gr.l0;
    }
  for (; k < 6; ++k) gr.L0u[k] = gr.L0n[k] = 0.0;
  gr.aniso = true;
  c->err.clear();
  return LSHOM_OK;
}

lshom_status lshom_workspace_size(const lshom_ctx* c, int precision, size_t* bytes) {
  if (!c || !bytes) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return LSHOM_ERR_STATE;
  if (precision != LSHOM_PRECISION_FP64 && precision != LSHOM_PRECISION_MIXED)
    return LSHOM_ERR_INVALID_ARG;
  *bytes = compute_layout(c->g, precision == LSHOM_PRECISION_MIXED).total;
  return LSHOM_OK;
}

lshom_status lshom_workspace_size_for(const lshom_ctx* c, const lshom_solve_opts* opts, size_t* bytes) {
  if (!c || !bytes) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return LSHOM_ERR_STATE;
  lshom_solve_opts o;
  lshom_default_opts(&o);
  if (opts) o = *opts;
  if (o.precision != LSHOM_PRECISION_FP64 && o.precision != LSHOM_PRECISION_MIXED) return LSHOM_ERR_INVALID_ARG;
  const bool extra = o.method == LSHOM_METHOD_BICG || o.method == LSHOM_METHOD_PIPECG;
  *bytes = compute_layout(c->g, o.precision == LSHOM_PRECISION_MIXED, extra).total;
  return LSHOM_OK;
}

lshom_status lshom_set_workspace(lshom_ctx* c, void* dev, size_t bytes) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return fail(c, LSHOM_ERR_STATE, "set_microstructure has not been called");
  if (!dev || (reinterpret_cast<uintptr_t>(dev) % kAlign) != 0)
    return fail(c, LSHOM_ERR_WORKSPACE, "workspace must be non-NULL and 256-byte aligned");
  // the largest layout that fits: [FP32 part] [BiCG fields]
  Layout use;
  bool found = false;
  for (int k = 3; k >= 0 && !found; --k) {
    const Layout l = compute_layout(c->g, (k & 1) != 0, (k & 2) != 0);
    if (bytes >= l.total) {
      use = l;
      found = true;
    }
  }
  if (!found) return fail(c, LSHOM_ERR_WORKSPACE, "workspace smaller than lshom_workspace_size()");
  DeviceGuard g(c->device);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  drop_graphs(c->graphs);
  drop_batch_graphs(c);
  c->ws_ready = false;
  c->g.ws = static_cast<char*>(dev);
  c->ws_bytes = bytes;
  c->g.lay = use;
  lshom_status s = prepare_workspace(c->g, c->cond, nullptr, {c->g.phase});
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
  for (int a = 0; a < c->g.d; ++a)
    if (!std::isfinite(E_host[a])) return fail(c, LSHOM_ERR_INVALID_ARG, "E must be finite");
  if ((s = check_equilibrium_grid(c, o, c->g.N, c->g.d)) != LSHOM_OK) return s;
  if (o.method != LSHOM_METHOD_CG && x0_dev)
    return fail(c, LSHOM_ERR_UNSUPPORTED, "the basic scheme, BiCG and pipelined CG start from e = E (no x0)");
  if (o.method == LSHOM_METHOD_PIPECG && !c->g.lay.has_bicg)
    return fail(c, LSHOM_ERR_WORKSPACE, "workspace has no extra fields (size it with lshom_workspace_size_for)");
  if (o.method == LSHOM_METHOD_BICG) {
    if (!c->g.lay.has_bicg)
      return fail(c, LSHOM_ERR_WORKSPACE, "workspace has no BiCG fields (size it with lshom_workspace_size_for)");
    if ((long long)c->g.d * c->g.nvox >= (1ll << 31))
      return fail(c, LSHOM_ERR_UNSUPPORTED, "BiCG fields above 2^31 values");
  }
  DeviceGuard g(c->device);
  HIP_TRY(c, order_after_user(c));
  Group& gr = c->g;
  double e2 = 0.0;
  for (int a = 0; a < gr.d; ++a) e2 += E_host[a] * E_host[a];
  if (e2 == 0.0) {
    // b = 0: the solution is e = 0 (Sec. 2.2, Eq. (15) is linear)
    if (e_dev) HIP_TRY(c, hipMemsetAsync(e_dev, 0, sizeof(double) * gr.d * gr.nvox, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (leff_host)
      for (int a = 0; a < gr.d; ++a) leff_host[a] = 0.0;
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->rel_res_true = 0.0;
    }
    return LSHOM_OK;
  }
  std::vector<DevState> init(
      1, initial_state(gr.d, gr.nvox, E_host, tol, gr.l0, o, true, gr.aniso ? gr.L0n : nullptr));
  if (o.method == LSHOM_METHOD_BICG)
    s = solve_bicg(gr, init[0], o, e_dev);
  else if (o.method == LSHOM_METHOD_PIPECG)
    s = solve_pipecg(gr, init[0], o, e_dev);
  else
    s = solve_group(gr, init, o, E_host, x0_dev, e_dev);
  if (s != LSHOM_OK) return s;
  const DevState& hs = gr.host_states[0];
  if (leff_host)
    for (int a = 0; a < gr.d; ++a) leff_host[a] = hs.leff[a];
  fill_info(hs, gr.l0, o, gr.warm_used, info);
  s = hs.status;
  if (s == LSHOM_OK) c->err.clear();
  else if (s == LSHOM_ERR_NOT_CONVERGED) c->err = "not converged within max_iter";
  else if (s == LSHOM_ERR_BREAKDOWN) c->err = "CG breakdown";
  return s;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free solve: the workspace is a file-scope device array
// ---------------------------------------------------------------------------

namespace {

// In host code this name is a stand-in, not a device address: kernels and
// copies get the per-device address from hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[LSHOM_STATIC_WORKSPACE_BYTES];

struct ScratchTable {
  std::mutex lock;
  std::map<int, char*> addr;                        // device -> address of `scratch`
  std::map<int, std::unique_ptr<std::mutex>> busy;  // device -> one call at a time
};

ScratchTable& scratch_table() {
  static ScratchTable t;
  return t;
}

// Address of this device's copy of `scratch` (the device is current) and the
// lock that serialises its users.
lshom_status scratch_for(lshom_ctx* c, char** out, std::mutex** busy) {
  ScratchTable& t = scratch_table();
  std::lock_guard<std::mutex> guard(t.lock);
  auto it = t.addr.find(c->device);
  if (it == t.addr.end()) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, LSHOM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    it = t.addr.emplace(c->device, static_cast<char*>(p)).first;
    t.busy.emplace(c->device, std::make_unique<std::mutex>());
  }
  *out = it->second;
  *busy = t.busy[c->device].get();
  return LSHOM_OK;
}

}  // namespace

extern "C" {

lshom_status lshom_solve_static(lshom_ctx* c, const double* E_host, double tol, const lshom_solve_opts* opts,
                                double* e_dev, double* leff_host, lshom_solve_info* info) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return fail(c, LSHOM_ERR_STATE, "set_microstructure has not been called");
  lshom_solve_opts o;
  lshom_default_opts(&o);
  if (opts) o = *opts;
  lshom_status s = validate_opts(c, &o);
  if (s != LSHOM_OK) return s;
  const bool extra = o.method == LSHOM_METHOD_BICG || o.method == LSHOM_METHOD_PIPECG;
  const Layout need = compute_layout(c->g, o.precision == LSHOM_PRECISION_MIXED, extra);
  if (need.total > LSHOM_STATIC_WORKSPACE_BYTES)
    return fail(c, LSHOM_ERR_UNSUPPORTED,
                "this problem needs " + std::to_string(need.total) + " bytes of workspace; the static scratch holds " +
                    std::to_string((size_t)LSHOM_STATIC_WORKSPACE_BYTES) + " (use lshom_solve with a workspace)");
  DeviceGuard dg(c->device);
  char* ptr = nullptr;
  std::mutex* busy = nullptr;
  if ((s = scratch_for(c, &ptr, &busy)) != LSHOM_OK) return s;
  std::lock_guard<std::mutex> one_at_a_time(*busy);
  // the context lends its problem; its own workspace (and the iteration
  // graphs captured on it) come back on every exit
  struct Restore {
    lshom_ctx* c;
    char* ws;
    Layout lay;
    size_t bytes;
    bool ready;
    ~Restore() {
      c->g.ws = ws;
      c->g.lay = lay;
      c->ws_bytes = bytes;
      c->ws_ready = ready;
    }
  } restore{c, c->g.ws, c->g.lay, c->ws_bytes, c->ws_ready};
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->g.ws = ptr;
  c->g.lay = need;
  c->ws_bytes = LSHOM_STATIC_WORKSPACE_BYTES;
  c->ws_ready = false;
  if ((s = prepare_workspace(c->g, c->cond, nullptr, {c->g.phase})) != LSHOM_OK) return s;
  c->ws_ready = true;
  o.graph_block = 0;
  return lshom_solve(c, E_host, tol, &o, nullptr, e_dev, leff_host, info);
}

lshom_status lshom_homogenize(lshom_ctx* c, double tol, const lshom_solve_opts* opts,
                              double* leff_host, lshom_solve_info* infos) {
  if (!c || !leff_host) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return fail(c, LSHOM_ERR_STATE, "set_microstructure has not been called");
  const int d = c->g.d;
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
  s = apply_real(c->g, p_dev, q_dev);
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
  s = time_passes(c->g, precision, reps, ms_out, bytes_out);
  if (s == LSHOM_OK) c->err.clear();
  return s;
}

// ---------------------------------------------------------------------------
// Many problems: one group (same launches) per distinct grid
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {

struct BatchPlan {
  std::vector<Group> groups;
  std::vector<std::vector<int>> members;  // problem indices of each group
  std::vector<size_t> offsets;            // workspace offset of each group
  size_t total = 0;
};

lshom_status plan_batch(lshom_ctx* c, int n, const lshom_problem* probs, int precision, BatchPlan* bp) {
  if (n < 1 || !probs) return fail(c, LSHOM_ERR_INVALID_ARG, "n must be >= 1 and probs non-NULL");
  std::map<std::vector<int64_t>, int> by_grid;
  for (int i = 0; i < n; ++i) {
    const lshom_problem& p = probs[i];
    lshom_status s = lshom_check_problem(p.d, p.N, p.n_phases, p.cond_host, p.l0 > 0 ? p.l0 : 0.0, p.E, p.tol);
    if (s != LSHOM_OK) return fail(c, s, "problem " + std::to_string(i) + " is invalid");
    if (!p.phase_dev) return fail(c, LSHOM_ERR_INVALID_ARG, "problem " + std::to_string(i) + ": phase_dev is NULL");
    {
      bool zero = true, ok = true;
      for (int a = 0; a < p.d; ++a) {
        zero = zero && p.cell[a] == 0.0;
        ok = ok && std::isfinite(p.cell[a]) && p.cell[a] > 0.0;
      }
      if (!zero && !ok)
        return fail(c, LSHOM_ERR_INVALID_ARG, "problem " + std::to_string(i) + ": cell lengths must be all 0 or > 0");
    }
    if (!(p.tol >= 0.0)) return fail(c, LSHOM_ERR_INVALID_ARG, "problem " + std::to_string(i) + ": tol < 0");
    // problems share launches when they share the grid and the cell
    std::vector<int64_t> key(p.N, p.N + p.d);
    key.insert(key.begin(), p.d);
    for (int a = 0; a < p.d; ++a) {
      int64_t bits;
      std::memcpy(&bits, &p.cell[a], sizeof(bits));
      key.push_back(bits);
    }
    auto it = by_grid.find(key);
    if (it == by_grid.end()) {
      it = by_grid.emplace(key, (int)bp->groups.size()).first;
      bp->groups.emplace_back();
      bp->members.emplace_back();
    }
    bp->members[it->second].push_back(i);
  }
  size_t off = 0;
  for (size_t gi = 0; gi < bp->groups.size(); ++gi) {
    Group& g = bp->groups[gi];
    const lshom_problem& p0 = probs[bp->members[gi][0]];
    int nph = 1;
    for (int i : bp->members[gi]) nph = std::max(nph, probs[i].n_phases);
    g.ctx = c;
    if (group_setup(g, p0.d, p0.N, nph) != LSHOM_OK)
      return fail(c, LSHOM_ERR_UNSUPPORTED, "grid too long for one LDS-resident FFT batch");
    for (int a = 0; a < p0.d; ++a) g.cell_inv[a] = p0.cell[a] > 0.0 ? 1.0 / p0.cell[a] : 1.0;
    g.nprob = (int)bp->members[gi].size();
    g.batched = true;
    g.lay = compute_layout(g, precision == LSHOM_PRECISION_MIXED);
    bp->offsets.push_back(off);
    off += (g.lay.total + kAlign - 1) / kAlign * kAlign;
  }
  bp->total = off;
  return LSHOM_OK;
}

// Carve group gi of a batch plan in the workspace and upload its tables.
lshom_status prepare_batch_group(lshom_ctx* c, BatchPlan& bp, size_t gi, const lshom_problem* probs,
                                 void* ws_dev, const lshom_solve_opts& o, std::vector<ProbEntry>* tab,
                                 std::vector<DevState>* init) {
  Group& g = bp.groups[gi];
  const std::vector<int>& mem = bp.members[gi];
  g.ws = static_cast<char*>(ws_dev) + bp.offsets[gi];
  std::vector<double> cond((size_t)g.nprob * g.n_phases, 1.0);
  tab->assign(g.nprob, ProbEntry{});
  init->assign(g.nprob, DevState{});
  std::vector<const uint8_t*> phases;
  g.warm_has.assign(g.nprob, 0);
  g.warm_any = false;
  for (int j = 0; j < g.nprob; ++j) {
    const lshom_problem& p = probs[mem[j]];
    g.warm_has[j] = p.x0_dev ? 1 : 0;
    g.warm_any = g.warm_any || p.x0_dev;
    double lo = p.cond_host[0], hi = p.cond_host[0];
    for (int i = 0; i < p.n_phases; ++i) {
      cond[(size_t)j * g.n_phases + i] = p.cond_host[i];
      lo = std::min(lo, p.cond_host[i]);
      hi = std::max(hi, p.cond_host[i]);
    }
    ProbEntry& e = (*tab)[j];
    e.phase = p.phase_dev;
    e.e_out = p.e_dev;
    e.x0 = p.x0_dev;
    e.l0 = p.l0 > 0.0 ? p.l0 : 0.5 * (lo + hi);
    phases.push_back(p.phase_dev);
    (*init)[j] = initial_state(p.d, g.nvox, p.E, p.tol, e.l0, o, false);
  }
  lshom_status s = prepare_workspace(g, cond, tab, phases);
  if (s != LSHOM_OK) return s;
  // a phase index must be below the problem's own phase count: conductivities
  // beyond it are never valid, so they are poisoned (the solve then breaks down)
  for (int j = 0; j < g.nprob; ++j) {
    const int np = probs[mem[j]].n_phases;
    if (np >= g.n_phases) continue;
    std::vector<double> bad((size_t)(g.n_phases - np), std::nan(""));
    std::vector<float> badf(bad.size(), std::nanf(""));
    HIP_TRY(c, hipMemcpyAsync(g.ws + g.lay.off_cond64 + ((size_t)j * kCondStride + np) * sizeof(double),
                              bad.data(), bad.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(g.ws + g.lay.off_cond32 + ((size_t)j * kCondStride + np) * sizeof(float),
                              badf.data(), badf.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return LSHOM_OK;
}

void to_c_schedule(const Group& g, const Schedule& s, int precision, lshom_schedule* out) {
  std::memset(out, 0, sizeof(*out));
  out->d = g.d;
  for (int a = 0; a < 3; ++a) out->N[a] = g.N[a];
  out->precision = precision;
  out->rows_per_block = s.shape.rows_per_block;
  out->tile0 = s.shape.tile0;
  out->tile1 = s.shape.tile1;
  out->row_split = s.shape.row_split;
  out->threads_row = s.shape.threads_row;
  out->threads_col = s.shape.threads_col;
  for (int a = 0; a < g.d; ++a) {
    out->nstages[a] = s.plan[a].nstages;
    for (int k = 0; k < s.plan[a].nstages; ++k) out->radix[a][k] = s.plan[a].radix[k];
  }
  out->ms_per_iter = s.ms_per_iter;
  out->tail_rows = s.tail_rows;
}

lshom_status from_c_schedule(lshom_ctx* c, const lshom_schedule* in, Schedule* s) {
  if (in->d != 2 && in->d != 3) return fail(c, LSHOM_ERR_INVALID_ARG, "schedule: d must be 2 or 3");
  if (in->precision != LSHOM_PRECISION_FP64 && in->precision != LSHOM_PRECISION_MIXED)
    return fail(c, LSHOM_ERR_INVALID_ARG, "schedule: precision must be 0 or 1");
  for (int a = 0; a < in->d; ++a) {
    if (in->nstages[a] < 1 || in->nstages[a] > kMaxStages ||
        !make_plan((int)in->N[a], in->radix[a], in->nstages[a], &s->plan[a]))
      return fail(c, LSHOM_ERR_INVALID_ARG, "schedule: radices do not factor N");
  }
  s->shape.rows_per_block = in->rows_per_block;
  s->shape.tile0 = in->tile0;
  s->shape.tile1 = in->d == 3 ? in->tile1 : 1;
  s->shape.row_split = in->row_split;
  s->shape.threads_row = in->threads_row;
  s->shape.threads_col = in->threads_col;
  s->ms_per_iter = in->ms_per_iter;
  if (in->tail_rows < 0) return fail(c, LSHOM_ERR_INVALID_ARG, "schedule: tail_rows must be >= 0");
  s->tail_rows = in->tail_rows;
  return LSHOM_OK;
}

std::string arch_name(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

}  // namespace

extern "C" {

lshom_status lshom_batch_workspace_size(lshom_ctx* c, int32_t n, const lshom_problem* probs,
                                        int precision, size_t* bytes) {
  if (!c || !bytes) return LSHOM_ERR_INVALID_ARG;
  if (precision != LSHOM_PRECISION_FP64 && precision != LSHOM_PRECISION_MIXED)
    return fail(c, LSHOM_ERR_INVALID_ARG, "precision must be FP64 (0) or MIXED (1)");
  BatchPlan bp;
  lshom_status s = plan_batch(c, n, probs, precision, &bp);
  if (s != LSHOM_OK) return s;
  *bytes = bp.total;
  return LSHOM_OK;
}

lshom_status lshom_solve_batched(lshom_ctx* c, int32_t n, const lshom_problem* probs,
                                 const lshom_solve_opts* opts, void* ws_dev, size_t ws_bytes,
                                 double* leff_host, lshom_solve_info* infos) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  lshom_solve_opts o;
  lshom_default_opts(&o);
  if (opts) o = *opts;
  lshom_status s = validate_opts(c, &o);
  if (s != LSHOM_OK) return s;
  if (o.history_dev) return fail(c, LSHOM_ERR_INVALID_ARG, "history_dev must be NULL for batched solves");
  if (o.method == LSHOM_METHOD_BICG || o.method == LSHOM_METHOD_PIPECG)
    return fail(c, LSHOM_ERR_UNSUPPORTED, "BiCG and pipelined CG run single solves only");
  BatchPlan bp;
  if ((s = plan_batch(c, n, probs, o.precision, &bp)) != LSHOM_OK) return s;
  if (o.method != LSHOM_METHOD_CG)
    for (int32_t i = 0; i < n; ++i)
      if (probs[i].x0_dev)
        return fail(c, LSHOM_ERR_UNSUPPORTED, "the basic scheme starts from e = E (problem " + std::to_string(i) +
                                                  " has x0_dev)");
  for (int32_t i = 0; i < n; ++i)
    if ((s = check_equilibrium_grid(c, o, probs[i].N, probs[i].d)) != LSHOM_OK) return s;
  if (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) % kAlign) != 0)
    return fail(c, LSHOM_ERR_WORKSPACE, "workspace must be non-NULL and 256-byte aligned");
  if (ws_bytes < bp.total) return fail(c, LSHOM_ERR_WORKSPACE, "workspace smaller than lshom_batch_workspace_size()");
  DeviceGuard dg(c->device);
  HIP_TRY(c, order_after_user(c));
  lshom_status worst = LSHOM_OK;
  const size_t ng = bp.groups.size();
  std::vector<std::vector<ProbEntry>> tabs(ng);
  std::vector<std::vector<DevState>> inits(ng);
  if (c->batch_graphs.size() + ng > 64) drop_batch_graphs(c);
  for (size_t gi = 0; gi < ng; ++gi) {
    Group& g = bp.groups[gi];
    if ((s = prepare_batch_group(c, bp, gi, probs, ws_dev, o, &tabs[gi], &inits[gi])) != LSHOM_OK) return s;
    // the captured launches carry the group's wave-vector scale 1 / Y (cell
    // side lengths) as kernel arguments, so the cell is part of the tag
    std::vector<long long> tag = {(long long)reinterpret_cast<uintptr_t>(g.ws), g.d, (long long)g.N[0],
                                  (long long)g.N[1], (long long)g.N[2], g.nprob, g.n_phases,
                                  (long long)g.lay.total, g.lay.has32 ? 1 : 0};
    for (int a = 0; a < 3; ++a) {
      long long bits;
      std::memcpy(&bits, &g.cell_inv[a], sizeof(bits));
      tag.push_back(bits);
    }
    g.graph_cache = &c->batch_graphs[tag];
  }
  // Grids of different sizes run concurrently: each group on a stream of its
  // own, driven by a host thread of its own (its blocks, read-backs and
  // schedule switches are independent of the other groups'), so the
  // launch-bound small grids and the tails of the large ones overlap.  With
  // pass timing on (one event pool) they run one after another.
  std::vector<lshom_status> gst(ng, LSHOM_OK);
  if (ng > 1 && !c->timer.on) {
    while (c->group_streams.size() < ng) {
      hipStream_t st = nullptr;
      HIP_TRY(c, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      c->group_streams.push_back(st);
    }
    // the set-up above is ordered on the context stream
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::vector<std::thread> th;
    th.reserve(ng);
    for (size_t gi = 0; gi < ng; ++gi) {
      bp.groups[gi].stream = c->group_streams[gi];
      th.emplace_back([&, gi] {
        if (hipSetDevice(c->device) != hipSuccess) {
          gst[gi] = fail(c, LSHOM_ERR_HIP, "hipSetDevice in a group thread");
          return;
        }
        gst[gi] = solve_group(bp.groups[gi], inits[gi], o, nullptr, nullptr, nullptr);
        (void)hipStreamSynchronize(bp.groups[gi].stream);
      });
    }
    for (std::thread& t : th) t.join();
    for (size_t gi = 0; gi < ng; ++gi) bp.groups[gi].stream = nullptr;
  } else {
    for (size_t gi = 0; gi < ng && (gi == 0 || gst[gi - 1] == LSHOM_OK); ++gi)
      gst[gi] = solve_group(bp.groups[gi], inits[gi], o, nullptr, nullptr, nullptr);
  }
  for (size_t gi = 0; gi < ng; ++gi)
    if (gst[gi] != LSHOM_OK) return gst[gi];
  for (size_t gi = 0; gi < ng; ++gi) {
    Group& g = bp.groups[gi];
    const std::vector<ProbEntry>& tab = tabs[gi];
    const std::vector<int>& mem = bp.members[gi];
    for (int j = 0; j < g.nprob; ++j) {
      const DevState& hs = g.host_states[j];
      const int i = mem[j];
      if (leff_host)
        for (int t = 0; t < 3; ++t) leff_host[(size_t)i * 3 + t] = t < g.d ? hs.leff[t] : 0.0;
      if (infos) fill_info(hs, tab[j].l0, o, j < (int)g.warm_flags.size() ? g.warm_flags[j] : 0, &infos[i]);
      if (hs.status != LSHOM_OK && worst == LSHOM_OK) worst = hs.status;
    }
  }
  if (worst == LSHOM_OK) c->err.clear();
  return worst;
}

lshom_status lshom_get_schedule(lshom_ctx* c, int precision, lshom_schedule* out) {
  if (!c || !out) return LSHOM_ERR_INVALID_ARG;
  if (!c->have_problem) return fail(c, LSHOM_ERR_STATE, "set_microstructure has not been called");
  if (precision != LSHOM_PRECISION_FP64 && precision != LSHOM_PRECISION_MIXED)
    return fail(c, LSHOM_ERR_INVALID_ARG, "precision must be FP64 (0) or MIXED (1)");
  Schedule s = current_schedule(c->g, precision);
  auto it = c->schedules.find(SchedKey(c->g.d, c->g.N[0], c->g.N[1], c->g.N[2], precision));
  if (it != c->schedules.end()) s.ms_per_iter = it->second.ms_per_iter;
  to_c_schedule(c->g, s, precision, out);
  return LSHOM_OK;
}

lshom_status lshom_set_schedule(lshom_ctx* c, const lshom_schedule* in) {
  if (!c || !in) return LSHOM_ERR_INVALID_ARG;
  Schedule s;
  lshom_status st = from_c_schedule(c, in, &s);
  if (st != LSHOM_OK) return st;
  Group probe;
  if (group_setup(probe, in->d, in->N, c->have_problem ? c->g.n_phase_ids : 1, c->have_problem && c->g.tensor) !=
      LSHOM_OK)
    return fail(c, LSHOM_ERR_UNSUPPORTED, "grid too long for one LDS-resident FFT batch");
  if (!schedule_fits(probe, s, in->precision))
    return fail(c, LSHOM_ERR_INVALID_ARG, "schedule exceeds the FFT batch or LDS limits");
  if (s.tail_rows > 0) {
    // a tail schedule serves batched launches only (kept under precision + 2)
    c->schedules[SchedKey(in->d, probe.N[0], probe.N[1], probe.N[2], in->precision + 2)] = s;
    drop_batch_graphs(c);
    c->err.clear();
    return LSHOM_OK;
  }
  c->schedules[SchedKey(in->d, probe.N[0], probe.N[1], probe.N[2], in->precision)] = s;
  if (c->have_problem && c->g.d == in->d && c->g.N[0] == probe.N[0] && c->g.N[1] == probe.N[1] &&
      c->g.N[2] == probe.N[2] && schedule_fits(c->g, s, in->precision)) {
    DeviceGuard dg(c->device);
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c->graphs);
    drop_batch_graphs(c);
    apply_schedule(c->g, s, in->precision);
  }
  c->err.clear();
  return LSHOM_OK;
}

lshom_status lshom_autotune(lshom_ctx* c, int precision, int reps, lshom_schedule* best) {
  if (!c || reps < 1) return LSHOM_ERR_INVALID_ARG;
  if (precision != LSHOM_PRECISION_FP64 && precision != LSHOM_PRECISION_MIXED)
    return fail(c, LSHOM_ERR_INVALID_ARG, "precision must be FP64 (0) or MIXED (1)");
  lshom_status s = check_ready(c, precision);
  if (s != LSHOM_OK) return s;
  DeviceGuard dg(c->device);
  HIP_TRY(c, order_after_user(c));
  drop_graphs(c->graphs);
  drop_batch_graphs(c);
  Schedule tuned;
  if ((s = autotune_group(c->g, precision, reps, &tuned)) != LSHOM_OK) return s;
  apply_schedule(c->g, tuned, precision);
  c->schedules[SchedKey(c->g.d, c->g.N[0], c->g.N[1], c->g.N[2], precision)] = tuned;
  if (best) to_c_schedule(c->g, tuned, precision, best);
  c->err.clear();
  return LSHOM_OK;
}

lshom_status lshom_autotune_batched(lshom_ctx* c, int32_t n, const lshom_problem* probs, int precision,
                                    int reps, void* ws_dev, size_t ws_bytes, lshom_schedule* best,
                                    int32_t* n_best) {
  if (!c || reps < 1) return LSHOM_ERR_INVALID_ARG;
  if (precision != LSHOM_PRECISION_FP64 && precision != LSHOM_PRECISION_MIXED)
    return fail(c, LSHOM_ERR_INVALID_ARG, "precision must be FP64 (0) or MIXED (1)");
  BatchPlan bp;
  lshom_status s = plan_batch(c, n, probs, precision, &bp);
  if (s != LSHOM_OK) return s;
  if (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) % kAlign) != 0)
    return fail(c, LSHOM_ERR_WORKSPACE, "workspace must be non-NULL and 256-byte aligned");
  if (ws_bytes < bp.total) return fail(c, LSHOM_ERR_WORKSPACE, "workspace smaller than lshom_batch_workspace_size()");
  DeviceGuard dg(c->device);
  HIP_TRY(c, order_after_user(c));
  lshom_solve_opts o;
  lshom_default_opts(&o);
  o.precision = precision;
  const int cap = n_best ? *n_best : 0;
  int n_tail = 0;
  for (size_t gi = 0; gi < bp.groups.size(); ++gi) {
    Group& g = bp.groups[gi];
    std::vector<ProbEntry> tab;
    std::vector<DevState> init;
    if ((s = prepare_batch_group(c, bp, gi, probs, ws_dev, o, &tab, &init)) != LSHOM_OK) return s;
    // the timing needs meaningful vectors: one short solve fills them
    lshom_solve_opts warm = o;
    warm.max_iter = 2;
    warm.graph_block = 0;
    std::vector<DevState> short_init = init;
    for (DevState& st : short_init) st.max_iter = 2;
    if ((s = solve_group(g, short_init, warm, nullptr, nullptr, nullptr)) != LSHOM_OK) return s;
    Schedule tuned;
    if ((s = autotune_group(g, precision, reps, &tuned)) != LSHOM_OK) return s;
    c->schedules[SchedKey(g.d, g.N[0], g.N[1], g.N[2], precision)] = tuned;
    if (best && (int)gi < cap) to_c_schedule(g, tuned, precision, &best[gi]);
    // the tail of the batch: launches that cover only kTailRows unfinished
    // problems (few blocks per CU) are tuned on their own
    if (g.nprob > kTailRows) {
      Schedule tail;
      if ((s = autotune_tail(g, precision, reps, kTailRows, &tail)) != LSHOM_OK) return s;
      apply_schedule(g, tuned, precision);
      c->schedules[SchedKey(g.d, g.N[0], g.N[1], g.N[2], precision + 2)] = tail;
      if (best && (int)(bp.groups.size() + n_tail) < cap)
        to_c_schedule(g, tail, precision, &best[bp.groups.size() + n_tail]);
      ++n_tail;
    }
  }
  drop_batch_graphs(c);  // captured with the previous schedules
  if (n_best) *n_best = (int32_t)(bp.groups.size() + n_tail);
  c->err.clear();
  return LSHOM_OK;
}

lshom_status lshom_set_pass_timing(lshom_ctx* c, int enable) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  c->timer.on = enable != 0;
  c->timer.reset();
  return LSHOM_OK;
}

lshom_status lshom_get_pass_timing(lshom_ctx* c, double* ms_out, double* bytes_out, int64_t* launches_out) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  for (int k = 0; k < LSHOM_PASS_COUNT; ++k) {
    if (ms_out) ms_out[k] = c->timer.ms[k];
    if (bytes_out) bytes_out[k] = c->timer.bytes[k];
    if (launches_out) launches_out[k] = c->timer.launches[k];
  }
  return LSHOM_OK;
}

lshom_status lshom_save_schedules(lshom_ctx* c, const char* path) {
  if (!c || !path) return LSHOM_ERR_INVALID_ARG;
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(c, LSHOM_ERR_INVALID_ARG, std::string("cannot write ") + path);
  const std::string arch = arch_name(c->device);
  for (const auto& kv : c->schedules) {
    const int d = std::get<0>(kv.first);
    const int prec = std::get<4>(kv.first) & 1;
    const Schedule& s = kv.second;
    std::fprintf(f, "{\"arch\": \"%s\", \"d\": %d, \"N\": [%lld, %lld, %lld], \"precision\": %d, "
                    "\"rows_per_block\": %d, \"row_split\": %d, \"threads_row\": %d, \"threads_col\": %d, "
                    "\"tile0\": %d, \"tile1\": %d, \"radix\": [",
                 arch.c_str(), d, (long long)std::get<1>(kv.first), (long long)std::get<2>(kv.first),
                 (long long)std::get<3>(kv.first), prec, s.shape.rows_per_block, s.shape.row_split,
                 s.shape.threads_row, s.shape.threads_col, s.shape.tile0, s.shape.tile1);
    for (int a = 0; a < d; ++a) {
      std::fprintf(f, "%s[", a ? ", " : "");
      for (int k = 0; k < s.plan[a].nstages; ++k) std::fprintf(f, "%s%d", k ? ", " : "", s.plan[a].radix[k]);
      std::fprintf(f, "]");
    }
    std::fprintf(f, "], \"ms_per_iter\": %.9g, \"tail_rows\": %d}\n", s.ms_per_iter, s.tail_rows);
  }
  std::fclose(f);
  return LSHOM_OK;
}

// Integers in s after `key` up to the end of its value (a number or a
// bracketed list, nested one level).
static bool json_ints(const std::string& s, const char* key, std::vector<long long>* out) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = s.find(k);
  if (p == std::string::npos) return false;
  p = s.find(':', p + k.size());
  if (p == std::string::npos) return false;
  ++p;
  while (p < s.size() && s[p] == ' ') ++p;
  size_t end = p;
  if (s[p] == '[') {
    int depth = 0;
    for (end = p; end < s.size(); ++end) {
      if (s[end] == '[') ++depth;
      if (s[end] == ']' && --depth == 0) break;
    }
  } else {
    while (end < s.size() && s[end] != ',' && s[end] != '}') ++end;
  }
  out->clear();
  long long v = 0;
  bool in = false, neg = false;
  for (size_t i = p; i <= end && i < s.size(); ++i) {
    const char ch = s[i];
    if (ch >= '0' && ch <= '9') {
      v = v * 10 + (ch - '0');
      in = true;
    } else if (ch == '-' && !in) {
      neg = true;
    } else {
      if (in) out->push_back(neg ? -v : v);
      v = 0;
      in = false;
      neg = false;
      if (ch == '.') return true;  // fractional part: keep the integer
    }
  }
  if (in) out->push_back(neg ? -v : v);
  return true;
}

lshom_status lshom_load_schedules(lshom_ctx* c, const char* path) {
  if (!c || !path) return LSHOM_ERR_INVALID_ARG;
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(c, LSHOM_ERR_INVALID_ARG, std::string("cannot read ") + path);
  const std::string arch = arch_name(c->device);
  char buf[4096];
  while (std::fgets(buf, sizeof(buf), f)) {
    std::string line(buf);
    if (line.find('{') == std::string::npos) continue;
    if (line.find("\"arch\": \"" + arch + "\"") == std::string::npos) continue;
    std::vector<long long> d, N, prec, rows, t0, t1, radix, split, ntr, ntc;
    if (!json_ints(line, "d", &d) || !json_ints(line, "N", &N) || !json_ints(line, "precision", &prec) ||
        !json_ints(line, "rows_per_block", &rows) || !json_ints(line, "tile0", &t0) ||
        !json_ints(line, "tile1", &t1) || d.size() != 1 || N.size() != 3) {
      std::fclose(f);
      return fail(c, LSHOM_ERR_INVALID_ARG, "schedule cache: malformed line");
    }
    lshom_schedule in;
    std::memset(&in, 0, sizeof(in));
    in.d = (int)d[0];
    for (int a = 0; a < 3; ++a) in.N[a] = N[a];
    in.precision = (int)prec[0];
    in.rows_per_block = (int)rows[0];
    in.tile0 = (int)t0[0];
    in.tile1 = (int)t1[0];
    in.row_split = (json_ints(line, "row_split", &split) && split.size() == 1) ? (int)split[0] : 0;
    in.threads_row = (json_ints(line, "threads_row", &ntr) && ntr.size() == 1) ? (int)ntr[0] : 0;
    in.threads_col = (json_ints(line, "threads_col", &ntc) && ntc.size() == 1) ? (int)ntc[0] : 0;
    std::vector<long long> tr;
    in.tail_rows = (json_ints(line, "tail_rows", &tr) && tr.size() == 1) ? (int)tr[0] : 0;
    // radix lists: split the bracketed value by inner brackets
    const size_t rp = line.find("\"radix\"");
    if (rp == std::string::npos) {
      std::fclose(f);
      return fail(c, LSHOM_ERR_INVALID_ARG, "schedule cache: missing radix");
    }
    size_t p = line.find('[', rp);
    for (int a = 0; a < in.d; ++a) {
      p = line.find('[', p + 1);
      const size_t e = line.find(']', p);
      if (p == std::string::npos || e == std::string::npos) {
        std::fclose(f);
        return fail(c, LSHOM_ERR_INVALID_ARG, "schedule cache: malformed radix list");
      }
      int k = 0;
      long long v = 0;
      bool inn = false;
      for (size_t i = p + 1; i <= e; ++i) {
        const char ch = line[i];
        if (ch >= '0' && ch <= '9') {
          v = v * 10 + (ch - '0');
          inn = true;
        } else if (inn) {
          if (k < 16) in.radix[a][k++] = (int)v;
          v = 0;
          inn = false;
        }
      }
      in.nstages[a] = k;
      p = e;
    }
    lshom_status s = lshom_set_schedule(c, &in);
    if (s != LSHOM_OK) {
      std::fclose(f);
      return s;
    }
  }
  std::fclose(f);
  return LSHOM_OK;
}

}  // extern "C"
