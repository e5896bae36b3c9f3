// Solve drivers: queue the pass kernels of the operator apply (Sec. 2.2,
// Eq. (16)) and of conjugate gradients (Sec. 2.3; Saad's Algorithm 6.18 as
// named in Sec. 3) on the context stream, in captured HIP graph blocks.
#include <cmath>
#include <cstring>

#include "ctx.hpp"

namespace lshom {

lshom_status fail(lshom_ctx* c, lshom_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

void drop_graphs(lshom_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

namespace {

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

long long inner0_of(const lshom_ctx* c) {
  long long inner = c->h;
  for (int t = 1; t < c->d - 1; ++t) inner *= c->N[t];
  return inner;
}

}  // namespace

Layout compute_layout(const lshom_ctx* c, bool with32) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.off_state = take(sizeof(DevState));
  L.off_scratch = take(256);
  // partial sums: one slot (three in AUX) per block of the widest launch
  long long maxb = kUpdateBlocks;
  for (int prec = 0; prec < (with32 ? 2 : 1); ++prec) {
    const PassShape& s = prec == 0 ? c->shape64 : c->shape32;
    maxb = std::max(maxb, ceil_div(c->nrows, s.rows_per_block));
    maxb = std::max(maxb, ceil_div(inner0_of(c), s.tile0));
    if (c->d == 3) maxb = std::max(maxb, c->N[0] * ceil_div(c->h, s.tile1));
  }
  L.part_stride = 3 * maxb;
  L.off_partials = take((size_t)L.part_stride * 4 * sizeof(double));
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

namespace {

DevState* dev_state(lshom_ctx* c) { return reinterpret_cast<DevState*>(c->ws + c->lay.off_state); }

Partials dev_parts(lshom_ctx* c) {
  Partials p;
  p.base = reinterpret_cast<double*>(c->ws + c->lay.off_partials);
  p.stride = c->lay.part_stride;
  return p;
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

// ---------------------------------------------------------------------------
// Pass argument builders
// ---------------------------------------------------------------------------

template <typename T>
ColArgs<T> col0_args(lshom_ctx* c, const Bufs<T>& b) {
  ColArgs<T> a{};
  a.L = (int)c->N[0];
  a.inner = inner0_of(c);
  a.outer = 1;
  if (c->transposed) {
    a.sl = 1;
    a.sii = a.L;
  } else {
    a.sl = a.inner;
    a.sii = 1;
  }
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
  a.parts = dev_parts(c);
  a.inv_n = 1.0 / (double)c->nvox;
  a.gate = GATE_ACTIVE;
  return a;
}

template <typename T>
ColArgs<T> col1_args(lshom_ctx* c, const Bufs<T>& b, int dir) {
  ColArgs<T> a{};
  a.L = (int)c->N[1];
  a.inner = c->h;
  a.outer = c->N[0];
  a.sl = a.inner;
  a.sii = 1;
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
  a.parts = dev_parts(c);
  a.inv_n = 1.0 / (double)c->nvox;
  a.gate = GATE_ACTIVE;
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
  row_lds_bytes(a.n, a.rows_per_block, a.d, (int)sizeof(cx<T>), (int)c->cond.size(), &a.ss);
  if (c->transposed) {
    a.rs_row = 1;
    a.rs_k = c->nrows;
    a.row_fast = 1;
  } else {
    a.rs_row = c->h;
    a.rs_k = 1;
    a.row_fast = 0;
  }
  for (int t = 0; t < c->d; ++t) a.spec[t] = b.w[t];
  a.phase = c->phase;
  a.cond = b.cond;
  a.n_phases = (int)c->cond.size();
  a.l0 = (T)c->l0;
  a.inv_n = (T)(1.0 / (double)c->nvox);
  a.plan = c->plan[last];
  a.tw = b.tw[last];
  a.st = dev_state(c);
  a.parts = dev_parts(c);
  a.gate = GATE_ACTIVE;
  return a;
}

long long klast_div_of(const lshom_ctx* c) { return c->transposed ? c->N[0] : 1; }

template <typename T>
long long col0_block_count(lshom_ctx* c, const Bufs<T>& b) {
  return col_blocks(col0_args(c, b));
}

template <typename T>
long long row_block_count(lshom_ctx* c, const Bufs<T>& b) {
  return row_blocks(row_args(c, b));
}

hipError_t enq_finalize(lshom_ctx* c, int mode, long long n, int gate) {
  FinArgs f{};
  f.st = dev_state(c);
  f.parts = dev_parts(c);
  f.mode = mode;
  f.n = (int)n;
  f.d = c->d;
  f.inv_n = 1.0 / (double)c->nvox;
  f.gate = gate;
  return launch_finalize(f, c->stream);
}

// ---------------------------------------------------------------------------
// Operator sequences (see the pass kernels for the algebra)
// ---------------------------------------------------------------------------

// Forward half: [3-D axis-1 forward], axis-0 forward + projection.
template <typename T>
hipError_t enq_forward_project(lshom_ctx* c, const Bufs<T>& b, cx<T>* out, const cx<T>* base,
                               T coef_base, T coef_s, int dot, int dot_region, int gate) {
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
  a.dot_region = dot_region;
  a.gate = gate;
  return launch_col(a, c->stream);
}

// Inverse half: axis-0 inverse from the scalar c (or the CG direction step
// p = r + beta p), [3-D axis-1 inverse].
template <typename T>
hipError_t enq_inverse_from_c(lshom_ctx* c, const Bufs<T>& b, const cx<T>* c_in, cx<T>* p_io,
                              const cx<T>* r_in, int gate) {
  hipError_t e;
  ColArgs<T> a = col0_args(c, b);
  a.mode = COL_INV_C;
  a.c_in = c_in;
  a.p_io = p_io;
  a.r_in = r_in;
  a.cg_step = p_io != nullptr;
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
                          T coef_base, T coef_s, int dot, int dot_region, int gate) {
  hipError_t e;
  if ((e = enq_inverse_from_c(c, b, c_in, p_io, r_in, gate)) != hipSuccess) return e;
  RowArgs<T> r = row_args(c, b);
  r.mode = ROW_FUSED;
  for (int t = 0; t < c->d; ++t) r.E[t] = E ? (T)E[t] : T(0);
  r.gate = gate;
  if ((e = launch_row(r, c->stream)) != hipSuccess) return e;
  return enq_forward_project(c, b, out, base, coef_base, coef_s, dot, dot_region, gate);
}

// One CG iteration in the spectral coordinate:
//   direction step (p = r + beta p, or stop), q = p + (1/l0) P dL u(p) with
//   (p, q), then alpha = (r, r) / (p, q), x += alpha p, r -= alpha q, (r, r).
template <typename T>
hipError_t enq_cg_iteration(lshom_ctx* c, const Bufs<T>& b, int gate) {
  hipError_t e;
  cx<T>* r = b.v[1];
  cx<T>* p = b.v[2];
  cx<T>* q = b.v[3];
  if ((e = enq_apply_spec<T>(c, b, nullptr, p, r, nullptr, q, p, T(1), T(1.0 / c->l0), 1, PART_PQ,
                             gate)) != hipSuccess)
    return e;
  UpdArgs<T> u{};
  u.n = c->nhalf;
  u.h = c->h;
  u.n_last = (int)c->N[c->d - 1];
  u.klast_div = klast_div_of(c);
  u.x = b.v[0];
  u.r = r;
  u.p = p;
  u.q = q;
  u.st = dev_state(c);
  u.parts = dev_parts(c);
  u.n_pq = (int)col0_block_count(c, b);
  u.inv_n = 1.0 / (double)c->nvox;
  u.gate = gate;
  return launch_update(u, c->stream);
}

// Residual of the spectral iterate x for the load E:
// r = -(x + (1/l0) P dL (E + u(x))).
template <typename T>
hipError_t enq_true_residual(lshom_ctx* c, const Bufs<T>& b, const cx<T>* x, const double* E,
                             cx<T>* out, int dot_region, int gate) {
  return enq_apply_spec<T>(c, b, x, nullptr, nullptr, E, out, x, T(-1), T(-1.0 / c->l0), 2,
                           dot_region, gate);
}

// r0 for x0 = E: r0 = -(1/l0) P dL E.
template <typename T>
hipError_t enq_residual_of_E(lshom_ctx* c, const Bufs<T>& b, const double* E, cx<T>* out,
                             int dot_region) {
  hipError_t e;
  RowArgs<T> r = row_args(c, b);
  r.mode = ROW_FWD;
  r.flags = ROWF_DL | ROWF_CONST_E;
  for (int t = 0; t < c->d; ++t) r.E[t] = (T)E[t];
  r.gate = GATE_ALWAYS;
  if ((e = launch_row(r, c->stream)) != hipSuccess) return e;
  return enq_forward_project<T>(c, b, out, nullptr, T(0), T(-1.0 / c->l0), 2, dot_region,
                                GATE_ALWAYS);
}

// Real FP64 field v (d x |N|) -> spectral coordinate of P v (of P dL v / l0).
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
                                     PART_AUX, GATE_ALWAYS);
}

// Real field out = add + E + u(x); with leff, <lambda out> into state.leff.
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
  r.gate = GATE_ALWAYS;
  if ((e = launch_row(r, c->stream)) != hipSuccess) return e;
  if (leff) return enq_finalize(c, FZ_LEFF, row_blocks(r), GATE_ALWAYS);
  return hipSuccess;
}

MixArgs mix_args(lshom_ctx* c, const Bufs<double>& b64, const Bufs<float>& b32, int gate) {
  MixArgs m{};
  m.n = c->nhalf;
  m.h = c->h;
  m.n_last = (int)c->N[c->d - 1];
  m.klast_div = klast_div_of(c);
  m.x64 = b64.v[0];
  m.x32 = b32.v[0];
  m.r64 = b64.v[1];
  m.r32 = b32.v[1];
  m.st = dev_state(c);
  m.parts = dev_parts(c);
  m.inv_n = 1.0 / (double)c->nvox;
  m.gate = gate;
  return m;
}

// Mixed precision refresh (reliable update): x64 += x32, x32 = 0;
// r64 = b - A64 x64 in FP64; r32 = r64 with its (r, r) partials; the
// finalize step decides convergence on the FP64 value and clears the request.
hipError_t enq_mix_refresh(lshom_ctx* c, const Bufs<double>& b64, const Bufs<float>& b32,
                           const double* E, int gate) {
  hipError_t e;
  MixArgs m = mix_args(c, b64, b32, gate);
  if ((e = launch_mix_accumulate(m, c->stream)) != hipSuccess) return e;
  if ((e = enq_true_residual<double>(c, b64, b64.v[0], E, b64.v[1], PART_AUX, gate)) != hipSuccess)
    return e;
  if ((e = launch_mix_convert(m, c->stream)) != hipSuccess) return e;
  return enq_finalize(c, FZ_REFRESH, col0_block_count(c, b64), gate);
}

hipError_t sync_state(lshom_ctx* c) {
  hipError_t e = hipMemcpyAsync(c->host_state, dev_state(c), sizeof(DevState),
                                hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(c->stream);
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

DevState initial_state(const lshom_ctx* c, const double* E, double tol, int max_iter) {
  DevState s{};
  double e2 = 0.0;
  for (int t = 0; t < c->d; ++t) e2 += E[t] * E[t];
  s.b2 = e2 * (double)c->nvox;
  s.tol2b2 = tol * tol * s.b2;
  s.max_iter = max_iter;
  return s;
}

void fill_info(lshom_ctx* c, const lshom_solve_opts& o, int warm_used, bool mixed, lshom_solve_info* info) {
  const DevState& hs = *c->host_state;
  if (!info) return;
  info->iterations = hs.iter_a;
  info->applies_fp32 = mixed ? hs.iter_a : 0;
  info->applies_fp64 = mixed ? hs.n_refresh : hs.iter_a;
  info->status = hs.status;
  info->warm_start_used = warm_used;
  info->refreshes = mixed ? hs.n_refresh : 0;
  const double rr = mixed ? hs.rr_true : hs.rr_log;
  info->rel_res = std::sqrt(rr / hs.b2);
  info->rel_res_true = o.true_residual ? std::sqrt(hs.rr_true / hs.b2) : -1.0;
  info->eta_r = c->l0 * std::sqrt(rr / hs.b2);
}

}  // namespace

// ---------------------------------------------------------------------------
// Workspace preparation
// ---------------------------------------------------------------------------

lshom_status prepare_workspace(lshom_ctx* c) {
  const Layout& use = c->lay;
  std::vector<double> c64(kMaxPhases, 0.0);
  std::vector<float> c32(kMaxPhases, 0.0f);
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
  // every phase index must name a conductivity
  unsigned* mx = reinterpret_cast<unsigned*>(c->ws + use.off_scratch);
  unsigned host_max = 0;
  HIP_TRY(c, hipMemcpy(mx, &host_max, sizeof(unsigned), hipMemcpyHostToDevice));
  HIP_TRY(c, launch_max_phase(c->phase, c->nvox, mx, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(&host_max, mx, sizeof(unsigned), hipMemcpyDeviceToHost));
  if (host_max >= c->cond.size())
    return fail(c, LSHOM_ERR_INVALID_ARG, "phase image holds an index >= n_phases");
  return LSHOM_OK;
}

// ---------------------------------------------------------------------------
// FP64 solve: the plain method
// ---------------------------------------------------------------------------

lshom_status solve_fp64(lshom_ctx* c, const double* E, double tol, const lshom_solve_opts& o,
                        const double* x0, double* e_out, double* leff, lshom_solve_info* info) {
  Bufs<double> b = get_bufs<double>(c);
  cx<double>* x = b.v[0];
  cx<double>* r = b.v[1];
  cx<double>* p = b.v[2];
  cx<double>* q = b.v[3];
  const long long ncol = col0_block_count(c, b);
  DevState init = initial_state(c, E, tol, o.max_iter);
  HIP_TRY(c, launch_state_init(dev_state(c), init, c->stream));
  HIP_TRY(c, launch_fill_zero(x, c->nhalf, c->stream));
  HIP_TRY(c, launch_fill_zero(p, c->nhalf, c->stream));
  int warm_used = 0;
  if (x0) {
    // residual of E for the admissibility test, then of E + P x0
    HIP_TRY(c, (enq_residual_of_E<double>(c, b, E, r, PART_AUX)));
    HIP_TRY(c, enq_finalize(c, FZ_AUX, ncol, GATE_ALWAYS));
    HIP_TRY(c, enq_project_real(c, b, x0, false, x));
    HIP_TRY(c, (enq_true_residual<double>(c, b, x, E, r, PART_RR0, GATE_ALWAYS)));
    HIP_TRY(c, enq_finalize(c, FZ_CHECK, 0, GATE_ALWAYS));
    HIP_TRY(c, sync_state(c));
    const DevState& hs = *c->host_state;
    if (std::isfinite(hs.rr_log) && hs.rr_log < hs.dot_aux) {
      warm_used = 1;
    } else {
      HIP_TRY(c, launch_state_init(dev_state(c), init, c->stream));
      HIP_TRY(c, launch_fill_zero(x, c->nhalf, c->stream));
    }
  }
  if (!warm_used) {
    HIP_TRY(c, (enq_residual_of_E<double>(c, b, E, r, PART_RR0)));
    HIP_TRY(c, enq_finalize(c, FZ_CHECK, 0, GATE_ALWAYS));
  }
  const int K = o.graph_block;
  const int per = K > 0 ? K : 8;
  HIP_TRY(c, sync_state(c));
  lshom_status s = run_blocks(c, 0, K, (long long)o.max_iter / per + 4, [&]() -> hipError_t {
    for (int k = 0; k < per; ++k) {
      hipError_t e = enq_cg_iteration<double>(c, b, GATE_ACTIVE);
      if (e != hipSuccess) return e;
    }
    return enq_finalize(c, FZ_CHECK, 0, GATE_ACTIVE);
  });
  if (s != LSHOM_OK) return s;
  if (o.true_residual) {
    HIP_TRY(c, (enq_true_residual<double>(c, b, x, E, q, PART_AUX, GATE_ALWAYS)));
    HIP_TRY(c, enq_finalize(c, FZ_RR_TRUE, ncol, GATE_ALWAYS));
  }
  HIP_TRY(c, enq_field_out(c, b, x, E, nullptr, e_out, true));
  HIP_TRY(c, sync_state(c));
  const DevState& hs = *c->host_state;
  if (leff)
    for (int t = 0; t < c->d; ++t) leff[t] = hs.leff[t];
  fill_info(c, o, warm_used, false, info);
  return hs.status;
}

// ---------------------------------------------------------------------------
// Mixed precision: FP32 operator, FP32 vectors, FP64 dots; FP64 iterate and
// FP64 true residual at every refresh (reliable update; p is kept).
// ---------------------------------------------------------------------------

lshom_status solve_mixed(lshom_ctx* c, const double* E, double tol, const lshom_solve_opts& o,
                         const double* x0, double* e_out, double* leff, lshom_solve_info* info) {
  Bufs<double> b64 = get_bufs<double>(c);
  Bufs<float> b32 = get_bufs<float>(c);
  cx<double>* x64 = b64.v[0];
  cx<double>* r64 = b64.v[1];
  const long long ncol = col0_block_count(c, b64);
  DevState init = initial_state(c, E, tol, o.max_iter);
  init.refresh_every = o.refresh_every;
  init.drop2 = o.refresh_drop * o.refresh_drop;
  HIP_TRY(c, launch_state_init(dev_state(c), init, c->stream));
  HIP_TRY(c, launch_fill_zero(x64, c->nhalf, c->stream));
  HIP_TRY(c, launch_fill_zero(b32.v[0], c->nhalf, c->stream));
  HIP_TRY(c, launch_fill_zero(b32.v[2], c->nhalf, c->stream));
  int warm_used = 0;
  if (x0) {
    HIP_TRY(c, (enq_residual_of_E<double>(c, b64, E, r64, PART_AUX)));
    HIP_TRY(c, enq_finalize(c, FZ_AUX, ncol, GATE_ALWAYS));
    HIP_TRY(c, enq_project_real(c, b64, x0, false, x64));
    HIP_TRY(c, (enq_true_residual<double>(c, b64, x64, E, r64, PART_AUX, GATE_ALWAYS)));
    HIP_TRY(c, enq_finalize(c, FZ_REFRESH_INIT, ncol, GATE_ALWAYS));
    HIP_TRY(c, sync_state(c));
    const DevState& hs = *c->host_state;
    if (std::isfinite(hs.rr_true) && hs.rr_true < hs.dot_aux) {
      warm_used = 1;
    } else {
      HIP_TRY(c, launch_state_init(dev_state(c), init, c->stream));
      HIP_TRY(c, launch_fill_zero(x64, c->nhalf, c->stream));
    }
  }
  if (!warm_used) {
    HIP_TRY(c, (enq_residual_of_E<double>(c, b64, E, r64, PART_AUX)));
    HIP_TRY(c, enq_finalize(c, FZ_REFRESH_INIT, ncol, GATE_ALWAYS));
  }
  HIP_TRY(c, launch_mix_convert(mix_args(c, b64, b32, GATE_ALWAYS), c->stream));
  HIP_TRY(c, sync_state(c));
  const int K = o.graph_block;
  const int per = K > 0 ? K : 8;
  // a refresh may cut a block short: at least one iteration per block is certain
  lshom_status s = run_blocks(c, 1, K, (long long)o.max_iter + 4, [&]() -> hipError_t {
    for (int k = 0; k < per; ++k) {
      hipError_t e = enq_cg_iteration<float>(c, b32, GATE_NO_REFRESH);
      if (e != hipSuccess) return e;
    }
    return enq_mix_refresh(c, b64, b32, E, GATE_REFRESH);
  });
  if (s != LSHOM_OK) return s;
  // fold what a breakdown left in the FP32 correction (no-op after a refresh)
  HIP_TRY(c, launch_mix_accumulate(mix_args(c, b64, b32, GATE_ALWAYS), c->stream));
  if (o.true_residual) {
    HIP_TRY(c, (enq_true_residual<double>(c, b64, x64, E, b64.v[3], PART_AUX, GATE_ALWAYS)));
    HIP_TRY(c, enq_finalize(c, FZ_RR_TRUE, ncol, GATE_ALWAYS));
  }
  HIP_TRY(c, enq_field_out(c, b64, x64, E, nullptr, e_out, true));
  HIP_TRY(c, sync_state(c));
  const DevState& hs = *c->host_state;
  if (leff)
    for (int t = 0; t < c->d; ++t) leff[t] = hs.leff[t];
  fill_info(c, o, warm_used, true, info);
  return hs.status;
}

// ---------------------------------------------------------------------------
// One FP64 apply on a real field: q = p + B p
// ---------------------------------------------------------------------------

lshom_status apply_real(lshom_ctx* c, const double* p, double* q) {
  Bufs<double> b = get_bufs<double>(c);
  HIP_TRY(c, enq_project_real(c, b, p, true, b.v[3]));
  HIP_TRY(c, enq_field_out(c, b, b.v[3], nullptr, p, q, false));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LSHOM_OK;
}

// ---------------------------------------------------------------------------
// Per-kernel timing of one CG iteration's launches
// ---------------------------------------------------------------------------

namespace {

template <typename T>
lshom_status time_passes_t(lshom_ctx* c, const Bufs<T>& b, int reps, double* ms_out, double* bytes_out) {
  cx<T>* x = b.v[0];
  cx<T>* r = b.v[1];
  cx<T>* p = b.v[2];
  cx<T>* q = b.v[3];
  // a state in which the direction step proceeds (beta = 0) and the update
  // uses alpha = 0, so repeated launches keep the vectors bounded
  DevState init{};
  init.max_iter = 1 << 30;
  init.tol2b2 = -1.0;
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
  hipError_t err;
  {
    ColArgs<T> a = col0_args(c, b);
    a.mode = COL_INV_C;
    a.p_io = p;
    a.r_in = r;
    a.cg_step = 1;
    a.gate = GATE_ALWAYS;
    // reads r, p; writes p and the d pass components
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
    RowArgs<T> rr = row_args(c, b);
    rr.mode = ROW_FUSED;
    rr.gate = GATE_ALWAYS;
    // reads and writes the d components, reads one phase byte per voxel
    err = timed(LSHOM_PASS_ROW, 2.0 * d * nh * cs + (double)c->nvox, [&] { return launch_row(rr, c->stream); });
  }
  if (err == hipSuccess) {
    ColArgs<T> a = col0_args(c, b);
    a.mode = COL_FWD_PROJ;
    a.out = q;
    a.base = p;
    a.coef_base = T(1);
    a.coef_s = T(1.0 / c->l0);
    a.dot = 1;
    a.dot_region = PART_PQ;
    a.gate = GATE_ALWAYS;
    // reads the d components and p; writes q
    err = timed(LSHOM_PASS_AXIS0_FORWARD, (d + 2.0) * nh * cs, [&] { return launch_col(a, c->stream); });
  }
  if (err == hipSuccess) {
    UpdArgs<T> u{};
    u.n = c->nhalf;
    u.h = c->h;
    u.n_last = (int)c->N[c->d - 1];
    u.klast_div = klast_div_of(c);
    u.x = x;
    u.r = r;
    u.p = p;
    u.q = q;
    u.st = dev_state(c);
    u.parts = dev_parts(c);
    u.n_pq = (int)col0_block_count(c, b);
    u.inv_n = 1.0 / (double)c->nvox;
    u.gate = GATE_ALWAYS;
    // reads x, r, p, q; writes x, r
    err = timed(LSHOM_PASS_UPDATE, 6.0 * nh * cs, [&] { return launch_update(u, c->stream); });
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(c, LSHOM_ERR_HIP, std::string("time_passes: ") + hipGetErrorString(err));
  return LSHOM_OK;
}

}  // namespace

lshom_status time_passes(lshom_ctx* c, int precision, int reps, double* ms_out, double* bytes_out) {
  if (precision == LSHOM_PRECISION_FP64) return time_passes_t<double>(c, get_bufs<double>(c), reps, ms_out, bytes_out);
  return time_passes_t<float>(c, get_bufs<float>(c), reps, ms_out, bytes_out);
}

}  // namespace lshom
