// Solve drivers: queue the pass kernels of the operator apply (Sec. 2.2,
// Eq. (16)) and of conjugate gradients (Sec. 2.3; Saad's Algorithm 6.18 as
// named in Sec. 3) on the context stream, in captured HIP graph blocks.
// A group advances one or many problems of the same grid with the same
// launches (grid dimension y = problem).
#include <algorithm>
#include <cmath>
#include <cstring>

#include <mutex>

#include "ctx.hpp"

namespace lshom {

lshom_status fail(lshom_ctx* c, lshom_status s, const std::string& msg) {
  if (c) {
    std::lock_guard<std::mutex> lock(c->err_mutex);
    c->err = msg;
  }
  return s;
}

void drop_graphs(std::map<std::pair<int, int>, hipGraphExec_t>& cache) {
  for (auto& kv : cache) (void)hipGraphExecDestroy(kv.second);
  cache.clear();
}

void drop_batch_graphs(lshom_ctx* c) {
  for (auto& kv : c->batch_graphs) drop_graphs(kv.second);
  c->batch_graphs.clear();
}

namespace {

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

long long inner0_of(const Group& g) {
  long long inner = g.h;
  for (int t = 1; t < g.d - 1; ++t) inner *= g.N[t];
  return inner;
}

}  // namespace

size_t lds_limit_of(const Group& g) { return g.ctx ? g.ctx->lds_limit : kLdsLimit; }

PassShape default_shape_within(int d, const int64_t* N, const FftPlan* plans, int elem_bytes, size_t limit,
                               bool transposed, int n_phases, bool allow_split, bool* fits) {
  const size_t pref = std::min(limit, kLdsPreferred);
  PassShape s = default_shape(d, N, plans, elem_bytes, pref, kMinBlocks, transposed, n_phases, allow_split);
  if (shape_fits(d, N, plans, s, elem_bytes, pref, n_phases)) {
    *fits = true;
    return s;
  }
  s = default_shape(d, N, plans, elem_bytes, limit, kMinBlocks, transposed, n_phases, allow_split);
  *fits = shape_fits(d, N, plans, s, elem_bytes, limit, n_phases);
  return s;
}

lshom_status group_setup(Group& g, int d, const int64_t* N, int n_phases_in, bool tensor) {
  const int n_phases = n_phases_in * (tensor ? d * (d + 1) / 2 : 1);  // table entries
  g.tensor = tensor;
  g.n_phase_ids = n_phases_in;
  g.d = d;
  g.nvox = 1;
  for (int a = 0; a < 3; ++a) g.N[a] = a < d ? N[a] : 1;
  for (int a = 0; a < d; ++a) g.nvox *= N[a];
  g.h = (int)(N[d - 1] / 2 + 1);
  g.nrows = g.nvox / N[d - 1];
  g.nhalf = g.nrows * g.h;
  g.w3ok = d == 3 && !tensor && wave_fft_length(N[0]) && wave_fft_length(N[1]) && wave_fft_length(N[2]);
  g.w3 = false;
  g.nhp = g.w3ok ? w3_entries(N[0], N[1], N[2]) : 0;
  g.nvec = std::max(g.nhalf, g.nhp);
  // in-kernel index arithmetic is 32-bit
  if (g.nvox >= (1ll << 31)) return LSHOM_ERR_UNSUPPORTED;
  g.transposed = (d == 2);
  g.n_phases = n_phases;
  for (int a = 0; a < d; ++a) g.plan64[a] = g.plan32[a] = default_plan((int)N[a]);
  bool fit64 = false, fit32 = false;
  g.shape64 = default_shape_within(d, g.N, g.plan64, (int)sizeof(cx<double>), lds_limit_of(g), g.transposed,
                                   n_phases, !tensor, &fit64);
  g.shape32 = default_shape_within(d, g.N, g.plan32, (int)sizeof(cx<float>), lds_limit_of(g), g.transposed,
                                   n_phases, !tensor, &fit32);
  if (!fit64 || !fit32) return LSHOM_ERR_UNSUPPORTED;
  if (g.ctx) {
    for (int prec = 0; prec < 2; ++prec) {
      auto it = g.ctx->schedules.find(SchedKey(d, g.N[0], g.N[1], g.N[2], prec));
      if (it != g.ctx->schedules.end() && schedule_fits(g, it->second, prec)) apply_schedule(g, it->second, prec);
      // tail schedules are kept under precision + 2
      auto tt = g.ctx->schedules.find(SchedKey(d, g.N[0], g.N[1], g.N[2], prec + 2));
      if (tt != g.ctx->schedules.end() && schedule_fits(g, tt->second, prec) && tt->second.tail_rows > 0) {
        g.tail_sched[prec] = tt->second;
        g.has_tail[prec] = true;
        g.tail_rows = std::max(g.tail_rows, tt->second.tail_rows);
      }
    }
  }
  return LSHOM_OK;
}

bool schedule_fits(const Group& g, const Schedule& s, int precision) {
  if (g.tensor && s.shape.row_split) return false;
  for (int a = 0; a < g.d; ++a) {
    if (s.plan[a].n != g.N[a]) return false;
    FftPlan chk;
    if (!make_plan((int)g.N[a], s.plan[a].radix, s.plan[a].nstages, &chk)) return false;
  }
  const int es = precision == LSHOM_PRECISION_FP64 ? (int)sizeof(cx<double>) : (int)sizeof(cx<float>);
  return shape_fits(g.d, g.N, s.plan, s.shape, es, lds_limit_of(g), g.n_phases);
}

void apply_schedule(Group& g, const Schedule& s, int precision) {
  FftPlan* pl = precision == LSHOM_PRECISION_FP64 ? g.plan64 : g.plan32;
  for (int a = 0; a < g.d; ++a) pl[a] = s.plan[a];
  (precision == LSHOM_PRECISION_FP64 ? g.shape64 : g.shape32) = s.shape;
}

Schedule current_schedule(const Group& g, int precision) {
  Schedule s;
  const FftPlan* pl = precision == LSHOM_PRECISION_FP64 ? g.plan64 : g.plan32;
  for (int a = 0; a < 3; ++a) s.plan[a] = a < g.d ? pl[a] : FftPlan{};
  s.shape = precision == LSHOM_PRECISION_FP64 ? g.shape64 : g.shape32;
  return s;
}

Layout compute_layout(const Group& g, bool with32, bool with_bicg) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const long long np = g.nprob;
  L.off_state = take(sizeof(DevState) * np);
  L.off_scratch = take(256);
  L.off_tab = take(sizeof(ProbEntry) * np);
  L.off_live = take(sizeof(int) * np);
  // partial sums: one slot (three in AUX) per block of the widest launch
  // any schedule can make (two rows per row-pass block, tiles of one)
  (void)with32;
  long long maxb = kUpdateBlocks;
  maxb = std::max(maxb, (long long)g.d * ceil_div(g.nrows, 2));
  maxb = std::max(maxb, inner0_of(g));
  if (g.d == 3) maxb = std::max(maxb, g.N[0] * (long long)g.h);
  L.part_stride = 3 * maxb;
  L.pstride = kPartRegions * L.part_stride;
  L.off_partials = take((size_t)L.pstride * np * sizeof(double));
  L.off_cond64 = take((size_t)kCondStride * np * sizeof(double));
  L.off_cond32 = take((size_t)kCondStride * np * sizeof(float));
  for (int a = 0; a < g.d; ++a) {
    L.off_tw64[a] = take((size_t)g.N[a] * sizeof(cx<double>));
    L.off_tw32[a] = take((size_t)g.N[a] * sizeof(cx<float>));
  }
  const size_t v64 = (size_t)g.nvec * np * sizeof(cx<double>);
  const size_t v32 = (size_t)g.nvec * np * sizeof(cx<float>);
  for (int i = 0; i < 4; ++i) L.off_v64[i] = take(v64);
  for (int a = 0; a < g.d; ++a) L.off_w64[a] = take(v64);
  if (g.w3ok)
    for (int a = 0; a < g.d; ++a) L.off_g64[a] = take(v64);
  L.has32 = with32;
  if (with32) {
    for (int i = 0; i < 4; ++i) L.off_v32[i] = take(v32);
    for (int a = 0; a < g.d; ++a) L.off_w32[a] = take(v32);
    if (g.w3ok)
      for (int a = 0; a < g.d; ++a) L.off_g32[a] = take(v32);
  }
  L.has_bicg = with_bicg;
  if (with_bicg)
    for (int i = 0; i < 7; ++i) L.off_bicg[i] = take((size_t)g.d * g.nvox * np * sizeof(double));
  L.total = off;
  return L;
}

// Work that must not overlap another context's stream capture (host-staged
// uploads, events on the caller's stream) and the captures themselves are
// serialised process-wide.
std::mutex& setup_mutex() {
  static std::mutex m;
  return m;
}

namespace {

DevState* dev_state(Group& g) { return reinterpret_cast<DevState*>(g.ws + g.lay.off_state); }

Partials dev_parts(Group& g) {
  Partials p;
  p.base = reinterpret_cast<double*>(g.ws + g.lay.off_partials);
  p.stride = g.lay.part_stride;
  return p;
}

Batch batch_of(Group& g) {
  Batch b{};
  b.nprob = g.live_rows > 0 ? g.live_rows : g.nprob;
  b.vstride = g.nvec;
  b.pstride = g.lay.pstride;
  b.tab = g.batched ? reinterpret_cast<const ProbEntry*>(g.ws + g.lay.off_tab) : nullptr;
  b.live = g.live_rows > 0 ? reinterpret_cast<const int*>(g.ws + g.lay.off_live) : nullptr;
  return b;
}

template <typename T>
Bufs<T> get_bufs(Group& g);

template <>
Bufs<double> get_bufs<double>(Group& g) {
  Bufs<double> b{};
  for (int i = 0; i < 4; ++i) b.v[i] = reinterpret_cast<cx<double>*>(g.ws + g.lay.off_v64[i]);
  for (int a = 0; a < g.d; ++a) {
    b.w[a] = reinterpret_cast<cx<double>*>(g.ws + g.lay.off_w64[a]);
    b.gl[a] = g.w3ok ? reinterpret_cast<cx<double>*>(g.ws + g.lay.off_g64[a]) : nullptr;
    b.tw[a] = reinterpret_cast<const cx<double>*>(g.ws + g.lay.off_tw64[a]);
  }
  b.cond = reinterpret_cast<const double*>(g.ws + g.lay.off_cond64);
  b.shape = g.shape64;
  for (int a = 0; a < 3; ++a) b.plan[a] = g.plan64[a];
  return b;
}

template <>
Bufs<float> get_bufs<float>(Group& g) {
  Bufs<float> b{};
  for (int i = 0; i < 4; ++i) b.v[i] = reinterpret_cast<cx<float>*>(g.ws + g.lay.off_v32[i]);
  for (int a = 0; a < g.d; ++a) {
    b.w[a] = reinterpret_cast<cx<float>*>(g.ws + g.lay.off_w32[a]);
    b.gl[a] = g.w3ok ? reinterpret_cast<cx<float>*>(g.ws + g.lay.off_g32[a]) : nullptr;
    b.tw[a] = reinterpret_cast<const cx<float>*>(g.ws + g.lay.off_tw32[a]);
  }
  b.cond = reinterpret_cast<const float*>(g.ws + g.lay.off_cond32);
  b.shape = g.shape32;
  for (int a = 0; a < 3; ++a) b.plan[a] = g.plan32[a];
  return b;
}

hipStream_t stream_of(Group& g) { return g.stream ? g.stream : g.ctx->stream; }

// Launch f; inside the CG loop with pass timing on, between two events.
template <typename F>
hipError_t timed_launch(Group& g, int kind, F&& f) {
  if (!g.timer || !g.timer->on || !g.in_cg) return f();
  PassTimer& t = *g.timer;
  const size_t i = t.kinds.size();
  while (t.pool.size() < 2 * i + 2) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    t.pool.push_back(ev);
  }
  hipError_t e = hipEventRecord(t.pool[2 * i], stream_of(g));
  if (e != hipSuccess) return e;
  if ((e = f()) != hipSuccess) return e;
  if ((e = hipEventRecord(t.pool[2 * i + 1], stream_of(g))) != hipSuccess) return e;
  t.kinds.push_back(kind);
  return hipSuccess;
}

// Fold the pending launch timings (after a stream synchronisation) and the
// bytes of the problem-iterations advanced since `prev_iters`.
hipError_t harvest_timing(Group& g, long long advanced) {
  if (!g.timer || !g.timer->on) return hipSuccess;
  PassTimer& t = *g.timer;
  bool seen[LSHOM_PASS_COUNT] = {};
  for (size_t i = 0; i < t.kinds.size(); ++i) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, t.pool[2 * i], t.pool[2 * i + 1]);
    if (e != hipSuccess) return e;
    t.ms[t.kinds[i]] += ms;
    t.launches[t.kinds[i]] += 1;
    seen[t.kinds[i]] = true;
  }
  for (int k = 0; k < LSHOM_PASS_COUNT; ++k)
    if (seen[k]) t.bytes[k] += (double)advanced * t.unit_bytes[k];
  t.kinds.clear();
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Pass argument builders
// ---------------------------------------------------------------------------

template <typename T>
ColArgs<T> col0_args(Group& g, const Bufs<T>& b) {
  ColArgs<T> a{};
  a.L = (int)g.N[0];
  a.inner = inner0_of(g);
  a.outer = 1;
  if (g.transposed) {
    a.sl = 1;
    a.sii = a.L;
  } else {
    a.sl = a.inner;
    a.sii = 1;
  }
  a.tile = b.shape.tile0;
  a.tiles_per_outer = (int)ceil_div(a.inner, a.tile);
  a.d = g.d;
  col_lds_bytes(a.L, a.tile, a.d, (int)sizeof(cx<T>), &a.ss);
  a.fd_L = make_fastdiv((uint32_t)a.L);
  a.fd_C = make_fastdiv((uint32_t)a.tile);
  a.fd_h = make_fastdiv((uint32_t)g.h);
  a.nt = b.shape.threads_col;
  for (int t = 0; t < g.d; ++t) {
    a.comp[t] = b.w[t];
    a.nd[t] = (int)g.N[t];
  }
  for (int t = 0; t < kMaxDim; ++t) a.cinv[t] = g.cell_inv[t];
  a.dims = g.d;
  a.h = g.h;
  a.plan = b.plan[0];
  a.tw = b.tw[0];
  a.st = dev_state(g);
  a.parts = dev_parts(g);
  a.inv_n = 1.0 / (double)g.nvox;
  a.gate = GATE_ACTIVE;
  a.l0 = g.l0;
  a.aniso = g.aniso ? 1 : 0;
  for (int i = 0; i < 6; ++i) a.L0n[i] = g.L0n[i];
  a.bt = batch_of(g);
  return a;
}

template <typename T>
ColArgs<T> col1_args(Group& g, const Bufs<T>& b, int dir) {
  ColArgs<T> a{};
  a.L = (int)g.N[1];
  a.inner = g.h;
  a.outer = g.N[0];
  a.sl = a.inner;
  a.sii = 1;
  a.tile = b.shape.tile1;
  a.tiles_per_outer = (int)ceil_div(a.inner, a.tile);
  a.d = g.d;
  col_lds_bytes(a.L, a.tile, a.d, (int)sizeof(cx<T>), &a.ss);
  a.fd_L = make_fastdiv((uint32_t)a.L);
  a.fd_C = make_fastdiv((uint32_t)a.tile);
  a.fd_h = make_fastdiv((uint32_t)g.h);
  a.nt = b.shape.threads_col;
  for (int t = 0; t < g.d; ++t) {
    a.comp[t] = b.w[t];
    a.nd[t] = (int)g.N[t];
  }
  for (int t = 0; t < kMaxDim; ++t) a.cinv[t] = g.cell_inv[t];
  a.dims = g.d;
  a.h = g.h;
  a.mode = COL_PLAIN;
  a.dir = dir;
  a.plan = b.plan[1];
  a.tw = b.tw[1];
  a.st = dev_state(g);
  a.parts = dev_parts(g);
  a.inv_n = 1.0 / (double)g.nvox;
  a.gate = GATE_ACTIVE;
  a.l0 = g.l0;
  a.bt = batch_of(g);
  return a;
}

template <typename T>
RowArgs<T> row_args(Group& g, const Bufs<T>& b) {
  RowArgs<T> a{};
  const int last = g.d - 1;
  a.n = (int)g.N[last];
  a.h = g.h;
  a.nrows = g.nrows;
  a.rows_per_block = b.shape.rows_per_block;
  a.d = g.d;
  a.split = b.shape.row_split;
  a.nt = b.shape.threads_row;
  const int comps = a.split ? 1 : a.d;
  row_lds_bytes(a.n, a.rows_per_block, comps, (int)sizeof(cx<T>), g.n_phases, &a.ss);
  a.fd_n = make_fastdiv((uint32_t)a.n);
  a.fd_np = make_fastdiv((uint32_t)(comps * (a.rows_per_block / 2)));
  a.fd_h = make_fastdiv((uint32_t)a.h);
  a.fd_half = make_fastdiv((uint32_t)(a.rows_per_block / 2));
  if (g.transposed) {
    a.rs_row = 1;
    a.rs_k = g.nrows;
    a.row_fast = 1;
  } else {
    a.rs_row = g.h;
    a.rs_k = 1;
    a.row_fast = 0;
  }
  for (int t = 0; t < g.d; ++t) a.spec[t] = b.w[t];
  a.phase = g.phase;
  a.cond = b.cond;
  a.n_phases = g.n_phases;
  a.tensor = g.tensor ? 1 : 0;
  a.aniso = g.aniso ? 1 : 0;
  for (int i = 0; i < 6; ++i) a.L0u[i] = (T)g.L0u[i];
  a.l0 = (T)g.l0;
  a.inv_n = (T)(1.0 / (double)g.nvox);
  a.plan = b.plan[last];
  a.tw = b.tw[last];
  a.st = dev_state(g);
  a.parts = dev_parts(g);
  a.gate = GATE_ACTIVE;
  a.bt = batch_of(g);
  return a;
}

long long klast_div_of(const Group& g) { return g.transposed ? g.N[0] : 1; }

// Entries per problem the elementwise kernels of the current solve cover.
long long vec_entries(const Group& g) { return g.w3 ? g.nhp : g.nhalf; }

template <typename T>
W3Args<T> w3_args(Group& g, const Bufs<T>& b) {
  W3Args<T> a{};
  a.N0 = (int)g.N[0];
  a.N1 = (int)g.N[1];
  a.N2 = (int)g.N[2];
  a.h = g.h;
  a.G = w3_groups(g.h);
  a.nhp = g.nhp;
  for (int t = 0; t < kMaxDim; ++t) {
    a.gl[t] = b.gl[t];
    a.hl[t] = b.w[t];
    a.tw[t] = b.tw[t];
    a.cinv[t] = g.cell_inv[t];
  }
  a.phase = g.phase;
  a.cond = b.cond;
  a.n_phases = g.n_phases;
  a.l0 = (T)g.l0;
  a.l0d = g.l0;
  a.inv_n = (T)(1.0 / (double)g.nvox);
  a.inv_nd = 1.0 / (double)g.nvox;
  a.st = dev_state(g);
  a.parts = dev_parts(g);
  a.gate = GATE_ACTIVE;
  a.bt = batch_of(g);
  return a;
}

template <typename T>
long long col0_block_count(Group& g, const Bufs<T>& b) {
  if (g.w3) return w3_blocks(W3_FWD0, (int)g.N[0], (int)g.N[1], (int)g.N[2]);
  return col_blocks(col0_args(g, b));
}

hipError_t enq_finalize(Group& g, int mode, long long n, int gate, int eq = 0) {
  FinArgs f{};
  f.eq = eq;
  f.st = dev_state(g);
  f.parts = dev_parts(g);
  f.mode = mode;
  f.n = (int)n;
  f.d = g.d;
  f.inv_n = 1.0 / (double)g.nvox;
  f.gate = gate;
  f.bt = batch_of(g);
  return launch_finalize(f, stream_of(g));
}

template <typename T>
UpdArgs<T> upd_args(Group& g, const Bufs<T>& b) {
  UpdArgs<T> u{};
  u.n = vec_entries(g);
  u.w3 = g.w3 ? 1 : 0;
  u.fd_w3n0 = make_fastdiv((uint32_t)g.N[0]);
  u.w3g = w3_groups(g.h);
  u.h = g.h;
  u.n_last = (int)g.N[g.d - 1];
  u.klast_div = klast_div_of(g);
  u.fd_kd = make_fastdiv((uint32_t)u.klast_div);
  u.fd_h = make_fastdiv((uint32_t)g.h);
  u.x = b.v[0];
  u.r = b.v[1];
  u.p = b.v[2];
  u.q = b.v[3];
  u.st = dev_state(g);
  u.parts = dev_parts(g);
  u.inv_n = 1.0 / (double)g.nvox;
  u.gate = GATE_ACTIVE;
  u.bt = batch_of(g);
  u.eq = g.eq ? 1 : 0;
  u.dims = g.d;
  for (int t = 0; t < 3; ++t) u.nd[t] = (int)g.N[t];
  u.fd_n1 = make_fastdiv((uint32_t)g.N[1]);
  for (int t = 0; t < kMaxDim; ++t) u.cinv[t] = g.cell_inv[t];
  u.aniso = g.aniso ? 1 : 0;
  for (int i = 0; i < 6; ++i) u.L0n[i] = g.L0n[i];
  return u;
}

// The row pass of r: the wave pass when the solve uses them, else r itself.
template <typename T>
hipError_t launch_row_pass(Group& g, const Bufs<T>& b, const RowArgs<T>& r) {
  if (!g.w3) return launch_row(r, stream_of(g));
  W3Args<T> a = w3_args(g, b);
  a.mode = r.mode;
  a.flags = r.flags;
  for (int t = 0; t < kMaxDim; ++t) {
    a.real_in[t] = r.real_in[t];
    a.real_out[t] = r.real_out[t];
    a.real_add[t] = r.real_add[t];
    a.E[t] = r.E[t];
  }
  a.gate = r.gate;
  return launch_w3(W3_ROW, a, stream_of(g));
}

template <typename T>
long long row_block_count(Group& g, const RowArgs<T>& r) {
  if (g.w3) return w3_blocks(W3_ROW, (int)g.N[0], (int)g.N[1], (int)g.N[2]);
  return row_blocks(r);
}

// ---------------------------------------------------------------------------
// Operator sequences (see the pass kernels for the algebra)
// ---------------------------------------------------------------------------

// After a producer of blocks partials in dot_region (and eq_region): fold
// them when the producer is wide and the region's consumers read its count
// in every block.
hipError_t enq_fold_if_wide(Group& g, long long blocks, int dot, int dot_region, int eq_region, int gate) {
  if (!dot || blocks <= kFoldAbove || (dot_region != PART_RR0 && dot_region != PART_PQ)) return hipSuccess;
  FoldArgs f{};
  f.st = dev_state(g);
  f.parts = dev_parts(g);
  f.region = dot_region;
  f.eq_region = eq_region;
  f.gate = gate;
  f.bt = batch_of(g);
  return launch_fold_partials(f, stream_of(g));
}

// Forward half: [3-D axis-1 forward], axis-0 forward + projection.
// out = coef_base * base + coef_s * [1 / l0] * (-i khat) . tau_hat
template <typename T>
hipError_t enq_forward_project(Group& g, const Bufs<T>& b, cx<T>* out, const cx<T>* base,
                               T coef_base, T coef_s, int s_inv_l0, int dot, int dot_region, int gate,
                               int eq = 0, int pipe = 0) {
  hipError_t e;
  if (g.w3) {
    W3Args<T> m = w3_args(g, b);
    m.dir = -1;
    m.gate = gate;
    if ((e = timed_launch(g, LSHOM_PASS_AXIS1_FORWARD, [&] { return launch_w3(W3_COL1, m, stream_of(g)); })) !=
        hipSuccess)
      return e;
    W3Args<T> f = w3_args(g, b);
    f.out = out;
    f.base = base;
    f.coef_base = coef_base;
    f.coef_s = coef_s;
    f.s_inv_l0 = s_inv_l0;
    f.dot = dot;
    f.dot_region = dot_region;
    f.gate = gate;
    if ((e = timed_launch(g, LSHOM_PASS_AXIS0_FORWARD, [&] { return launch_w3(W3_FWD0, f, stream_of(g)); })) !=
        hipSuccess)
      return e;
    return enq_fold_if_wide(g, w3_blocks(W3_FWD0, (int)g.N[0], (int)g.N[1], (int)g.N[2]), dot, dot_region, -1,
                            gate);
  }
  if (g.d == 3) {
    ColArgs<T> m = col1_args(g, b, -1);
    m.gate = gate;
    if ((e = timed_launch(g, LSHOM_PASS_AXIS1_FORWARD, [&] { return launch_col(m, stream_of(g)); })) != hipSuccess)
      return e;
  }
  ColArgs<T> a = col0_args(g, b);
  a.mode = COL_FWD_PROJ;
  a.out = out;
  a.base = base;
  a.coef_base = coef_base;
  a.coef_s = coef_s;
  a.s_inv_l0 = s_inv_l0;
  a.dot = dot;
  a.dot_region = dot_region;
  a.eq = eq;
  a.eq_region = PART_EQ0;
  a.gate = gate;
  a.pipe = pipe;
  if ((e = timed_launch(g, LSHOM_PASS_AXIS0_FORWARD, [&] { return launch_col(a, stream_of(g)); })) != hipSuccess)
    return e;
  if (pipe) return hipSuccess;
  return enq_fold_if_wide(g, col_blocks(a), dot, dot_region,
                          (eq && dot != 1 && dot_region == PART_RR0) ? PART_EQ0 : -1, gate);
}

// The CG update of the wave passes leaves x += alpha p to the next direction
// step (the axis-0 inverse pass), which reads p anyway.
bool cg_defers_x(const Group& g) { return g.w3 && !g.eq; }

// Inverse half: axis-0 inverse from the scalar c (or the CG direction step
// p = r + beta p), [3-D axis-1 inverse].
template <typename T>
hipError_t enq_inverse_from_c(Group& g, const Bufs<T>& b, const cx<T>* c_in, cx<T>* p_io,
                              const cx<T>* r_in, int gate, int eq = 0) {
  hipError_t e;
  if (g.w3) {
    W3Args<T> a = w3_args(g, b);
    a.c_in = c_in;
    a.p_io = p_io;
    a.r_in = r_in;
    a.cg_step = p_io != nullptr;
    // the CG loop's update leaves x to this step (one read of p fewer)
    a.x_io = (a.cg_step && g.in_cg && cg_defers_x(g)) ? b.v[0] : nullptr;
    a.gate = gate;
    if ((e = timed_launch(g, LSHOM_PASS_AXIS0_INVERSE, [&] { return launch_w3(W3_INV0, a, stream_of(g)); })) !=
        hipSuccess)
      return e;
    W3Args<T> m = w3_args(g, b);
    m.dir = +1;
    m.clear_xpend = a.x_io != nullptr;
    m.gate = gate;
    return timed_launch(g, LSHOM_PASS_AXIS1_INVERSE, [&] { return launch_w3(W3_COL1, m, stream_of(g)); });
  }
  ColArgs<T> a = col0_args(g, b);
  a.mode = COL_INV_C;
  a.c_in = c_in;
  a.p_io = p_io;
  a.r_in = r_in;
  a.cg_step = p_io != nullptr;
  a.eq = eq;
  a.gate = gate;
  if ((e = timed_launch(g, LSHOM_PASS_AXIS0_INVERSE, [&] { return launch_col(a, stream_of(g)); })) != hipSuccess)
    return e;
  if (g.d == 3) {
    ColArgs<T> m = col1_args(g, b, +1);
    m.gate = gate;
    if ((e = timed_launch(g, LSHOM_PASS_AXIS1_INVERSE, [&] { return launch_col(m, stream_of(g)); })) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// out = coef_base * base + coef_s * (1/l0) (-i khat) . F[dL (E + u(c_in))]
template <typename T>
hipError_t enq_apply_spec(Group& g, const Bufs<T>& b, const cx<T>* c_in, cx<T>* p_io,
                          const cx<T>* r_in, const double* E, cx<T>* out, const cx<T>* base,
                          T coef_base, T coef_s, int dot, int dot_region, int gate, int eq = 0) {
  hipError_t e;
  if ((e = enq_inverse_from_c(g, b, c_in, p_io, r_in, gate, eq)) != hipSuccess) return e;
  RowArgs<T> r = row_args(g, b);
  r.mode = ROW_FUSED;
  for (int t = 0; t < g.d; ++t) r.E[t] = E ? (T)E[t] : T(0);
  if (!E) r.flags |= ROWF_STATE_E;
  r.gate = gate;
  if ((e = timed_launch(g, LSHOM_PASS_ROW, [&] { return launch_row_pass(g, b, r); })) != hipSuccess) return e;
  return enq_forward_project(g, b, out, base, coef_base, coef_s, 1, dot, dot_region, gate, eq);
}

// One CG iteration in the spectral coordinate:
//   direction step (p = r + beta p, or stop), q = p + (1/l0) P dL u(p) with
//   (p, q), then alpha = (r, r) / (p, q), x += alpha p, r -= alpha q, (r, r).
template <typename T>
hipError_t enq_cg_iteration(Group& g, const Bufs<T>& b, int gate) {
  hipError_t e;
  cx<T>* r = b.v[1];
  cx<T>* p = b.v[2];
  cx<T>* q = b.v[3];
  static const double kZero[3] = {0.0, 0.0, 0.0};
  g.in_cg = true;
  e = enq_apply_spec<T>(g, b, nullptr, p, r, kZero, q, p, T(1), T(1), 1, PART_PQ, gate, g.eq ? 1 : 0);
  if (e == hipSuccess) {
    UpdArgs<T> u = upd_args(g, b);
    u.gate = gate;
    u.defer_x = cg_defers_x(g) ? 1 : 0;
    e = timed_launch(g, LSHOM_PASS_UPDATE, [&] { return launch_update(u, stream_of(g)); });
  }
  g.in_cg = false;
  return e;
}

// The x step of the last update, for the problems of a CG loop that stopped
// after an update (wave passes defer it to the next direction step).
template <typename T>
hipError_t enq_flush_x(Group& g, const Bufs<T>& b) {
  if (!cg_defers_x(g)) return hipSuccess;
  return launch_flush_x(upd_args(g, b), stream_of(g));
}

// Residual of the spectral iterate x for the load E:
// r = -(x + (1/l0) P dL (E + u(x))).
template <typename T>
hipError_t enq_true_residual(Group& g, const Bufs<T>& b, const cx<T>* x, const double* E,
                             cx<T>* out, int dot_region, int gate, int eq = 0) {
  return enq_apply_spec<T>(g, b, x, nullptr, nullptr, E, out, x, T(-1), T(-1), 2, dot_region, gate, eq);
}

// One step of the basic scheme (Sec. 2.3, Eq. (18)) in the spectral
// coordinate: x <- -(1/l0) P dL (E + u(x)), i.e. e^(m+1) = e0 - B e^(m); the
// step x_new - x (the residual of e^(m)) is reduced for the tests.
hipError_t enq_ffth_iteration(Group& g, const Bufs<double>& b, int gate) {
  hipError_t e;
  cx<double>* x = b.v[0];
  g.in_cg = true;
  e = enq_apply_spec<double>(g, b, x, nullptr, nullptr, nullptr, x, x, 0.0, -1.0, 3, PART_RR0, gate,
                             g.eq ? 1 : 0);
  g.in_cg = false;
  if (e != hipSuccess) return e;
  return enq_finalize(g, FZ_FFTH, col0_block_count(g, b), gate, g.eq ? 1 : 0);
}

// r0 for x0 = E: r0 = -(1/l0) P dL E.
template <typename T>
hipError_t enq_residual_of_E(Group& g, const Bufs<T>& b, const double* E, cx<T>* out, int dot_region,
                             int eq = 0) {
  hipError_t e;
  RowArgs<T> r = row_args(g, b);
  r.mode = ROW_FWD;
  r.flags = ROWF_DL | ROWF_CONST_E;
  for (int t = 0; t < g.d; ++t) r.E[t] = E ? (T)E[t] : T(0);
  if (!E) r.flags |= ROWF_STATE_E;
  r.gate = GATE_ALWAYS;
  if ((e = launch_row_pass(g, b, r)) != hipSuccess) return e;
  return enq_forward_project<T>(g, b, out, nullptr, T(0), T(-1), 1, 2, dot_region, GATE_ALWAYS, eq);
}

// Real FP64 field v (d x |N|) -> spectral coordinate of P v (green: of
// Gamma0 v, with dL: of Gamma0 dL v).
hipError_t enq_project_real(Group& g, const Bufs<double>& b, const double* v, bool with_dl, bool green,
                            cx<double>* out, int gate = GATE_ALWAYS) {
  hipError_t e;
  RowArgs<double> r = row_args(g, b);
  r.mode = ROW_FWD;
  r.flags = with_dl ? ROWF_DL : 0;
  for (int t = 0; t < g.d; ++t) r.real_in[t] = v + (size_t)t * g.nvox;
  r.gate = gate;
  if ((e = launch_row_pass(g, b, r)) != hipSuccess) return e;
  return enq_forward_project<double>(g, b, out, nullptr, 0.0, 1.0, green ? 1 : 0, 0, PART_AUX, gate);
}

// Real field out = add + E + u(x); with leff, <lambda out> into state.leff.
// dl_out: out = add + (L - L0) (E + u(x)).
hipError_t enq_field_out(Group& g, const Bufs<double>& b, const cx<double>* x, const double* E,
                         const double* add, double* out, bool leff, bool dl_out = false,
                         int gate = GATE_ALWAYS) {
  hipError_t e;
  if ((e = enq_inverse_from_c<double>(g, b, x, nullptr, nullptr, gate)) != hipSuccess) return e;
  RowArgs<double> r = row_args(g, b);
  r.mode = ROW_INV;
  r.flags = (add ? ROWF_ADD : 0) | (leff ? ROWF_LEFF : 0) | (dl_out ? ROWF_DL_OUT : 0);
  if (!E) r.flags |= ROWF_STATE_E;
  for (int t = 0; t < g.d; ++t) {
    r.E[t] = E ? E[t] : 0.0;
    r.real_out[t] = out ? out + (size_t)t * g.nvox : nullptr;
    r.real_add[t] = add ? add + (size_t)t * g.nvox : nullptr;
  }
  r.gate = gate;
  if ((e = launch_row_pass(g, b, r)) != hipSuccess) return e;
  if (leff) return enq_finalize(g, FZ_LEFF, row_block_count(g, r), gate);
  return hipSuccess;
}

const double kNoE[3] = {0.0, 0.0, 0.0};

// q = (I + B) v = v + Gamma0 dL v on real nodal fields (Sec. 2.2, Eq. (16)).
hipError_t enq_apply_A_real(Group& g, const Bufs<double>& b, const double* v, double* q, int gate) {
  hipError_t e = enq_project_real(g, b, v, true, true, b.v[3], gate);
  if (e != hipSuccess) return e;
  return enq_field_out(g, b, b.v[3], kNoE, v, q, false, false, gate);
}

// q = (I + B)^T v = v + dL Gamma0 v: the same passes in the other order
// (Green operator first, polarisation at the nodes last).
hipError_t enq_apply_AT_real(Group& g, const Bufs<double>& b, const double* v, double* q, int gate) {
  hipError_t e = enq_project_real(g, b, v, false, true, b.v[3], gate);
  if (e != hipSuccess) return e;
  return enq_field_out(g, b, b.v[3], kNoE, v, q, false, true, gate);
}

MixArgs mix_args(Group& g, const Bufs<double>& b64, const Bufs<float>& b32, int gate) {
  MixArgs m{};
  m.n = vec_entries(g);
  m.w3 = g.w3 ? 1 : 0;
  m.fd_w3n0 = make_fastdiv((uint32_t)g.N[0]);
  m.w3g = w3_groups(g.h);
  m.h = g.h;
  m.n_last = (int)g.N[g.d - 1];
  m.klast_div = klast_div_of(g);
  m.fd_kd = make_fastdiv((uint32_t)m.klast_div);
  m.fd_h = make_fastdiv((uint32_t)g.h);
  m.x64 = b64.v[0];
  m.x32 = b32.v[0];
  m.r64 = b64.v[1];
  m.r32 = b32.v[1];
  m.st = dev_state(g);
  m.parts = dev_parts(g);
  m.inv_n = 1.0 / (double)g.nvox;
  m.gate = gate;
  m.bt = batch_of(g);
  return m;
}

// Mixed precision refresh (reliable update): x64 += x32, x32 = 0;
// r64 = b - A64 x64 in FP64; r32 = r64 with its (r, r) partials; the
// finalize step decides convergence on the FP64 value and clears the request.
hipError_t enq_mix_refresh(Group& g, const Bufs<double>& b64, const Bufs<float>& b32,
                           const double* E, int gate) {
  hipError_t e;
  MixArgs m = mix_args(g, b64, b32, gate);
  if ((e = launch_mix_accumulate(m, stream_of(g))) != hipSuccess) return e;
  if ((e = enq_true_residual<double>(g, b64, b64.v[0], E, b64.v[1], PART_AUX, gate)) != hipSuccess)
    return e;
  if ((e = launch_mix_convert(m, stream_of(g))) != hipSuccess) return e;
  return enq_finalize(g, FZ_REFRESH, col0_block_count(g, b64), gate);
}

hipError_t sync_states(Group& g) {
  hipError_t e = hipMemcpyAsync(g.host_states.data(), dev_state(g), sizeof(DevState) * g.nprob,
                                hipMemcpyDeviceToHost, stream_of(g));
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(stream_of(g));
}

bool all_done(const Group& g) {
  for (const DevState& s : g.host_states)
    if (!s.done) return false;
  return true;
}

// Grid rows for n_live unfinished problems out of nprob: the smallest entry
// >= n_live of the ladder nprob, 3/4 nprob, 9/16 nprob, ..., 1.  The ladder
// bounds the number of distinct launch shapes (and captured graphs) by
// about 2.4 log2(nprob); a shape holds at most a third more rows than
// problems left.
int ladder_rows(int nprob, int n_live) {
  int r = nprob;
  for (;;) {
    const int next = std::max(1, (r * 3) / 4);
    if (next >= r || next < n_live) return r;
    r = next;
  }
}

// Run blocks of work until the device reports every problem done.  A block is
// captured once into a HIP graph and replayed (cached per key when the group
// has a cache); with K == 0 it is queued eagerly.  In a batch, the launches
// cover only the unfinished problems once enough have finished: a block then
// starts by listing them on the device, and its graph is cached per row count.
// Iterations for the next block: `per`, or, once the residuals of the live
// problems have fallen over a block, just enough to cover the iterations they
// need at the rate of that block plus one, so that the last block of a solve
// does not queue many launches that would only return at entry (an estimate
// that falls short costs one more block; CG usually speeds up, so it rarely
// does).  Blocks of 8 or more iterations stay per / 2^j (one graph each);
// shorter ones are queued directly.  Falls back to `per` whenever the rate is
// not usable.
int next_block_length(const Group& g, int per, const std::vector<double>& rr_prev,
                      const std::vector<int>& it_prev) {
  int need_max = 0;
  for (int p = 0; p < g.nprob; ++p) {
    const DevState& s = g.host_states[p];
    if (s.done) continue;
    const int di = s.iter_a - it_prev[p];
    if (!(rr_prev[p] > 0.0) || !(s.rr_log > 0.0) || !(s.rr_log < rr_prev[p]) || di <= 0) return per;
    const double rate = std::log(s.rr_log / rr_prev[p]) / di;  // log (r, r) per iteration, < 0
    const double need = s.rr_log > s.tol2b2 ? std::log(s.tol2b2 / s.rr_log) / rate : 0.0;
    if (!std::isfinite(need) || need > per) return per;
    need_max = std::max(need_max, (int)std::ceil(need) + 1);
  }
  if (need_max >= per) return per;
  if (need_max < 8) return std::max(need_max, 1);
  int n = per;
  while (n / 2 >= need_max) n /= 2;
  return n;
}

template <typename F>
lshom_status run_blocks(Group& g, int key, int K, int per, bool adapt, F&& enqueue_block) {
  lshom_ctx* c = g.ctx;
  HIP_TRY(c, sync_states(g));
  // the tail of a batch (few unfinished problems) may run with its own
  // schedules; the group's own ones come back on every exit
  const Schedule main_sched[2] = {current_schedule(g, LSHOM_PRECISION_FP64),
                                  current_schedule(g, LSHOM_PRECISION_MIXED)};
  struct ResetRows {
    Group& g;
    const Schedule* main;
    ~ResetRows() {
      g.live_rows = 0;
      for (int p = 0; p < 2; ++p)
        if (g.has_tail[p]) apply_schedule(g, main[p], p);
    }
  } reset_rows{g, main_sched};
  g.live_rows = 0;
  auto use_schedules_for = [&](int rows) {
    const bool tail = g.tail_rows > 0 && rows <= g.tail_rows;
    for (int p = 0; p < 2; ++p)
      if (g.has_tail[p]) apply_schedule(g, tail ? g.tail_sched[p] : main_sched[p], p);
  };
  int* live_dev = reinterpret_cast<int*>(g.ws + g.lay.off_live);
  auto enqueue = [&](int n) -> hipError_t {
    if (g.live_rows > 0) {
      hipError_t e = launch_compact_live(dev_state(g), g.nprob, g.live_rows, live_dev, stream_of(g));
      if (e != hipSuccess) return e;
    }
    return enqueue_block(n);
  };
  // graphs per (rows, block length): the group's cache, else owned here
  std::map<std::pair<int, int>, hipGraphExec_t> owned;
  struct DropOwned {
    std::map<std::pair<int, int>, hipGraphExec_t>& m;
    ~DropOwned() { drop_graphs(m); }
  } drop_owned{owned};
  hipGraphExec_t ex = nullptr;
  auto get_graph = [&](int n) -> lshom_status {
    ex = nullptr;
    if (K <= 0) return LSHOM_OK;
    const int rows = g.live_rows > 0 ? g.live_rows : g.nprob;
    auto gk = std::make_pair(key + 8 * rows, n);
    auto& cache = g.graph_cache ? *g.graph_cache : owned;
    auto it = cache.find(gk);
    if (it != cache.end()) {
      ex = it->second;
      return LSHOM_OK;
    }
    {
      std::lock_guard<std::mutex> lock(setup_mutex());
      hipGraph_t gr = nullptr;
      HIP_TRY(c, hipStreamBeginCapture(stream_of(g), hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue(n);
      hipError_t e2 = hipStreamEndCapture(stream_of(g), &gr);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return fail(c, LSHOM_ERR_HIP, std::string("graph capture failed: ") +
                                          hipGetErrorString(e != hipSuccess ? e : e2));
      }
      hipError_t e3 = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (e3 != hipSuccess)
        return fail(c, LSHOM_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e3));
      cache.emplace(gk, ex);
    }
    return LSHOM_OK;
  };
  lshom_status st = LSHOM_OK;
  std::vector<double> rr_prev(g.nprob, -1.0);
  std::vector<int> it_prev(g.nprob, 0);
  // the device sets `done` at the latest after max_iter iterations; every
  // block advances an iteration or (mixed precision) a refresh of some live
  // problem, so a block that advances neither means the state stopped
  // advancing
  for (;;) {
    if (all_done(g)) break;
    if (g.nprob > 1) {
      int n_live = 0;
      for (const DevState& s : g.host_states) n_live += s.done == 0;
      const int rows = ladder_rows(g.nprob, n_live);
      const int cur = g.live_rows > 0 ? g.live_rows : g.nprob;
      if (rows < cur) {
        g.live_rows = rows;
        use_schedules_for(rows);
      }
    }
    const int n = adapt ? next_block_length(g, per, rr_prev, it_prev) : per;
    // short final blocks are queued directly (a capture would cost more)
    if (n == per || n >= 8) {
      if ((st = get_graph(n)) != LSHOM_OK) return st;
    } else {
      ex = nullptr;
    }
    long long before = 0, moves_before = 0;
    for (int p = 0; p < g.nprob; ++p) {
      before += g.host_states[p].iter_a;
      moves_before += g.host_states[p].iter_a + g.host_states[p].n_refresh;
      rr_prev[p] = g.host_states[p].rr_log;
      it_prev[p] = g.host_states[p].iter_a;
    }
    hipError_t e = ex ? hipGraphLaunch(ex, stream_of(g)) : enqueue(n);
    if (e == hipSuccess) e = sync_states(g);
    long long after = 0, moves_after = 0;
    if (e == hipSuccess) {
      for (const DevState& s : g.host_states) {
        after += s.iter_a;
        moves_after += s.iter_a + s.n_refresh;
      }
      e = harvest_timing(g, after - before);
    }
    if (e != hipSuccess) {
      st = fail(c, LSHOM_ERR_HIP, std::string("iteration block: ") + hipGetErrorString(e));
      break;
    }
    if (moves_after == moves_before && !all_done(g)) {
      st = fail(c, LSHOM_ERR_HIP, "device CG state stopped advancing");
      break;
    }
  }
  return st;
}

}  // namespace

// ---------------------------------------------------------------------------
// Workspace preparation
// ---------------------------------------------------------------------------

lshom_status prepare_workspace(Group& g, const std::vector<double>& cond, const std::vector<ProbEntry>* tab,
                               const std::vector<const uint8_t*>& phases) {
  lshom_ctx* c = g.ctx;
  const Layout& use = g.lay;
  // uploads are ordered on the group's stream (no legacy-stream copies that
  // could disturb a graph capture of another context); the host staging
  // vectors below outlive them: the guard synchronises on every return path
  std::lock_guard<std::mutex> lock(setup_mutex());
  struct SyncOnExit {
    hipStream_t s;
    ~SyncOnExit() { (void)hipStreamSynchronize(s); }
  };
  std::vector<std::vector<double>> tw64(g.d);
  std::vector<std::vector<float>> tw32(g.d);
  const int np = g.nprob;
  std::vector<DevState> zero(np);
  std::vector<double> c64((size_t)kCondStride * np, 0.0);
  std::vector<float> c32((size_t)kCondStride * np, 0.0f);
  for (int p = 0; p < np; ++p)
    for (int i = 0; i < g.n_phases; ++i) {
      c64[(size_t)p * kCondStride + i] = cond[(size_t)p * g.n_phases + i];
      c32[(size_t)p * kCondStride + i] = (float)cond[(size_t)p * g.n_phases + i];
    }
  HIP_TRY(c, hipMemcpyAsync(g.ws + use.off_cond64, c64.data(), c64.size() * sizeof(double), hipMemcpyHostToDevice, stream_of(g)));
  HIP_TRY(c, hipMemcpyAsync(g.ws + use.off_cond32, c32.data(), c32.size() * sizeof(float), hipMemcpyHostToDevice, stream_of(g)));
  for (int a = 0; a < g.d; ++a) {
    twiddles((int)g.N[a], &tw64[a]);
    tw32[a].resize(tw64[a].size());
    for (size_t i = 0; i < tw64[a].size(); ++i) tw32[a][i] = (float)tw64[a][i];
    HIP_TRY(c, hipMemcpyAsync(g.ws + use.off_tw64[a], tw64[a].data(), tw64[a].size() * sizeof(double),
                              hipMemcpyHostToDevice, stream_of(g)));
    HIP_TRY(c, hipMemcpyAsync(g.ws + use.off_tw32[a], tw32[a].data(), tw32[a].size() * sizeof(float),
                              hipMemcpyHostToDevice, stream_of(g)));
  }
  if (tab)
    HIP_TRY(c, hipMemcpyAsync(g.ws + use.off_tab, tab->data(), tab->size() * sizeof(ProbEntry), hipMemcpyHostToDevice, stream_of(g)));
  SyncOnExit sync_guard{stream_of(g)};
  HIP_TRY(c, hipMemcpyAsync(g.ws + use.off_state, zero.data(), sizeof(DevState) * np, hipMemcpyHostToDevice,
                            stream_of(g)));
  g.host_states.assign(np, DevState{});
  // every phase index must name a conductivity: one maximum per image into
  // the (still unused) partial-sum area, read back with one synchronisation
  unsigned* mx = reinterpret_cast<unsigned*>(g.ws + use.off_partials);
  const size_t nimg = phases.size();
  HIP_TRY(c, hipMemsetAsync(mx, 0, sizeof(unsigned) * nimg, stream_of(g)));
  for (size_t i = 0; i < nimg; ++i) HIP_TRY(c, launch_max_phase(phases[i], g.nvox, mx + i, stream_of(g)));
  std::vector<unsigned> host_max(nimg, 0u);
  HIP_TRY(c, hipMemcpyAsync(host_max.data(), mx, sizeof(unsigned) * nimg, hipMemcpyDeviceToHost, stream_of(g)));
  HIP_TRY(c, hipStreamSynchronize(stream_of(g)));
  for (size_t i = 0; i < nimg; ++i)
    if (host_max[i] >= (unsigned)g.n_phase_ids)
      return fail(c, LSHOM_ERR_INVALID_ARG, "phase image " + std::to_string(i) + " holds an index >= n_phases");
  return LSHOM_OK;
}

// ---------------------------------------------------------------------------
// Solve every problem of a group (plain FP64 or mixed precision)
// ---------------------------------------------------------------------------

lshom_status solve_group(Group& g, const std::vector<DevState>& init, const lshom_solve_opts& o,
                         const double* E_single, const double* x0, double* e_single) {
  lshom_ctx* c = g.ctx;
  const bool mixed = o.precision == LSHOM_PRECISION_MIXED;
  const bool ffth = o.method == LSHOM_METHOD_FFTH;
  // the equilibrium sums ride along the loop when the norm or a history needs
  // them (FP64, odd grids: checked by the caller)
  struct EqReset {
    Group& g;
    ~EqReset() {
      g.eq = false;
      g.w3 = false;
    }
  } eq_reset{g};
  g.eq = !mixed && (o.norm == LSHOM_NORM_EQUILIBRIUM || o.history_dev != nullptr);
  // CG and the basic scheme on a qualifying 3-D grid with an isotropic
  // reference run the wave passes (the equilibrium sums keep the block passes)
  g.w3 = g.w3ok && !g.eq && !g.aniso && !g.tensor;
  bool odd = true;
  for (int a = 0; a < g.d; ++a) odd = odd && (g.N[a] & 1);
  const int eq_final = odd ? 1 : 0;
  const int eq_loop = g.eq ? 1 : 0;
  Bufs<double> b64 = get_bufs<double>(g);
  const long long ncol = col0_block_count(g, b64);
  const long long nall = g.nvec * g.nprob;
  // E of every problem is read from its device state: a captured graph then
  // serves every load case
  (void)E_single;
  const double* E = nullptr;
  cx<double>* x64 = b64.v[0];
  cx<double>* r64 = b64.v[1];
  DevState* init_dev = reinterpret_cast<DevState*>(g.ws + g.lay.off_partials);  // staged, then reused
  // initial scalars: staged through the partials area (overwritten later)
  HIP_TRY(c, hipMemcpyAsync(init_dev, init.data(), sizeof(DevState) * g.nprob, hipMemcpyHostToDevice,
                            stream_of(g)));
  HIP_TRY(c, launch_state_copy(dev_state(g), init_dev, g.nprob, stream_of(g)));
  HIP_TRY(c, launch_fill_zero(x64, nall, stream_of(g)));
  Bufs<float> b32{};
  if (mixed) {
    b32 = get_bufs<float>(g);
    HIP_TRY(c, launch_fill_zero(b32.v[0], nall, stream_of(g)));
    HIP_TRY(c, launch_fill_zero(b32.v[2], nall, stream_of(g)));
  } else {
    HIP_TRY(c, launch_fill_zero(b64.v[2], nall, stream_of(g)));
  }
  const int fin_init = mixed ? FZ_REFRESH_INIT : FZ_CHECK;
  const int init_region = mixed ? PART_AUX : PART_RR0;
  int warm_used = 0;
  g.warm_flags.assign(g.nprob, 0);
  // batched problems bring their warm starts in the problem table (the row
  // pass reads a missing one as zero)
  const bool warm_batch = g.batched && g.warm_any;
  if (x0 || warm_batch) {
    // residual of E for the admissibility test, then of E + P x0
    HIP_TRY(c, (enq_residual_of_E<double>(g, b64, E, r64, PART_AUX)));
    HIP_TRY(c, enq_finalize(g, FZ_AUX, ncol, GATE_ALWAYS));
    HIP_TRY(c, enq_project_real(g, b64, x0, false, false, x64));
    HIP_TRY(c, (enq_true_residual<double>(g, b64, x64, E, r64, init_region, GATE_ALWAYS, eq_loop)));
    HIP_TRY(c, enq_finalize(g, fin_init, mixed ? ncol : 0, GATE_ALWAYS, eq_loop));
    HIP_TRY(c, sync_states(g));
    int rejected = 0;
    for (int p = 0; p < g.nprob; ++p) {
      const DevState& hs = g.host_states[p];
      const double rr = mixed ? hs.rr_true : hs.rr_log;
      const bool has = x0 || g.warm_has[p];
      if (has && std::isfinite(rr) && rr < hs.dot_aux) {
        g.warm_flags[p] = 1;
      } else {
        // start this problem from e = E instead
        HIP_TRY(c, launch_fill_zero(x64 + (long long)p * g.nvec, g.nvec, stream_of(g)));
        rejected += has ? 1 : 0;
      }
    }
    int taken = 0;
    for (int f : g.warm_flags) taken += f;
    warm_used = taken > 0;
    if (warm_used && (rejected > 0 || taken < g.nprob)) {
      // some problems of the batch start from e = E: every residual is
      // formed again from the (partly zeroed) iterates with the initial
      // scalars (the kept warm starts get the same values as before)
      HIP_TRY(c, hipMemcpyAsync(init_dev, init.data(), sizeof(DevState) * g.nprob, hipMemcpyHostToDevice,
                                stream_of(g)));
      HIP_TRY(c, launch_state_copy(dev_state(g), init_dev, g.nprob, stream_of(g)));
      HIP_TRY(c, (enq_true_residual<double>(g, b64, x64, E, r64, init_region, GATE_ALWAYS, eq_loop)));
      HIP_TRY(c, enq_finalize(g, fin_init, mixed ? ncol : 0, GATE_ALWAYS, eq_loop));
    }
  }
  if (!warm_used) {
    // the staged initial states were consumed above only in the warm path;
    // reload them (the partials area is overwritten by the residual)
    HIP_TRY(c, hipMemcpyAsync(init_dev, init.data(), sizeof(DevState) * g.nprob, hipMemcpyHostToDevice,
                              stream_of(g)));
    HIP_TRY(c, launch_state_copy(dev_state(g), init_dev, g.nprob, stream_of(g)));
    // the basic scheme tests each iterate inside its own step
    if (!ffth) {
      HIP_TRY(c, (enq_residual_of_E<double>(g, b64, E, r64, init_region, eq_loop)));
      HIP_TRY(c, enq_finalize(g, fin_init, mixed ? ncol : 0, GATE_ALWAYS, eq_loop));
    }
  }
  if (mixed) HIP_TRY(c, launch_mix_convert(mix_args(g, b64, b32, GATE_ALWAYS), stream_of(g)));
  // (run_blocks starts by reading the states back)
  int max_iter = 0;
  for (const DevState& s : init) max_iter = std::max(max_iter, s.max_iter);
  // with pass timing on, the blocks are queued eagerly (events around each launch)
  PassTimer& tm = c->timer;
  g.timer = tm.on ? &tm : nullptr;
  const int K = tm.on ? 0 : o.graph_block;
  const int per = o.graph_block > 0 ? o.graph_block : 8;
  // block lengths follow the residual only when the residual is the test
  const bool adapt = o.norm == LSHOM_NORM_RESIDUAL;
  if (tm.on) {
    tm.kinds.clear();
    pass_model_bytes(g, o.precision, tm.unit_bytes, ffth);
  }
  lshom_status s;
  // the blocks take the buffers (and launch shapes) current when they are
  // queued: the tail of a batch may switch schedules
  if (ffth) {
    s = run_blocks(g, 3 + eq_loop, K, per, adapt, [&](int n) -> hipError_t {
      const Bufs<double> f64 = get_bufs<double>(g);
      for (int k = 0; k < n; ++k) {
        hipError_t e = enq_ffth_iteration(g, f64, GATE_ACTIVE);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    });
  } else if (!mixed) {
    s = run_blocks(g, 2 * eq_loop, K, per, adapt, [&](int n) -> hipError_t {
      const Bufs<double> f64 = get_bufs<double>(g);
      for (int k = 0; k < n; ++k) {
        hipError_t e = enq_cg_iteration<double>(g, f64, GATE_ACTIVE);
        if (e != hipSuccess) return e;
      }
      return enq_finalize(g, FZ_CHECK, 0, GATE_ACTIVE, eq_loop);
    });
  } else {
    // a refresh may cut a block short: at least one iteration per block is certain
    s = run_blocks(g, 1, K, per, adapt, [&](int n) -> hipError_t {
      const Bufs<double> f64 = get_bufs<double>(g);
      const Bufs<float> f32 = get_bufs<float>(g);
      for (int k = 0; k < n; ++k) {
        hipError_t e = enq_cg_iteration<float>(g, f32, GATE_NO_REFRESH);
        if (e != hipSuccess) return e;
      }
      return enq_mix_refresh(g, f64, f32, E, GATE_REFRESH);
    });
  }
  if (s != LSHOM_OK) return s;
  if (!ffth) {
    if (mixed) HIP_TRY(c, enq_flush_x<float>(g, b32));
    else HIP_TRY(c, enq_flush_x<double>(g, b64));
  }
  // fold what a breakdown left in the FP32 correction (no-op after a refresh)
  if (mixed) HIP_TRY(c, launch_mix_accumulate(mix_args(g, b64, b32, GATE_ALWAYS), stream_of(g)));
  if (o.true_residual) {
    HIP_TRY(c, (enq_true_residual<double>(g, b64, x64, E, b64.v[3], PART_AUX, GATE_ALWAYS, eq_final)));
    HIP_TRY(c, enq_finalize(g, FZ_RR_TRUE, ncol, GATE_ALWAYS, eq_final));
  }
  HIP_TRY(c, enq_field_out(g, b64, x64, E, nullptr, e_single, true));
  HIP_TRY(c, sync_states(g));
  g.warm_used = warm_used;
  return LSHOM_OK;
}

// ---------------------------------------------------------------------------
// One FP64 apply on a real field: q = p + B p (single problem)
// ---------------------------------------------------------------------------

lshom_status apply_real(Group& g, const double* p, double* q) {
  lshom_ctx* c = g.ctx;
  Bufs<double> b = get_bufs<double>(g);
  HIP_TRY(c, enq_project_real(g, b, p, true, true, b.v[3]));
  HIP_TRY(c, enq_field_out(g, b, b.v[3], kNoE, p, q, false));
  HIP_TRY(c, hipStreamSynchronize(stream_of(g)));
  return LSHOM_OK;
}

// ---------------------------------------------------------------------------
// BiCG on the nodal system (Sec. 2.3; Saad's Algorithm 7.3 as cited in Sec. 3)
// ---------------------------------------------------------------------------

lshom_status solve_bicg(Group& g, const DevState& init, const lshom_solve_opts& o, double* e_out) {
  lshom_ctx* c = g.ctx;
  Bufs<double> b = get_bufs<double>(g);
  auto field = [&](int i) { return reinterpret_cast<double*>(g.ws + g.lay.off_bicg[i]); };
  double* x = field(0);
  double* r = field(1);
  double* rs = field(2);
  double* p = field(3);
  double* ps = field(4);
  double* ap = field(5);
  double* atp = field(6);
  BicgArgs v{};
  v.n = g.nvox;
  v.d = g.d;
  v.x = x;
  v.r = r;
  v.rs = rs;
  v.p = p;
  v.ps = ps;
  v.ap = ap;
  v.atp = atp;
  v.phase = g.phase;
  v.cond = b.cond;
  v.tensor = g.tensor ? 1 : 0;
  v.st = dev_state(g);
  v.parts = dev_parts(g);
  v.fd_n = make_fastdiv((uint32_t)g.nvox);
  const long long nb = bicg_blocks(v);
  auto vec = [&](int mode, int gate) {
    BicgArgs a = v;
    a.mode = mode;
    a.gate = gate;
    return launch_bicg(a, stream_of(g));
  };
  // scalar steps over real-field sums (no spectral 1 / |N| factor)
  auto fin = [&](int mode, long long n, int gate, double inv_n) {
    FinArgs f{};
    f.st = dev_state(g);
    f.parts = dev_parts(g);
    f.mode = mode;
    f.n = (int)n;
    f.d = g.d;
    f.inv_n = inv_n;
    f.gate = gate;
    f.bt = batch_of(g);
    return launch_finalize(f, stream_of(g));
  };
  DevState* init_dev = reinterpret_cast<DevState*>(g.ws + g.lay.off_partials);
  HIP_TRY(c, hipMemcpyAsync(init_dev, &init, sizeof(DevState), hipMemcpyHostToDevice, stream_of(g)));
  HIP_TRY(c, launch_state_copy(dev_state(g), init_dev, 1, stream_of(g)));
  HIP_TRY(c, hipStreamSynchronize(stream_of(g)));
  // x0 = E, r0 = b - A x0, r0* = r0 = p0 = p0*
  HIP_TRY(c, vec(BV_FILL_E, GATE_ALWAYS));
  HIP_TRY(c, enq_apply_A_real(g, b, x, ap, GATE_ALWAYS));
  HIP_TRY(c, vec(BV_START, GATE_ALWAYS));
  HIP_TRY(c, fin(FZ_BICG_START, nb, GATE_ALWAYS, 1.0));
  HIP_TRY(c, sync_states(g));
  PassTimer& tm = c->timer;
  g.timer = tm.on ? &tm : nullptr;
  const int K = tm.on ? 0 : o.graph_block;
  const int per = o.graph_block > 0 ? o.graph_block : 8;
  tm.kinds.clear();
  pass_model_bytes(g, LSHOM_PRECISION_FP64, tm.unit_bytes);
  lshom_status s = run_blocks(g, 5, K, per, true, [&](int n) -> hipError_t {
    for (int k = 0; k < n; ++k) {
      hipError_t e;
      if ((e = enq_apply_A_real(g, b, p, ap, GATE_ACTIVE)) != hipSuccess) return e;
      if ((e = enq_apply_AT_real(g, b, ps, atp, GATE_ACTIVE)) != hipSuccess) return e;
      if ((e = vec(BV_DOT_APP, GATE_ACTIVE)) != hipSuccess) return e;
      if ((e = fin(FZ_BICG_ALPHA, nb, GATE_ACTIVE, 1.0)) != hipSuccess) return e;
      if ((e = vec(BV_UPDATE, GATE_ACTIVE)) != hipSuccess) return e;
      if ((e = fin(FZ_BICG_STEP, nb, GATE_ACTIVE, 1.0)) != hipSuccess) return e;
      if ((e = vec(BV_DIRECTION, GATE_ACTIVE)) != hipSuccess) return e;
    }
    return hipSuccess;
  });
  if (s != LSHOM_OK) return s;
  // FP64 true residual of the returned field and <lambda e>
  if (o.true_residual) {
    HIP_TRY(c, enq_apply_A_real(g, b, x, ap, GATE_ALWAYS));
    HIP_TRY(c, vec(BV_RESID, GATE_ALWAYS));
    HIP_TRY(c, fin(FZ_RR_TRUE, nb, GATE_ALWAYS, 1.0));
  }
  HIP_TRY(c, vec(BV_LEFF, GATE_ALWAYS));
  HIP_TRY(c, fin(FZ_LEFF, nb, GATE_ALWAYS, 1.0 / (double)g.nvox));
  if (e_out)
    HIP_TRY(c, hipMemcpyAsync(e_out, x, sizeof(double) * g.d * g.nvox, hipMemcpyDeviceToDevice, stream_of(g)));
  HIP_TRY(c, sync_states(g));
  return LSHOM_OK;
}

// ---------------------------------------------------------------------------
// Pipelined CG (single problem, FP64): the iterates of CG with one reduction
// per iteration.  Spectral vectors x, r, p (the CG slots) and w = A r,
// s = A p, z = A s (the extra-field area).
// ---------------------------------------------------------------------------

// One iteration: the scalar step (alpha, beta, stop) with the inverse pass of
// n = A w, the row pass, z = n + beta z with the forward pass, the update
// (which also reduces (r, r) and (w, r) for the next step).
hipError_t enq_pipe_iteration(Group& g, const Bufs<double>& b, cx<double>* w, cx<double>* s, cx<double>* z,
                              int gate) {
  hipError_t e;
  static const double kZero[3] = {0.0, 0.0, 0.0};
  g.in_cg = true;
  struct InCg {
    Group& g;
    ~InCg() { g.in_cg = false; }
  } in_cg{g};
  ColArgs<double> a = col0_args(g, b);
  a.mode = COL_INV_C;
  a.c_in = w;
  a.pipe = 1;
  a.gate = gate;
  if ((e = timed_launch(g, LSHOM_PASS_AXIS0_INVERSE, [&] { return launch_col(a, stream_of(g)); })) != hipSuccess)
    return e;
  if (g.d == 3) {
    ColArgs<double> m = col1_args(g, b, +1);
    m.gate = gate;
    if ((e = timed_launch(g, LSHOM_PASS_AXIS1_INVERSE, [&] { return launch_col(m, stream_of(g)); })) != hipSuccess)
      return e;
  }
  RowArgs<double> r = row_args(g, b);
  r.mode = ROW_FUSED;
  for (int t = 0; t < g.d; ++t) r.E[t] = kZero[t];
  r.gate = gate;
  if ((e = timed_launch(g, LSHOM_PASS_ROW, [&] { return launch_row_pass(g, b, r); })) != hipSuccess) return e;
  if ((e = enq_forward_project<double>(g, b, z, w, 1.0, 1.0, 1, 0, PART_AUX, gate, 0, 1)) != hipSuccess) return e;
  PipeArgs<double> u{};
  u.n = g.nhalf;
  u.h = g.h;
  u.n_last = (int)g.N[g.d - 1];
  u.klast_div = klast_div_of(g);
  u.fd_kd = make_fastdiv((uint32_t)u.klast_div);
  u.fd_h = make_fastdiv((uint32_t)g.h);
  u.x = b.v[0];
  u.r = b.v[1];
  u.p = b.v[2];
  u.w = w;
  u.s = s;
  u.z = z;
  u.st = dev_state(g);
  u.parts = dev_parts(g);
  u.gate = gate;
  u.bt = batch_of(g);
  return timed_launch(g, LSHOM_PASS_UPDATE, [&] { return launch_pipe_update(u, stream_of(g)); });
}

lshom_status solve_pipecg(Group& g, const DevState& init, const lshom_solve_opts& o, double* e_out) {
  lshom_ctx* c = g.ctx;
  Bufs<double> b = get_bufs<double>(g);
  auto field = [&](int i) { return reinterpret_cast<cx<double>*>(g.ws + g.lay.off_bicg[i]); };
  cx<double>* w = field(0);
  cx<double>* s = field(1);
  cx<double>* z = field(2);
  cx<double>* x = b.v[0];
  cx<double>* r = b.v[1];
  DevState* init_dev = reinterpret_cast<DevState*>(g.ws + g.lay.off_partials);
  HIP_TRY(c, hipMemcpyAsync(init_dev, &init, sizeof(DevState), hipMemcpyHostToDevice, stream_of(g)));
  HIP_TRY(c, launch_state_copy(dev_state(g), init_dev, 1, stream_of(g)));
  HIP_TRY(c, hipStreamSynchronize(stream_of(g)));
  for (cx<double>* v : {x, b.v[2], s, z}) HIP_TRY(c, launch_fill_zero(v, g.nhalf, stream_of(g)));
  // x0 = E: r0 and (r0, r0), the test on it; w0 = A r0 and (w0, r0)
  HIP_TRY(c, (enq_residual_of_E<double>(g, b, nullptr, r, PART_RR0)));
  HIP_TRY(c, enq_finalize(g, FZ_CHECK, 0, GATE_ALWAYS));
  static const double kZero[3] = {0.0, 0.0, 0.0};
  HIP_TRY(c, (enq_apply_spec<double>(g, b, r, nullptr, nullptr, kZero, w, r, 1.0, 1.0, 1, PART_PQ, GATE_ALWAYS)));
  HIP_TRY(c, sync_states(g));
  PassTimer& tm = c->timer;
  g.timer = tm.on ? &tm : nullptr;
  const int K = tm.on ? 0 : o.graph_block;
  const int per = o.graph_block > 0 ? o.graph_block : 8;
  tm.kinds.clear();
  pass_model_bytes(g, LSHOM_PRECISION_FP64, tm.unit_bytes);
  lshom_status st = run_blocks(g, 6, K, per, true, [&](int n) -> hipError_t {
    const Bufs<double> f64 = get_bufs<double>(g);
    for (int k = 0; k < n; ++k) {
      hipError_t e = enq_pipe_iteration(g, f64, w, s, z, GATE_ACTIVE);
      if (e != hipSuccess) return e;
    }
    return enq_finalize(g, FZ_CHECK, 0, GATE_ACTIVE);
  });
  if (st != LSHOM_OK) return st;
  const long long ncol = col0_block_count(g, b);
  if (o.true_residual) {
    HIP_TRY(c, (enq_true_residual<double>(g, b, x, nullptr, b.v[3], PART_AUX, GATE_ALWAYS)));
    HIP_TRY(c, enq_finalize(g, FZ_RR_TRUE, ncol, GATE_ALWAYS));
  }
  HIP_TRY(c, enq_field_out(g, b, x, nullptr, nullptr, e_out, true));
  HIP_TRY(c, sync_states(g));
  g.warm_used = 0;
  return LSHOM_OK;
}

// ---------------------------------------------------------------------------
// Per-kernel timing of one CG iteration's launches
// ---------------------------------------------------------------------------

void pass_model_bytes(const Group& g, int precision, double* out, bool basic_scheme) {
  const double cs = precision == LSHOM_PRECISION_FP64 ? (double)sizeof(cx<double>) : (double)sizeof(cx<float>);
  const double nh = (double)g.nhalf;
  const int d = g.d;
  for (int k = 0; k < LSHOM_PASS_COUNT; ++k) out[k] = 0.0;
  // axis-0 inverse with the direction step: reads r, p; writes p and the d pass components
  out[LSHOM_PASS_AXIS0_INVERSE] = (3.0 + d) * nh * cs;
  if (d == 3) {
    // read and write the d components
    out[LSHOM_PASS_AXIS1_INVERSE] = 2.0 * d * nh * cs;
    out[LSHOM_PASS_AXIS1_FORWARD] = 2.0 * d * nh * cs;
  }
  // reads and writes the d components, reads one phase byte per voxel
  out[LSHOM_PASS_ROW] = 2.0 * d * nh * cs + (double)g.nvox;
  // reads the d components and p; writes q
  out[LSHOM_PASS_AXIS0_FORWARD] = (d + 2.0) * nh * cs;
  // reads x, r, p, q; writes x, r
  out[LSHOM_PASS_UPDATE] = 6.0 * nh * cs;
  if (g.w3) {
    // wave passes: the axis-0 passes carry two fields (xi_1 and xi_2 are
    // applied in the axis-1 and last-axis spectra); x += alpha p moves from
    // the update (reads r, q; writes r) to the direction step (reads x, r, p;
    // writes x, p and the two fields)
    out[LSHOM_PASS_UPDATE] = 3.0 * nh * cs;
    out[LSHOM_PASS_AXIS0_INVERSE] = 7.0 * nh * cs;
    out[LSHOM_PASS_AXIS1_INVERSE] = 5.0 * nh * cs;
    out[LSHOM_PASS_AXIS1_FORWARD] = 5.0 * nh * cs;
    out[LSHOM_PASS_AXIS0_FORWARD] = 4.0 * nh * cs;
  }
  if (basic_scheme) {
    // one apply per step: the axis-0 inverse reads the iterate c and writes
    // the pass fields (two on the wave passes, d on the block passes); no update
    out[LSHOM_PASS_AXIS0_INVERSE] = (1.0 + (g.w3 ? 2.0 : (double)d)) * nh * cs;
    out[LSHOM_PASS_UPDATE] = 0.0;
  }
}

namespace {

template <typename T>
lshom_status time_passes_t(Group& g, const Bufs<T>& b, int reps, double* ms_out, double* bytes_out,
                           unsigned mask) {
  // Real CG iterations (FP64 decisions, no stopping) from the residual of a
  // unit load: every pass consumes the previous pass's output, so the data
  // stay those of a solve; each launch is bracketed by a pair of events.
  (void)mask;
  lshom_ctx* c = g.ctx;
  hipStream_t sm = stream_of(g);
  const long long nall = g.nvec * g.nprob;
  DevState init{};
  init.max_iter = 1 << 30;
  init.tol2b2 = -1.0;
  init.b2 = 1.0;
  init.E[0] = 1.0;
  {
    std::vector<DevState> all(g.nprob, init);
    DevState* staged = reinterpret_cast<DevState*>(g.ws + g.lay.off_partials);
    HIP_TRY(c, hipMemcpyAsync(staged, all.data(), sizeof(DevState) * g.nprob, hipMemcpyHostToDevice, sm));
    HIP_TRY(c, launch_state_copy(dev_state(g), staged, g.nprob, sm));
    HIP_TRY(c, hipStreamSynchronize(sm));
  }
  HIP_TRY(c, launch_fill_zero(b.v[0], nall, sm));
  HIP_TRY(c, launch_fill_zero(b.v[2], nall, sm));
  static const double kUnit[3] = {1.0, 0.0, 0.0};
  HIP_TRY(c, (enq_residual_of_E<T>(g, b, kUnit, b.v[1], PART_RR0)));
  // one untimed iteration, then `reps` timed ones
  HIP_TRY(c, (enq_cg_iteration<T>(g, b, GATE_ALWAYS)));
  PassTimer local;
  local.on = true;
  PassTimer* saved = g.timer;
  g.timer = &local;
  hipError_t err = hipSuccess;
  for (int i = 0; i < reps && err == hipSuccess; ++i) err = enq_cg_iteration<T>(g, b, GATE_ALWAYS);
  if (err == hipSuccess) err = hipStreamSynchronize(sm);
  if (err == hipSuccess) err = harvest_timing(g, 0);
  g.timer = saved;
  if (err != hipSuccess) return fail(c, LSHOM_ERR_HIP, std::string("time_passes: ") + hipGetErrorString(err));
  for (hipEvent_t ev : local.pool) (void)hipEventDestroy(ev);
  double model[LSHOM_PASS_COUNT];
  pass_model_bytes(g, sizeof(T) == sizeof(double) ? LSHOM_PRECISION_FP64 : LSHOM_PRECISION_MIXED, model);
  for (int k = 0; k < LSHOM_PASS_COUNT; ++k) {
    ms_out[k] = local.launches[k] ? local.ms[k] / (double)local.launches[k] : 0.0;
    if (bytes_out) bytes_out[k] = local.launches[k] ? model[k] * g.nprob : 0.0;
  }
  return LSHOM_OK;
}

}  // namespace

lshom_status time_passes(Group& g, int precision, int reps, double* ms_out, double* bytes_out) {
  // the passes a CG solve of this grid runs: the wave passes where they apply
  struct W3Reset {
    Group& g;
    ~W3Reset() { g.w3 = false; }
  } w3_reset{g};
  g.w3 = g.w3ok && !g.aniso && !g.tensor;
  if (precision == LSHOM_PRECISION_FP64)
    return time_passes_t<double>(g, get_bufs<double>(g), reps, ms_out, bytes_out, ~0u);
  return time_passes_t<float>(g, get_bufs<float>(g), reps, ms_out, bytes_out, ~0u);
}

// ---------------------------------------------------------------------------
// Autotuner: each pass kind is tuned on its own (its radix order and launch
// shape change only its own kernels), timing real launches on the group.
// ---------------------------------------------------------------------------

namespace {

// Radix orders to try for an axis: the default greedy schedule, its reverse,
// and the schedules with radix-9 stages split into two radix-3 stages.
std::vector<FftPlan> plan_candidates(int n) {
  std::vector<FftPlan> out;
  auto add = [&](const std::vector<int>& r) {
    FftPlan p;
    if (!make_plan(n, r.data(), (int)r.size(), &p)) return;
    for (const FftPlan& q : out)
      if (q.nstages == p.nstages && std::equal(q.radix, q.radix + q.nstages, p.radix)) return;
    out.push_back(p);
  };
  FftPlan d = default_plan(n);
  std::vector<int> base(d.radix, d.radix + d.nstages);
  add(base);
  std::vector<int> rev(base.rbegin(), base.rend());
  add(rev);
  std::vector<int> split;
  for (int r : base) {
    if (r == 9) {
      split.push_back(3);
      split.push_back(3);
    } else {
      split.push_back(r);
    }
  }
  add(split);
  // one radix-9 split (at the front)
  std::vector<int> one;
  bool done = false;
  for (int r : base) {
    if (r == 9 && !done) {
      one.push_back(3);
      one.push_back(3);
      done = true;
    } else {
      one.push_back(r);
    }
  }
  add(one);
  if (out.size() > 5) out.resize(5);
  return out;
}

template <typename T>
double time_mask(Group& g, int precision, int reps, unsigned mask, lshom_status* st) {
  double ms[LSHOM_PASS_COUNT];
  *st = time_passes_t<T>(g, get_bufs<T>(g), reps, ms, nullptr, mask);
  double t = 0.0;
  for (int k = 0; k < LSHOM_PASS_COUNT; ++k)
    if (mask & (1u << k)) t += ms[k];
  (void)precision;
  return t;
}

}  // namespace

lshom_status autotune_tail(Group& g, int precision, int reps, int rows, Schedule* best) {
  lshom_ctx* c = g.ctx;
  if (rows < 1 || rows > g.nprob) return fail(c, LSHOM_ERR_INVALID_ARG, "tail rows out of range");
  std::vector<int> live(rows);
  for (int i = 0; i < rows; ++i) live[i] = i;
  {
    std::lock_guard<std::mutex> lock(setup_mutex());
    HIP_TRY(c, hipMemcpyAsync(g.ws + g.lay.off_live, live.data(), sizeof(int) * rows, hipMemcpyHostToDevice,
                              stream_of(g)));
    HIP_TRY(c, hipStreamSynchronize(stream_of(g)));
  }
  g.live_rows = rows;
  lshom_status s = autotune_group(g, precision, reps, best);
  g.live_rows = 0;
  best->tail_rows = rows;
  return s;
}

lshom_status autotune_group(Group& g, int precision, int reps, Schedule* best) {
  const bool f64 = precision == LSHOM_PRECISION_FP64;
  Schedule cur = current_schedule(g, precision);
  const int last = g.d - 1;
  lshom_status st = LSHOM_OK;
  auto time_of = [&](const Schedule& s, unsigned mask) -> double {
    apply_schedule(g, s, precision);
    return f64 ? time_mask<double>(g, precision, reps, mask, &st) : time_mask<float>(g, precision, reps, mask, &st);
  };
  // row pass: radix order of the last axis x rows per block
  {
    const unsigned mask = 1u << LSHOM_PASS_ROW;
    double best_t = 1e300;
    Schedule bs = cur;
    for (const FftPlan& pl : plan_candidates((int)g.N[last])) {
      for (int split = 0; split <= 1; ++split) {
        for (int r = 2; r <= 32; r += 2) {
         for (int nt : {0, 256}) {
          Schedule s = cur;
          s.plan[last] = pl;
          s.shape.rows_per_block = r;
          s.shape.row_split = split;
          s.shape.threads_row = nt;
          if (!schedule_fits(g, s, precision)) continue;
          const double t = time_of(s, mask);
          if (st != LSHOM_OK) return st;
          if (t < best_t) {
            best_t = t;
            bs = s;
          }
         }
        }
      }
    }
    cur.plan[last] = bs.plan[last];
    cur.shape.rows_per_block = bs.shape.rows_per_block;
    cur.shape.row_split = bs.shape.row_split;
    cur.shape.threads_row = bs.shape.threads_row;
  }
  // axis-0 passes (inverse with the direction step, forward with the projection)
  if (last != 0) {
    const unsigned mask = (1u << LSHOM_PASS_AXIS0_INVERSE) | (1u << LSHOM_PASS_AXIS0_FORWARD);
    double best_t = 1e300;
    Schedule bs = cur;
    for (const FftPlan& pl : plan_candidates((int)g.N[0])) {
      for (int t0 = 1; t0 <= 16; t0 *= 2) {
        for (int nt : {0, 256}) {
          Schedule s = cur;
          s.plan[0] = pl;
          s.shape.tile0 = t0;
          s.shape.threads_col = nt;
          if (!schedule_fits(g, s, precision)) continue;
          const double t = time_of(s, mask);
          if (st != LSHOM_OK) return st;
          if (t < best_t) {
            best_t = t;
            bs = s;
          }
        }
      }
    }
    cur.plan[0] = bs.plan[0];
    cur.shape.tile0 = bs.shape.tile0;
    cur.shape.threads_col = bs.shape.threads_col;
  }
  // axis-1 passes (3-D)
  if (g.d == 3) {
    const unsigned mask = (1u << LSHOM_PASS_AXIS1_INVERSE) | (1u << LSHOM_PASS_AXIS1_FORWARD);
    double best_t = 1e300;
    Schedule bs = cur;
    for (const FftPlan& pl : plan_candidates((int)g.N[1])) {
      for (int t1 = 1; t1 <= 16; t1 *= 2) {
        Schedule s = cur;
        s.plan[1] = pl;
        s.shape.tile1 = t1;
        if (!schedule_fits(g, s, precision)) continue;
        const double t = time_of(s, mask);
        if (st != LSHOM_OK) return st;
        if (t < best_t) {
          best_t = t;
          bs = s;
        }
      }
    }
    cur.plan[1] = bs.plan[1];
    cur.shape.tile1 = bs.shape.tile1;
  }
  cur.ms_per_iter = time_of(cur, ~0u);
  if (st != LSHOM_OK) return st;
  *best = cur;
  return LSHOM_OK;
}

}  // namespace lshom
