#include "plan.hpp"

#include <cmath>

namespace lshom {

bool fft_size_ok(int64_t n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5, 7, 11, 13, 17})
    while (n % p == 0) n /= p;
  return n == 1;
}

// Per-stage divisors of the stage loop: n / radix and the product of the
// radices already applied.
static void finish_plan(FftPlan* p) {
  int ns = 1;
  for (int st = 0; st < kMaxStages; ++st) {
    if (st < p->nstages && p->radix[st] >= 1) {
      p->nr[st] = make_fastdiv((uint32_t)(p->n / p->radix[st]));
      p->ns[st] = make_fastdiv((uint32_t)ns);
      ns *= p->radix[st];
    } else {
      p->nr[st] = make_fastdiv(1);
      p->ns[st] = make_fastdiv(1);
    }
  }
}

FftPlan default_plan(int n) {
  FftPlan p{};
  p.n = n;
  p.nstages = 0;
  int rest = n;
  const int order[] = {9, 8, 7, 5, 6, 4, 3, 2, 17, 13, 11};
  while (rest > 1 && p.nstages < kMaxStages) {
    for (int r : order) {
      if (rest % r == 0) {
        p.radix[p.nstages++] = r;
        rest /= r;
        break;
      }
    }
  }
  if (p.nstages == 0) {  // n == 1
    p.radix[0] = 1;
  }
  finish_plan(&p);
  return p;
}

bool make_plan(int n, const int* radices, int nstages, FftPlan* plan) {
  if (nstages < 1 || nstages > kMaxStages) return false;
  long long prod = 1;
  for (int i = 0; i < nstages; ++i) {
    const int r = radices[i];
    if (r < 2 || (r > 9 && !is_wide_prime(r))) return false;
    prod *= r;
  }
  if (prod != n) return false;
  *plan = FftPlan{};
  plan->n = n;
  plan->nstages = nstages;
  for (int i = 0; i < nstages; ++i) plan->radix[i] = radices[i];
  finish_plan(plan);
  return true;
}

void twiddles(int n, std::vector<double>* re_im) {
  re_im->assign(2 * (size_t)n, 0.0);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int m = 0; m < n; ++m) {
    // long double carries 64 mantissa bits: the rounded double is within
    // about half an ulp of exp(-2 pi i m / n)
    const long double a = two_pi * (long double)m / (long double)n;
    (*re_im)[2 * m] = (double)std::cos(a);
    (*re_im)[2 * m + 1] = (double)(-std::sin(a));
  }
}

static long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

constexpr int kMaxThreads = 256;

PassShape default_shape(int d, const int64_t* N, const FftPlan* plans, int elem_bytes,
                        size_t lds_budget, long long min_blocks, bool transposed, int n_phases,
                        bool allow_split) {
  PassShape s{2, 1, 1, 0, 0, 0};
  const int last = d - 1;
  const int n_last = (int)N[last];
  const long long h = n_last / 2 + 1;
  long long nrows = 1;
  for (int a = 0; a < last; ++a) nrows *= N[a];

  // row pass: even row counts; in the transposed layout each global access
  // covers rows_per_block contiguous elements, so aim for 128-byte segments
  // (whole cache lines) with one component per block
  {
    const int cap = plan_batch_cap(plans[last], kMaxThreads);
    s.row_split = (transposed && allow_split) ? 1 : 0;
    const int comps = s.row_split ? 1 : d;
    const int target = transposed ? (128 / elem_bytes < 2 ? 2 : 128 / elem_bytes) : 64;
    int best = 2;
    for (int r = 2; r <= target; r += 2) {
      if ((long long)comps * (r / 2) * n_last > cap) break;
      if (row_lds_bytes(n_last, r, comps, elem_bytes, n_phases, nullptr) > lds_budget) break;
      best = r;
      if (!transposed && (long long)comps * (r / 2) * n_last >= 2048) break;
    }
    while (best > 2 && ceil_div(nrows, best) < min_blocks) best -= 2;
    s.rows_per_block = best;
  }
  // strided passes: contiguous columns need no tile (transposed); in the
  // natural layout a tile of `c` columns makes c * elem_bytes-byte segments
  auto pick_tile = [&](int L, long long inner, long long outer, const FftPlan& pl) {
    if (transposed) return 1;
    const int cap = plan_batch_cap(pl, kMaxThreads);
    int best = 1;
    for (int c = 1; c <= 16; c *= 2) {
      if ((long long)d * c * L > cap) break;
      if (col_lds_bytes(L, c, d, elem_bytes, nullptr) > lds_budget) break;
      if (c > inner) break;
      best = c;
      if (c * elem_bytes >= 64) break;
    }
    while (best > 1 && outer * ceil_div(inner, best) < min_blocks) best /= 2;
    return best;
  };
  long long inner0 = h;
  for (int a = 1; a < last; ++a) inner0 *= N[a];
  s.tile0 = pick_tile((int)N[0], inner0, 1, plans[0]);
  if (d == 3) s.tile1 = pick_tile((int)N[1], h, N[0], plans[1]);
  return s;
}

bool shape_fits(int d, const int64_t* N, const FftPlan* plans, const PassShape& s, int elem_bytes,
                size_t lds_budget, int n_phases) {
  const int last = d - 1;
  const int n_last = (int)N[last];
  if (s.rows_per_block < 2 || (s.rows_per_block & 1)) return false;
  if (s.tile0 < 1 || s.tile1 < 1) return false;
  if (s.row_split != 0 && s.row_split != 1) return false;
  auto nt_ok = [](int t) { return t == 0 || t == 128 || t == kMaxThreads; };
  if (!nt_ok(s.threads_row) || !nt_ok(s.threads_col)) return false;
  // a forced 128-thread block must still hold its batch
  auto cap_ok = [&](int t, long long points, const FftPlan& pl) { return t != 128 || points <= plan_batch_cap(pl, 128); };
  if (!cap_ok(s.threads_row, (long long)(s.row_split ? 1 : d) * (s.rows_per_block / 2) * n_last, plans[last])) return false;
  if (!cap_ok(s.threads_col, (long long)d * s.tile0 * N[0], plans[0])) return false;
  if (d == 3 && !cap_ok(s.threads_col, (long long)d * s.tile1 * N[1], plans[1])) return false;
  {
    const int comps = s.row_split ? 1 : d;
    const int npairs = comps * (s.rows_per_block / 2);
    if ((long long)npairs * n_last > plan_batch_cap(plans[last], kMaxThreads)) return false;
    if (row_lds_bytes(n_last, s.rows_per_block, comps, elem_bytes, n_phases, nullptr) > lds_budget)
      return false;
  }
  if ((long long)d * s.tile0 * N[0] > plan_batch_cap(plans[0], kMaxThreads)) return false;
  if (col_lds_bytes((int)N[0], s.tile0, d, elem_bytes, nullptr) > lds_budget) return false;
  if (d == 3) {
    if ((long long)d * s.tile1 * N[1] > plan_batch_cap(plans[1], kMaxThreads)) return false;
    if (col_lds_bytes((int)N[1], s.tile1, d, elem_bytes, nullptr) > lds_budget) return false;
  }
  return true;
}

}  // namespace lshom
