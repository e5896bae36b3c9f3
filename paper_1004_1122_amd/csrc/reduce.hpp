// Deterministic FP64 block reductions and the CG scalar decisions.
//
// A producing kernel stores one partial per block (plain store).  A consuming
// kernel, launched after it on the same stream, sums those partials in block
// order inside each of its blocks: every block obtains the identical value
// without atomics or fences, and the result does not depend on scheduling.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace lshom {

// Sum over the block (wave64 shuffles, then a fixed tree over the waves);
// the result is returned to every thread.
template <int NT>
__device__ __forceinline__ double block_sum_all(double v) {
  __shared__ double red[NT / 64];
  __shared__ double total;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    total = s;
  }
  __syncthreads();
  return total;
}

// Sum of p[0..n) (stride `step` between entries), identical in every block.
template <int NT>
__device__ __forceinline__ double sum_partials(const double* p, int n, int step = 1) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) acc += p[(long long)i * step];
  return block_sum_all<NT>(acc);
}

// Block partial of a dot product: block sum stored by thread 0.
template <int NT>
__device__ __forceinline__ void store_partial(double v, double* dst) {
  const double s = block_sum_all<NT>(v);
  if (threadIdx.x == 0) *dst = s;
}

// Entry gate of an iteration kernel.  Thread 0 reads the flags once and the
// block follows its decision, so that all waves of a block agree even while
// block 0 of the same kernel is updating the flags.
__device__ __forceinline__ bool gated_out(const DevState* st, int gate) {
  if (gate == GATE_ALWAYS) return false;
  __shared__ int skip;
  if (threadIdx.x == 0) {
    const int done = st->done;
    const int refresh = st->refresh;
    int s;
    if (gate == GATE_ACTIVE) s = done != 0;
    else if (gate == GATE_REFRESH) s = done != 0 || refresh == 0;
    else s = done != 0 || refresh != 0;  // GATE_NO_REFRESH
    skip = s;
  }
  __syncthreads();
  return skip != 0;
}

// Gate of a pass whose flags only earlier launches write (the row pass and the
// forward axis-0 pass): every wave reads the same values, so each decides on
// its own and no block barrier delays the first loads.
__device__ __forceinline__ bool gated_out_stable(const DevState* st, int gate) {
  if (gate == GATE_ALWAYS) return false;
  const int done = st->done;
  const int refresh = st->refresh;
  if (gate == GATE_ACTIVE) return done != 0;
  if (gate == GATE_REFRESH) return done != 0 || refresh == 0;
  return done != 0 || refresh != 0;  // GATE_NO_REFRESH
}

// Thread 0's reading of the entry flags (nonzero: skip the kernel).
__device__ __forceinline__ int gate_flags(const DevState* st, int gate) {
  if (gate == GATE_ALWAYS || threadIdx.x != 0) return 0;
  const int done = st->done;
  const int refresh = st->refresh;
  if (gate == GATE_ACTIVE) return done != 0;
  if (gate == GATE_REFRESH) return done != 0 || refresh == 0;
  return done != 0 || refresh != 0;  // GATE_NO_REFRESH
}

// This thread's share of the sum of p[0..n).
template <int NT>
__device__ __forceinline__ double partial_share(const double* p, int n) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) acc += p[i];
  return acc;
}

// Block sums of NS values together with thread 0's gate decision: one pass of
// barriers, and every wave leaves with the same sums and the same decision.
// Returns true when the block must skip the kernel.
template <int NT, int NS>
__device__ __forceinline__ bool block_sums_gated(double (&v)[NS], int skip0) {
  __shared__ double red[NS][NT / 64];
  __shared__ double total[NS];
  __shared__ int skip;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[s] += __shfl_down(v[s], off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) red[s][threadIdx.x >> 6] = v[s];
  }
  if (threadIdx.x == 0) skip = skip0;
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < NT / 64; ++i) t += red[s][i];
      total[s] = t;
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NS; ++s) v[s] = total[s];
  return skip != 0;
}

// The two termination norms of Sec. 3 for iterate m: eta_r = l0 ||r|| / ||e0||
// (Eq. (22)) from the real-space (r, r), and eta_e (Eq. (21)) from the
// |k|^2-weighted spectral residual sum eq: for an admissible field the
// divergence of the current in Fourier space is k . j_hat = -l0 k . r_hat and
// r_hat is parallel to k, so eta_e = l0 sqrt(eq) / |j_hat(0)| with
// j_hat(0) = jx + |N| L0 E.  (An anisotropic L0 has |k . j_hat| =
// |r_hat| (k . L0 . k) / |k|; with the scaled coordinate and the weight
// k . L0n . k in eq the same formula holds with l0 = tr(L0) / d.)  The lead
// thread records eta_e and, for m >= 0, history entry m.  Returns whether
// eta_e <= tol.
__device__ inline bool equilibrium_test(DevState* st, int m, double rr, double eq, bool lead) {
  const double l0 = st->l0;
  double j2 = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double jc = st->jx[c] + st->nvox * st->l0E[c];
    j2 += jc * jc;
  }
  const double eta_e = l0 * sqrt(eq / j2);
  if (lead) {
    if (m >= 0) {
      st->eta_e_log = eta_e;
      if (st->hist && m < st->hist_len) {
        st->hist[2 * m] = l0 * sqrt(rr / st->b2);
        st->hist[2 * m + 1] = eta_e;
      }
    } else {
      st->eta_e_true = eta_e;
    }
  }
  return eta_e * eta_e <= st->tol2;
}

// The CG direction step (start of iteration k = iter_a): convergence test on
// (r_k, r_k), iteration limit, and beta = (r_k, r_k) / (r_{k-1}, r_{k-1}).
// Mixed precision requests an FP64 refresh instead of stopping.  Returns
// false when the block must not compute the iteration.  Identical decision
// in every block; the one block with lead_block set records it.
// The entry gate is read with the sums: a block it sends back returns false
// without touching the state.
// With eq (plain FP64 CG only) the equilibrium sums of the same producer are
// summed too and the test follows the state's norm.
template <int NT>
__device__ bool cg_direction(DevState* st, const Partials& parts, double inv_n, double* beta_out, int gate,
                             int eq, bool lead_block) {
  const int skip0 = gate_flags(st, gate);
  const int k = st->iter_a;
  double v[3] = {partial_share<NT>(parts.region(k & 1), st->nparts[k & 1]),
                 k > 0 ? partial_share<NT>(parts.region((k + 1) & 1), st->nparts[(k + 1) & 1]) : 0.0,
                 eq ? partial_share<NT>(parts.region(PART_EQ0 + (k & 1)), st->nparts[k & 1]) : 0.0};
  if (block_sums_gated<NT, 3>(v, skip0)) return false;
  const double rr = v[0] * inv_n;
  const double rr_prev = v[1] * inv_n;
  const bool lead = lead_block && threadIdx.x == 0;
  bool stop = false;
  if (st->refresh_every > 0) {
    const int since = k - st->k_ref;
    if (since > 0 && (!isfinite(rr) || rr <= st->tol2b2 || k >= st->max_iter ||
                      since >= st->refresh_every || rr < st->drop2 * st->rr_ref)) {
      if (lead) st->refresh = 1;
      stop = true;
    } else if (!isfinite(rr)) {
      if (lead) {
        st->status = -6;
        st->done = 1;
      }
      stop = true;
    }
  } else {
    const bool eq_ok = eq && equilibrium_test(st, k, rr, v[2], lead);
    if (!isfinite(rr)) {
      if (lead) st->status = -6;
      stop = true;
    } else if ((eq && st->norm == 1) ? eq_ok : rr <= st->tol2b2) {
      stop = true;
    } else if (k >= st->max_iter) {
      if (lead) st->status = -5;
      stop = true;
    }
    if (stop && lead) st->done = 1;
  }
  if (lead) {
    st->iter_u = k;
    st->rr_log = rr;
  }
  *beta_out = (k == 0 || rr_prev == 0.0) ? 0.0 : rr / rr_prev;
  return !stop;
}

// The scalar step of pipelined CG at the start of iteration k = iter_a, from
// gamma_k = (r_k, r_k) (region k & 1) and delta_k = (w_k, r_k) (PQ), both
// reduced by the update that formed r_k and w_k: the stop tests as in
// cg_direction (residual norm only), then beta = gamma_k / gamma_{k-1} and
// alpha = gamma_k / (delta_k - beta gamma_k / alpha_{k-1}) (beta = 0,
// alpha = gamma_k / delta_k at k = 0).  gamma_{k-1} comes from the other
// (r, r) region and alpha_{k-1} from the state slot of parity k - 1, so no
// block reads a value the lead block writes in this launch.  The lead block
// (lead_block) records alpha and beta at parity k for the later passes of
// the iteration.
template <int NT>
__device__ bool pipe_direction(DevState* st, const Partials& parts, double inv_n, int gate, bool lead_block) {
  const int skip0 = gate_flags(st, gate);
  const int k = st->iter_a;
  double v[3] = {partial_share<NT>(parts.region(k & 1), st->nparts[k & 1]),
                 partial_share<NT>(parts.region(PART_PQ), st->nparts_pq),
                 k > 0 ? partial_share<NT>(parts.region((k + 1) & 1), st->nparts[(k + 1) & 1]) : 0.0};
  if (block_sums_gated<NT, 3>(v, skip0)) return false;
  const double gamma = v[0] * inv_n;
  const double delta = v[1] * inv_n;
  const double gamma_prev = v[2] * inv_n;
  const bool lead = lead_block && threadIdx.x == 0;
  double beta = 0.0, alpha = 0.0;
  bool stop = false;
  if (!isfinite(gamma)) {
    if (lead) st->status = -6;
    stop = true;
  } else if (gamma <= st->tol2b2) {
    stop = true;
  } else if (k >= st->max_iter) {
    if (lead) st->status = -5;
    stop = true;
  } else {
    if (k > 0) {
      beta = gamma / gamma_prev;
      alpha = gamma / (delta - beta * gamma / st->pipe_alpha[(k + 1) & 1]);
    } else {
      alpha = gamma / delta;
    }
    if (!(alpha > 0.0) || !isfinite(alpha)) {
      if (lead) {
        st->status = -6;
        st->pq_log = delta;
      }
      stop = true;
    }
  }
  if (lead) {
    if (stop) st->done = 1;
    st->iter_u = k;
    st->rr_log = gamma;
    st->pipe_alpha[k & 1] = alpha;
    st->pipe_beta[k & 1] = beta;
  }
  return !stop;
}

}  // namespace lshom
