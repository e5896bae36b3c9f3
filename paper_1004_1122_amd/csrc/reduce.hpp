// Deterministic FP64 grid reductions for the CG inner products.
//
// Each block reduces its values with wave64 shuffles and a fixed tree over
// the block's waves, stores one partial per block, and counts its arrival.
// The last block to arrive sums the partials in block order (fixed, so the
// result does not depend on scheduling) and applies the CG scalar update.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace lshom {

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i];
  }
  return s;  // valid in thread 0 only
}

__device__ __forceinline__ double load_acquire_f64(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_f64(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The CG scalar step taken by the last block (thread 0) once the grid-wide
// sums s[0..nv) are known.
__device__ inline void finalize_state(DevState* st, int fin, const double* s, int nv, double inv_n) {
  switch (fin) {
    case FIN_ALPHA: {
      const double pq = s[0];
      st->pq = pq;
      if (!(pq > 0.0) || !isfinite(pq)) {
        st->status = -6;
        st->done = 1;
      } else {
        st->alpha = st->rr / pq;
      }
      break;
    }
    case FIN_RR_INIT: {
      const double rr = s[0];
      st->rr = rr;
      st->rr0 = rr;
      st->rr_ref = rr;
      st->beta = 0.0;
      st->iter = 0;
      if (!isfinite(rr)) {
        st->status = -6;
        st->done = 1;
      } else if (rr <= st->tol2b2) {
        st->done = 1;
      }
      break;
    }
    case FIN_UPDATE: {
      const double rr_new = s[0];
      const double rr_old = st->rr;
      st->iter += 1;
      st->rr = rr_new;
      st->beta = rr_new / rr_old;
      if (st->refresh_every > 0) {
        // mixed precision: the FP32 recursion only proposes; convergence is
        // decided on the FP64 true residual of the refresh
        st->applies32 += 1;
        st->since_refresh += 1;
        const bool want = (st->since_refresh >= st->refresh_every) ||
                          (rr_new < st->drop2 * st->rr_ref) || (rr_new <= st->tol2b2) ||
                          (st->iter >= st->max_iter) || !isfinite(rr_new);
        st->refresh = want ? 1 : 0;
      } else {
        st->applies64 += 1;
        if (!isfinite(rr_new)) {
          st->status = -6;
          st->done = 1;
        } else if (rr_new <= st->tol2b2) {
          st->done = 1;
        } else if (st->iter >= st->max_iter) {
          st->status = -5;
          st->done = 1;
        }
      }
      break;
    }
    case FIN_RR_TRUE:
      st->rr_true = s[0];
      break;
    case FIN_LEFF:
      for (int i = 0; i < nv; ++i) st->leff[i] = s[i] * inv_n;
      break;
    case FIN_AUX:
      st->dot_aux = s[0];
      break;
    case FIN_REFRESH: {
      // true residual of the FP64 iterate replaces the recursive one
      const double rr = s[0];
      st->rr_true = rr;
      st->n_refresh += 1;
      st->since_refresh = 0;
      st->applies64 += 1;
      st->rr = rr;
      st->rr_ref = rr;
      if (!isfinite(rr)) {
        st->status = -6;
        st->done = 1;
      } else if (rr <= st->tol2b2) {
        st->done = 1;
      } else if (st->iter >= st->max_iter) {
        st->status = -5;
        st->done = 1;
      }
      break;
    }
    case FIN_CLEAR_REFRESH:
      st->refresh = 0;
      break;
    default:
      break;
  }
}

// Grid reduction of nv (<= 3) values with last-block finalisation.  `vals`
// are this thread's contributions.  All threads of all blocks must call it.
template <int NT>
__device__ void grid_reduce_finalize(const double* vals, int nv, double* partials, DevState* st,
                                     int fin, double inv_n) {
  __shared__ double red[NT / 64];
  __shared__ double sums[4];
  __shared__ int is_last;
  double bs[4];
  for (int i = 0; i < nv; ++i) bs[i] = block_sum<NT>(vals[i], red);
  if (threadIdx.x == 0) {
    for (int i = 0; i < nv; ++i) store_f64(&partials[(size_t)blockIdx.x * nv + i], bs[i]);
    __threadfence();
    const unsigned prev = atomicAdd(&st->counter, 1u);
    is_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  for (int i = 0; i < nv; ++i) {
    double acc = 0.0;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += NT)
      acc += load_acquire_f64(&partials[(size_t)b * nv + i]);
    const double tot = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) sums[i] = tot;
  }
  if (threadIdx.x == 0) {
    double s[4];
    for (int i = 0; i < nv; ++i) s[i] = sums[i];
    if (fin != FIN_LEFF) {
      for (int i = 0; i < nv; ++i) s[i] *= inv_n;
    }
    finalize_state(st, fin, s, nv, inv_n);
    __hip_atomic_store(&st->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
  }
}

// True when a gated kernel must return at entry.
__device__ __forceinline__ bool gated_out(const DevState* st, int gate) {
  if (gate == GATE_ALWAYS) return false;
  const int done = st->done;
  if (gate == GATE_ACTIVE) return done != 0;
  if (gate == GATE_REFRESH) return done != 0 || st->refresh == 0;
  return done != 0 || st->refresh != 0;  // GATE_NO_REFRESH
}

}  // namespace lshom
