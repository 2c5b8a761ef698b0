// Deterministic FP64 block and grid reductions with a last-block finisher.
//
// Each workgroup reduces its kRedSlots partial sums with wave64 shuffles and
// an LDS pass over the 4 waves in a fixed order, writes them to
// red.part[block], and bumps a counter.  The workgroup that finishes last
// sums all partials in block order (fixed, so the result does not depend on
// scheduling), hands the totals to the task's finisher and resets the
// counter for the next launch.  This keeps CG scalars (alpha, beta, norms,
// convergence flags) on the device with no host round trip.
#pragma once

#include "pfem_internal.h"

namespace pfem {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// On return thread 0 holds the block totals in v.
__device__ __forceinline__ void block_sum(double (&v)[kRedSlots], double* sm) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kRedSlots; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kRedSlots; ++k) sm[wave * kRedSlots + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kRedSlots; ++k) {
      double s = 0.0;
      for (int w = 0; w < kThreads / 64; ++w) s += sm[w * kRedSlots + k];
      v[k] = s;
    }
  }
}

__device__ __forceinline__ void run_finisher(const Task* tp, const double (&s)[kRedSlots]) {
  Scalars* sc = tp->sc;
  switch (tp->finisher) {
    case FIN_STORE:   // two values, so two reductions can share one Scalars.red
      tp->red.out[0] = s[0];
      tp->red.out[1] = s[1];
      break;
    case FIN_PQ: {
      sc->pq = s[0];
      if (!(s[0] > 0.0)) {
        sc->state = 3;  // breakdown / negative curvature
      } else {
        sc->alpha = sc->rz / s[0];
      }
      break;
    }
    case FIN_RZ: {
      const double rz = s[0], rr = s[1];
      sc->beta = rz / sc->rz;
      sc->rz = rz;
      sc->rr = rr;
      sc->rho = sqrt(rr) / sc->den;
      sc->k += 1;
      sc->total_k += 1;
      if (tp->hist != nullptr && sc->hist_len < sc->hist_cap)
        tp->hist[sc->hist_len++] = sc->rho;
      if (!(rr == rr) || !(rz == rz))
        sc->state = 3;
      else if (rr <= sc->target2)
        sc->state = 1;
      else if (!(rz > 0.0))
        sc->state = 3;
      else if (sc->k >= sc->kmax)
        sc->state = 2;
      break;
    }
    case FIN_INIT: {
      const double rz = s[0], rr = s[1];
      sc->rz = rz;
      sc->rr = rr;
      sc->bnorm = sqrt(rr);
      sc->rho = sqrt(rr) / sc->den;
      sc->k = 0;
      if (tp->hist != nullptr && sc->hist_len == 0 && sc->hist_cap > 0)
        tp->hist[sc->hist_len++] = sc->rho;
      if (rr <= sc->target2)
        sc->state = 1;
      else if (!(rz > 0.0) || !(rr == rr))
        sc->state = 3;
      else if (sc->kmax <= 0)
        sc->state = 2;
      else
        sc->state = 0;
      break;
    }
    default:
      break;
  }
}

// Reduce v over the task's `nblk` workgroups; the last one runs the finisher.
__device__ __forceinline__ void reduce_finish(const Task* tp, int blk, int nblk,
                                              double (&v)[kRedSlots]) {
  __shared__ double sm[kRedSlots * (kThreads / 64)];
  __shared__ int is_last;
  if (tp->red.part == nullptr) return;
  block_sum(v, sm);
  if (threadIdx.x == 0) {
    double* pp = tp->red.part + (size_t)blk * kRedSlots;
#pragma unroll
    for (int k = 0; k < kRedSlots; ++k)
      __hip_atomic_store(pp + k, v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned prev = atomicAdd(tp->red.counter, 1u);
    is_last = (prev == (unsigned)(nblk - 1));
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double s[kRedSlots];
#pragma unroll
  for (int k = 0; k < kRedSlots; ++k) s[k] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kThreads) {
#pragma unroll
    for (int k = 0; k < kRedSlots; ++k)
      s[k] += __hip_atomic_load(tp->red.part + (size_t)b * kRedSlots + k,
                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  block_sum(s, sm);
  if (threadIdx.x == 0) {
    run_finisher(tp, s);
    __threadfence();
    __hip_atomic_store(tp->red.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace pfem
