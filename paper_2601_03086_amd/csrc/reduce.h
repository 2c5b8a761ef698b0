// Deterministic FP64 block reductions without inter-workgroup waits.
//
// A producing kernel reduces its per-thread sums inside each workgroup
// (wave64 shuffles, then the 4 waves in a fixed order through LDS) and
// stores one partial per slot and block.  The consuming kernel -- the next
// launch on the stream -- sums the partials of the slots it needs in block
// order, every workgroup redundantly (the partials are a few KB and sit in
// L2).  Kernel boundaries order the two, so no fence, atomic counter or
// "last block" election is needed, and the result is the same on every run.
#pragma once

#include "pfem_internal.h"

namespace pfem {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of v over the workgroup (NT threads), returned to every thread.
template <int NS, int NT = kThreads>
__device__ __forceinline__ void block_sum_all(double (&v)[NS]) {
  __shared__ double sm[NS * (NT / 64)];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NS; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();   // previous users of sm are done
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) sm[wave * NS + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += sm[w * NS + k];
    v[k] = s;
  }
}

// Store this workgroup's partials of slots [k0, k1).  A kernel must never
// store a slot that other workgroups of the same launch are still reading.
template <int NT = kThreads>
__device__ __forceinline__ void write_partials(const RedDev& red, int nb, int blk,
                                               double (&v)[kRedSlots], int k0, int k1) {
  if (red.part == nullptr) return;
  block_sum_all<kRedSlots, NT>(v);
  if (threadIdx.x == 0) {
    for (int k = k0; k < k1; ++k) stg(red.part + (size_t)k * nb + blk, v[k]);
  }
}

// Totals of slots k0 and k1 over all blocks (fixed order), in every thread.
__device__ __forceinline__ void sum_slots2(const double* part, int nb, int k0, int k1,
                                           double& s0, double& s1) {
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += kThreads) {
    v[0] += ldg(part + (size_t)k0 * nb + b);
    v[1] += ldg(part + (size_t)k1 * nb + b);
  }
  block_sum_all<2>(v);
  s0 = v[0];
  s1 = v[1];
}

// Totals of slots 0, 1, 2 over all blocks (fixed order), in every thread.
template <int NT = kThreads>
__device__ __forceinline__ void sum_slots3(const double* part, int nb, double& s0,
                                           double& s1, double& s2) {
  double v[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += NT) {
    v[0] += ldg(part + b);
    v[1] += ldg(part + (size_t)nb + b);
    v[2] += ldg(part + (size_t)2 * nb + b);
  }
  block_sum_all<3, NT>(v);
  s0 = v[0];
  s1 = v[1];
  s2 = v[2];
}

}  // namespace pfem
