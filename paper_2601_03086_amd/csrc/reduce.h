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

// One DPP move of a double (two 32-bit halves); CTRL is the DPP control.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wave, in every lane, in a fixed order:
// within each row of 16 lanes by data-parallel-primitive moves (quad
// exchanges 1 and 2, then the half-row and row mirrors), then the four row
// sums through scalar lane reads.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);   // row_half_mirror
  v += dpp_move<0x140>(v);   // row_mirror
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
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
