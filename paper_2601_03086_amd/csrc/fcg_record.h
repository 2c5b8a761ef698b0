// Fused PCG per-node records and the point step shared by the element
// kernel (which evaluates it at gathered nodes) and the start-up kernels.
#pragma once

#include "pfem_internal.h"

namespace pfem {

// Per-node record of the fused PCG: {r, w, s, M^-1}, 4 * D values.
template <int D, typename T>
__device__ __forceinline__ void load_record(const T* __restrict__ rec, int n, T (&o)[4 * D]) {
  if constexpr (sizeof(T) == 4) {
    const pf4* q = reinterpret_cast<const pf4*>(rec);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const pf4 t = ldx(q, (uint32_t)(n * D + k));
      o[4 * k] = t.x;
      o[4 * k + 1] = t.y;
      o[4 * k + 2] = t.z;
      o[4 * k + 3] = t.w;
    }
  } else {
    const pd2* q = reinterpret_cast<const pd2*>(rec);
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
      const pd2 t = ldx(q, (uint32_t)(n * 2 * D + k));
      o[2 * k] = t.x;
      o[2 * k + 1] = t.y;
    }
  }
}

template <int D, typename T>
__device__ __forceinline__ void store_record(T* __restrict__ rec, int n, const T (&o)[4 * D]) {
  if constexpr (sizeof(T) == 4) {
    pf4* q = reinterpret_cast<pf4*>(rec + (size_t)n * 4 * D);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      pf4 t;
      t.x = o[4 * k];
      t.y = o[4 * k + 1];
      t.z = o[4 * k + 2];
      t.w = o[4 * k + 3];
      stg(q + k, t);
    }
  } else {
    pd2* q = reinterpret_cast<pd2*>(rec + (size_t)n * 4 * D);
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
      pd2 t;
      t.x = o[2 * k];
      t.y = o[2 * k + 1];
      stg(q + k, t);
    }
  }
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One node component of the fused PCG step: s = w + beta s_old,
// r' = r - alpha s, u' = M^-1 r'.  Every workgroup that gathers the node
// evaluates this same expression on the same record.
template <typename T>
__device__ __forceinline__ void fcg_step(T r, T w, T s_old, T mi, T alpha, T beta, T& s,
                                         T& rn, T& un) {
  s = fma_t(beta, s_old, w);
  rn = fma_t(-alpha, s, r);
  un = mi * rn;
}

}  // namespace pfem
