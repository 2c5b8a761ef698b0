// Two-level preconditioned CG (classic loop) on the device.
//
// M^-1 r = D^-1 r + P A_c^-1 P^T r: the Jacobi part pointwise, the coarse
// part through three passes that ride on the PCG's own launches --
//   restriction: every owner block sums the raw rigid modes of its nodes
//     against the new residual, in the same pass as the residual update;
//   coarse solve: one workgroup per (solve, kCoarseRows rows) sums the
//     block partials of every aggregate (the raw restriction R^T r) and
//     multiplies its rows of B = T A_c^-1 T^T with it, giving the raw-mode
//     coefficients y of the coarse correction (T maps raw modes to the
//     orthonormal coarse basis; it is folded into B on the host); its
//     partial of (R^T r) . y is the coarse share of r . M^-1 r;
//   prolongation: the direction pass evaluates z = D^-1 r + R(x) y at every
//     DOF it owns, so p = z + beta p needs no extra vector.
// Every sum runs in a fixed order, as the other reductions of the library.
#include "pfem_internal.h"
#include "reduce.h"

namespace pfem {

namespace {

template <int D>
__device__ __forceinline__ int tl_modes() { return D == 2 ? 3 : 6; }

// Raw rigid mode j at component c of a node with coordinates y relative to
// its aggregate's centroid (2D: translations, rotation (-y1, y0); 3D:
// translations, rotations (0, -y2, y1), (y2, 0, -y0), (-y1, y0, 0)).
template <int D, typename T>
__device__ __forceinline__ double mode_val(int c, int j, const T* y) {
  if (j < D) return c == j ? 1.0 : 0.0;
  if constexpr (D == 2) {
    return c == 0 ? -(double)y[1] : (double)y[0];
  } else {
    const double y0 = y[0], y1 = y[1], y2 = y[2];
    if (j == 3) return c == 0 ? 0.0 : (c == 1 ? -y2 : y1);
    if (j == 4) return c == 0 ? y2 : (c == 1 ? 0.0 : -y0);
    return c == 0 ? -y1 : (c == 1 ? y0 : 0.0);
  }
}

// Coarse part of z at DOF c of node n: sum_j R(n)[c][j] y[agg(n)][j].
template <int D, typename T>
__device__ __forceinline__ double coarse_part(const Task* tp, const TwoLevelDev& tl, int n,
                                              int c) {
  const T* rel = static_cast<const T*>(tl.rel) + (size_t)n * D;
  const int a = (n / tp->m.bn) / tl.G;
  const double* y = tl.y + (size_t)a * 6;
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < tl_modes<D>(); ++j) s += mode_val<D, T>(c, j, rel) * ldg(y + j);
  return s;
}

// Store this block's restriction partials: sum over its DOFs of R^T r.
__device__ __forceinline__ void write_restriction(const TwoLevelDev& tl, int blk,
                                                  double (&rc)[6]) {
  block_sum_all<6>(rc);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < 6; ++j) tl.rc_part[(size_t)blk * 6 + j] = rc[j];
}

}  // namespace

// r = -g; d = 0; restriction partials of r.  Partials: slot 1 = r.D^-1 r,
// slot 2 = r.r (p follows after the coarse solve).
template <int D, typename T>
__global__ void __launch_bounds__(kThreads)
k_tl_init(const Task* __restrict__ tasks, const int2* __restrict__ work) {
  const int2 wk = work[blockIdx.x];
  const Task* tp = tasks + wk.x;
  if (!tp->active) return;
  const TwoLevelDev tl = *tp->tl;
  const int n0 = wk.y * tp->m.bn;
  const int nloc = min(tp->m.bn, tp->m.n_nodes - n0);
  const double* G = static_cast<const double*>(tp->u);
  const T* Mi = static_cast<const T*>(tp->minv);
  T* R = static_cast<T*>(tp->r);
  T* Dd = static_cast<T*>(tp->d);
  const T* rel = static_cast<const T*>(tl.rel);
  double part[kRedSlots] = {0.0, 0.0, 0.0, 0.0};
  double rc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nloc * D; i += kThreads) {
    const size_t g = (size_t)n0 * D + i;
    const T r = (T)(-ldg(G + g));
    stg(R + g, r);
    stg(Dd + g, T(0));
    part[1] += (double)r * (double)ldg(Mi + g) * (double)r;
    part[2] += (double)r * (double)r;
    const int n = n0 + i / D, c = i % D;
#pragma unroll
    for (int j = 0; j < tl_modes<D>(); ++j)
      rc[j] += mode_val<D, T>(c, j, rel + (size_t)n * D) * (double)r;
  }
  write_restriction(tl, wk.y, rc);
  write_partials(tp->red, tp->m.n_blocks, wk.y, part, 1, 3);
}

// The coarse solve of one chunk of kCoarseRows rows of B (see the file
// comment): every workgroup gathers the whole raw restriction R^T r into LDS,
// then each wave takes two rows of B at once.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_tl_coarse(const Task* __restrict__ tasks, const int2* __restrict__ cwork, int init) {
  static_assert(kCoarseRows == 2 * (kThreads / 64), "two rows of B per wave");
  __shared__ double rc[kCoarseMax];
  __shared__ double ys[kCoarseRows];
  const int2 wk = cwork[blockIdx.x];
  const Task* tp = tasks + wk.x;
  if (!tp->active) return;
  if (!init && ldg(&tp->sc->state) != 0) return;
  const TwoLevelDev tl = *tp->tl;
  const int nrb = tl.nrb, nb = tp->m.n_blocks, n_c = tl.n_c;
  for (int i = threadIdx.x; i < n_c; i += kThreads) {
    const int a = i / nrb, j = i - a * nrb;
    const int b1 = min(nb, (a + 1) * tl.G);
    double s = 0.0;
    for (int b = a * tl.G; b < b1; ++b) s += ldg(tl.rc_part + (size_t)b * 6 + j);
    rc[i] = s;
  }
  __syncthreads();
  const int r0 = wk.y * kCoarseRows, r1 = min(n_c, r0 + kCoarseRows);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T* B = static_cast<const T*>(tl.B);
  const int i0 = r0 + 2 * wave;          // uniform over the wave
  if (i0 < r1) {
    const bool two = i0 + 1 < r1;
    const T* ra = B + (size_t)i0 * n_c;
    const T* rb = B + (size_t)(two ? i0 + 1 : i0) * n_c;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    int j = lane;
    for (; j + 192 < n_c; j += 256) {
      const double x0 = rc[j], x1 = rc[j + 64], x2 = rc[j + 128], x3 = rc[j + 192];
      a0 += (double)ldg(ra + j) * x0;
      a1 += (double)ldg(ra + j + 64) * x1;
      a2 += (double)ldg(ra + j + 128) * x2;
      a3 += (double)ldg(ra + j + 192) * x3;
      b0 += (double)ldg(rb + j) * x0;
      b1 += (double)ldg(rb + j + 64) * x1;
      b2 += (double)ldg(rb + j + 128) * x2;
      b3 += (double)ldg(rb + j + 192) * x3;
    }
    for (; j < n_c; j += 64) {
      a0 += (double)ldg(ra + j) * rc[j];
      b0 += (double)ldg(rb + j) * rc[j];
    }
    const double sa = wave_sum((a0 + a1) + (a2 + a3));
    const double sb = wave_sum((b0 + b1) + (b2 + b3));
    if (lane == 0) {
      ys[i0 - r0] = sa;
      if (two) ys[i0 + 1 - r0] = sb;
    }
  }
  __syncthreads();
  double v[1] = {0.0};
  if ((int)threadIdx.x < r1 - r0) {
    const int i = r0 + threadIdx.x, a = i / nrb, j = i - a * nrb;
    tl.y[(size_t)a * 6 + j] = ys[threadIdx.x];
    v[0] = rc[i] * ys[threadIdx.x];
  }
  block_sum_all<1>(v);
  if (threadIdx.x == 0) tl.gc_part[wk.y] = v[0];
}

// Start: p = M^-1 r.
template <int D, typename T>
__global__ void __launch_bounds__(kThreads)
k_tl_prolong_init(const Task* __restrict__ tasks, const int2* __restrict__ work) {
  const int2 wk = work[blockIdx.x];
  const Task* tp = tasks + wk.x;
  if (!tp->active) return;
  const TwoLevelDev tl = *tp->tl;
  const int n0 = wk.y * tp->m.bn;
  const int nloc = min(tp->m.bn, tp->m.n_nodes - n0);
  const T* Mi = static_cast<const T*>(tp->minv);
  const T* R = static_cast<const T*>(tp->r);
  T* P = static_cast<T*>(tp->p);
  for (int i = threadIdx.x; i < nloc * D; i += kThreads) {
    const size_t g = (size_t)n0 * D + i;
    const int n = n0 + i / D, c = i % D;
    const bool con = (ldg(tp->m.dmask + n) >> c) & 1;
    const double z = (double)ldg(Mi + g) * (double)ldg(R + g) +
                     (con ? 0.0 : coarse_part<D, T>(tp, tl, n, c));
    stg(P + g, (T)z);
  }
}

// alpha from p.q (slot 0); r -= alpha q; d += alpha p; restriction partials
// of the new r; partials slot 1 = r.D^-1 r, slot 2 = r.r.
template <int D, typename T>
__global__ void __launch_bounds__(kThreads)
k_tl_update(const Task* __restrict__ tasks, const int2* __restrict__ work, int it) {
  const int2 wk = work[blockIdx.x];
  const Task* tp = tasks + wk.x;
  if (!tp->active) return;
  Scalars* sc = tp->sc;
  if (ldg(&sc->state) != 0) return;
  const int nb = tp->m.n_blocks;
  double pq, unused;
  sum_slots2(tp->red.part, nb, 0, 0, pq, unused);
  const int j = tp->k_base + it;
  if (!(pq > 0.0)) {   // breakdown (not SPD) or NaN: nothing moves
    if (wk.y == 0 && threadIdx.x == 0) {
      sc->pq = pq;
      sc->state = 3;
    }
    return;
  }
  const double alpha64 = ldg(&sc->rz2[j & 1]) / pq;
  const T alpha = (T)alpha64;
  if (wk.y == 0 && threadIdx.x == 0) {
    sc->pq = pq;
    sc->alpha = alpha64;
  }
  const TwoLevelDev tl = *tp->tl;
  const int n0 = wk.y * tp->m.bn;
  const int nloc = min(tp->m.bn, tp->m.n_nodes - n0);
  const T* Q = static_cast<const T*>(tp->y);
  const T* P = static_cast<const T*>(tp->p);
  const T* Mi = static_cast<const T*>(tp->minv);
  T* R = static_cast<T*>(tp->r);
  T* Dd = static_cast<T*>(tp->d);
  const T* rel = static_cast<const T*>(tl.rel);
  double part[kRedSlots] = {0.0, 0.0, 0.0, 0.0};
  double rc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nloc * D; i += kThreads) {
    const size_t g = (size_t)n0 * D + i;
    const T p = ldg(P + g);
    const T r = ldg(R + g) - alpha * ldg(Q + g);
    stg(R + g, r);
    if constexpr (sizeof(T) == 8) stg(Dd + g, ldg(Dd + g) + alpha64 * p);
    else stg(Dd + g, ldg(Dd + g) + alpha * p);
    part[1] += (double)r * (double)ldg(Mi + g) * (double)r;
    part[2] += (double)r * (double)r;
    const int n = n0 + i / D, c = i % D;
#pragma unroll
    for (int jj = 0; jj < tl_modes<D>(); ++jj)
      rc[jj] += mode_val<D, T>(c, jj, rel + (size_t)n * D) * (double)r;
  }
  write_restriction(tl, wk.y, rc);
  write_partials(tp->red, nb, wk.y, part, 1, 3);   // slot 0 is still being read
}

// beta = (r.M^-1 r) / previous, the stopping tests, and p = M^-1 r + beta p.
template <int D, typename T>
__global__ void __launch_bounds__(kThreads)
k_tl_direction(const Task* __restrict__ tasks, const int2* __restrict__ work, int it) {
  const int2 wk = work[blockIdx.x];
  const Task* tp = tasks + wk.x;
  if (!tp->active) return;
  Scalars* sc = tp->sc;
  if (ldg(&sc->state) != 0) return;
  const int nb = tp->m.n_blocks;
  const TwoLevelDev tl = *tp->tl;
  double rz, rr;
  sum_slots2(tp->red.part, nb, 1, 2, rz, rr);
  {
    double v[1] = {0.0};
    for (int c = threadIdx.x; c < tl.n_chunks; c += kThreads) v[0] += ldg(tl.gc_part + c);
    block_sum_all<1>(v);
    rz += v[0];
  }
  const int j = tp->k_base + it;
  const double beta64 = rz / ldg(&sc->rz2[j & 1]);
  int state = 0;
  if (!(rr == rr) || !(rz == rz))
    state = 3;
  else if (rr <= ldg(&sc->target2))
    state = 1;
  else if (!(rz > 0.0))
    state = 3;
  else if (j + 1 >= ldg(&sc->kmax))
    state = 2;
  if (wk.y == 0 && threadIdx.x == 0) {
    sc->rz2[(j + 1) & 1] = rz;
    sc->rr = rr;
    sc->beta = beta64;
    const double rho = sqrt(rr) / sc->den;
    sc->rho = rho;
    sc->k = j + 1;
    sc->total_k += 1;
    const int h = tp->hist_base + j;
    if (tp->hist != nullptr && h < sc->hist_cap) {
      tp->hist[h] = rho;
      sc->hist_len = h + 1;
    }
    if (state != 0) sc->state = state;
  }
  if (state != 0) return;
  const T beta = (T)beta64;
  const int n0 = wk.y * tp->m.bn;
  const int nloc = min(tp->m.bn, tp->m.n_nodes - n0);
  const T* Mi = static_cast<const T*>(tp->minv);
  const T* R = static_cast<const T*>(tp->r);
  T* P = static_cast<T*>(tp->p);
  for (int i = threadIdx.x; i < nloc * D; i += kThreads) {
    const size_t g = (size_t)n0 * D + i;
    const int n = n0 + i / D, c = i % D;
    const bool con = (ldg(tp->m.dmask + n) >> c) & 1;
    const double z = (double)ldg(Mi + g) * (double)ldg(R + g) +
                     (con ? 0.0 : coarse_part<D, T>(tp, tl, n, c));
    stg(P + g, (T)z + beta * ldg(P + g));
  }
}

// ---------------------------------------------------------------- launchers
#define PFEM_TL_LAUNCH(KERNEL, FAM, ...)                                                 \
  do {                                                                                   \
    if (n_work <= 0) return;                                                             \
    hipEvent_t ev = nullptr;                                                             \
    ctx->timing_begin(FAM, &ev);                                                         \
    dim3 grid(n_work), block(kThreads);                                                  \
    if (dim == 2 && prec == PFEM_FP32)                                                   \
      hipLaunchKernelGGL((KERNEL<2, float>), grid, block, 0, ctx->stream, __VA_ARGS__);  \
    else if (dim == 2)                                                                   \
      hipLaunchKernelGGL((KERNEL<2, double>), grid, block, 0, ctx->stream, __VA_ARGS__); \
    else if (prec == PFEM_FP32)                                                          \
      hipLaunchKernelGGL((KERNEL<3, float>), grid, block, 0, ctx->stream, __VA_ARGS__);  \
    else                                                                                 \
      hipLaunchKernelGGL((KERNEL<3, double>), grid, block, 0, ctx->stream, __VA_ARGS__); \
    PFEM_HIP(hipGetLastError());                                                         \
    ctx->timing_end(FAM, ev);                                                            \
  } while (0)

void launch_tl_init(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                    int n_work) {
  PFEM_TL_LAUNCH(k_tl_init, FAM_UPDATE, tasks, work);
}

void launch_tl_prolong_init(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                            int n_work) {
  PFEM_TL_LAUNCH(k_tl_prolong_init, FAM_DIRECTION, tasks, work);
}

void launch_tl_update(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                      int n_work, int it) {
  PFEM_TL_LAUNCH(k_tl_update, FAM_UPDATE, tasks, work, it);
}

void launch_tl_direction(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                         int n_work, int it) {
  PFEM_TL_LAUNCH(k_tl_direction, FAM_DIRECTION, tasks, work, it);
}

void launch_tl_coarse(Ctx* ctx, int prec, const Task* tasks, const int2* cwork, int n_cwork,
                      int init) {
  if (n_cwork <= 0) return;
  hipEvent_t ev = nullptr;
  ctx->timing_begin(FAM_DIRECTION, &ev);
  if (prec == PFEM_FP32)
    hipLaunchKernelGGL(k_tl_coarse<float>, dim3(n_cwork), dim3(kThreads), 0, ctx->stream, tasks,
                       cwork, init);
  else
    hipLaunchKernelGGL(k_tl_coarse<double>, dim3(n_cwork), dim3(kThreads), 0, ctx->stream, tasks,
                       cwork, init);
  PFEM_HIP(hipGetLastError());
  ctx->timing_end(FAM_DIRECTION, ev);
}

}  // namespace pfem
