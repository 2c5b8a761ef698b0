// Jacobi-PCG vector passes and small vector kernels.
//
// PCG (Saad, Alg. 9.1, with the Jacobi preconditioner M = diag A; App. B
// iteration U^(k+1) = phi(U^(k))) solves A d = r0 for the correction d.  One
// iteration is three launches over the owned node blocks of every live task:
//   apply      q = A p; partials of p.q                     (element kernel)
//   update     pq from the apply partials; alpha = rz / pq;
//              d += alpha p, r -= alpha q; partials of r.M^-1 r and r.r
//   direction  rz', rr from the update partials; beta = rz' / rz; the
//              convergence test; p = M^-1 r + beta p
// Every workgroup sums the previous kernel's partials itself (fixed order),
// so the scalars never leave the device and no workgroup waits for another.
// Block 0 of a task records the scalars, the residual history and the
// state; the next launch returns at once for a task that left "running".
// z = M^-1 r is never stored.  The fused variant (one element launch per
// iteration) lives with the element kernels; its start-up passes are here.
#include "pfem_internal.h"
#include "fcg_record.h"
#include "reduce.h"

namespace pfem {

template <int D>
__device__ __forceinline__ void block_range(const Task* tp, int blk, size_t& g0, int& n) {
  const int n0 = blk * tp->m.bn;
  const int nloc = min(tp->m.bn, tp->m.n_nodes - n0);
  g0 = (size_t)n0 * D;
  n = nloc * D;
}

// r = -g (g: float64 gradient at the outer iterate, Dirichlet-masked);
// d = 0; p = M^-1 r.  Partials: slot 1 = r.M^-1 r, slot 2 = r.r.
template <int D, typename T>
__global__ void __launch_bounds__(kThreads)
k_pcg_init(const Task* __restrict__ tasks, const int2* __restrict__ work) {
  const int2 wk = work[blockIdx.x];
  const Task* tp = tasks + wk.x;
  if (!tp->active) return;
  size_t g0;
  int n;
  block_range<D>(tp, wk.y, g0, n);
  const double* G = static_cast<const double*>(tp->u);
  const T* Mi = static_cast<const T*>(tp->minv);
  T* R = static_cast<T*>(tp->r);
  T* P = static_cast<T*>(tp->p);
  T* Dd = static_cast<T*>(tp->d);
  double part[kRedSlots] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const size_t g = g0 + i;
    const T r = (T)(-ldg(G + g));
    const T z = ldg(Mi + g) * r;
    stg(R + g, r);
    stg(P + g, z);
    stg(Dd + g, T(0));
    part[1] += (double)r * (double)z;
    part[2] += (double)r * (double)r;
  }
  write_partials(tp->red, tp->m.n_blocks, wk.y, part, 1, 3);
}

// Fused PCG start: r = -g; record {r, w = 0, s = 0, M^-1} of parity 0;
// p = u = M^-1 r (the vector the start-up apply multiplies); d = 0.
// Partials: slot 1 = r.u, slot 2 = r.r.
template <int D, typename T>
__global__ void __launch_bounds__(kThreads)
k_fcg_init(const Task* __restrict__ tasks, const int2* __restrict__ work) {
  const int2 wk = work[blockIdx.x];
  const Task* tp = tasks + wk.x;
  if (!tp->active) return;
  const int n0 = wk.y * tp->m.bn;
  const int nloc = min(tp->m.bn, tp->m.n_nodes - n0);
  const double* G = static_cast<const double*>(tp->u);
  const T* Mi = static_cast<const T*>(tp->minv);
  T* Rec = static_cast<T*>(tp->rec[0]);
  T* P = static_cast<T*>(tp->p);
  T* Dd = static_cast<T*>(tp->d);
  double part[kRedSlots] = {0.0, 0.0, 0.0, 0.0};
  for (int ln = threadIdx.x; ln < nloc; ln += kThreads) {
    const int n = n0 + ln;
    T o[4 * D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const size_t g = (size_t)n * D + c;
      const T r = (T)(-ldg(G + g));
      const T mi = ldg(Mi + g);
      const T u = mi * r;
      o[c] = r;
      o[D + c] = T(0);
      o[2 * D + c] = T(0);
      o[3 * D + c] = mi;
      stg(P + g, u);
      stg(Dd + g, T(0));
      part[1] += (double)r * (double)u;
      part[2] += (double)r * (double)r;
    }
    store_record<D, T>(Rec, n, o);
  }
  write_partials(tp->red, tp->m.n_blocks, wk.y, part, 1, 3);
}

// Fused PCG start, after tmp = A u: w of the parity-0 records = tmp.
template <int D, typename T>
__global__ void __launch_bounds__(kThreads)
k_fcg_init_w(const Task* __restrict__ tasks, const int2* __restrict__ work) {
  const int2 wk = work[blockIdx.x];
  const Task* tp = tasks + wk.x;
  if (!tp->active) return;
  const int n0 = wk.y * tp->m.bn;
  const int nloc = min(tp->m.bn, tp->m.n_nodes - n0);
  T* Rec = static_cast<T*>(tp->rec[0]);
  const T* W = static_cast<const T*>(tp->tmp);
  for (int ln = threadIdx.x; ln < nloc; ln += kThreads) {
    const int n = n0 + ln;
    T o[4 * D];
    load_record<D, T>(Rec, n, o);
#pragma unroll
    for (int c = 0; c < D; ++c) o[D + c] = ldg(W + (size_t)n * D + c);
    store_record<D, T>(Rec, n, o);
  }
}

// One workgroup per task: scalars at the start of an inner solve.
__global__ void __launch_bounds__(kThreads) k_pcg_init_finish(const Task* __restrict__ tasks) {
  const Task* tp = tasks + blockIdx.x;
  if (!tp->active) return;
  double rz, rr;
  sum_slots2(tp->red.part, tp->m.n_blocks, 1, 2, rz, rr);
  if (tp->tl != nullptr) {   // two-level: the coarse share of r.M^-1 r
    const TwoLevelDev* tl = tp->tl;
    double v[1] = {0.0};
    for (int c = threadIdx.x; c < tl->n_chunks; c += kThreads) v[0] += ldg(tl->gc_part + c);
    block_sum_all<1>(v);
    rz += v[0];
  }
  if (threadIdx.x != 0) return;
  Scalars* sc = tp->sc;
  sc->rz2[0] = rz;
  sc->rr = rr;
  sc->bnorm = sqrt(rr);
  sc->rho = sqrt(rr) / sc->den;
  sc->k = 0;
  if (tp->hist != nullptr && sc->hist_len == 0 && sc->hist_cap > 0) {
    tp->hist[0] = sc->rho;
    sc->hist_len = 1;
  }
  if (!(rr == rr) || !(rz == rz))
    sc->state = 3;
  else if (rr <= sc->target2)
    sc->state = 1;
  else if (!(rz > 0.0))
    sc->state = 3;
  else if (sc->kmax <= 0)
    sc->state = 2;
  else
    sc->state = 0;
}

template <int D, typename T>
__global__ void __launch_bounds__(kThreads)
k_pcg_update(const Task* __restrict__ tasks, const int2* __restrict__ work, int it) {
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
  size_t g0;
  int n;
  block_range<D>(tp, wk.y, g0, n);
  const T* Q = static_cast<const T*>(tp->y);
  const T* P = static_cast<const T*>(tp->p);
  const T* Mi = static_cast<const T*>(tp->minv);
  T* R = static_cast<T*>(tp->r);
  T* Dd = static_cast<T*>(tp->d);
  double part[kRedSlots] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const size_t g = g0 + i;
    const T p = ldg(P + g);
    const T r = ldg(R + g) - alpha * ldg(Q + g);
    stg(R + g, r);
    if constexpr (sizeof(T) == 8) stg(Dd + g, ldg(Dd + g) + alpha64 * p);
    else stg(Dd + g, ldg(Dd + g) + alpha * p);
    part[1] += (double)r * (double)ldg(Mi + g) * (double)r;
    part[2] += (double)r * (double)r;
  }
  write_partials(tp->red, nb, wk.y, part, 1, 3);   // slot 0 is still being read
}

template <int D, typename T>
__global__ void __launch_bounds__(kThreads)
k_pcg_direction(const Task* __restrict__ tasks, const int2* __restrict__ work, int it) {
  const int2 wk = work[blockIdx.x];
  const Task* tp = tasks + wk.x;
  if (!tp->active) return;
  Scalars* sc = tp->sc;
  if (ldg(&sc->state) != 0) return;
  const int nb = tp->m.n_blocks;
  double rz, rr;
  sum_slots2(tp->red.part, nb, 1, 2, rz, rr);
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
  size_t g0;
  int n;
  block_range<D>(tp, wk.y, g0, n);
  const T* Mi = static_cast<const T*>(tp->minv);
  const T* R = static_cast<const T*>(tp->r);
  T* P = static_cast<T*>(tp->p);
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const size_t g = g0 + i;
    stg(P + g, ldg(Mi + g) * ldg(R + g) + beta * ldg(P + g));
  }
}

// Partials of u . v (u float64, v kernel type) in slot 0.
template <int D, typename T>
__global__ void __launch_bounds__(kThreads)
k_dot(const Task* __restrict__ tasks, const int2* __restrict__ work) {
  const int2 wk = work[blockIdx.x];
  const Task* tp = tasks + wk.x;
  if (!tp->active) return;
  size_t g0;
  int n;
  block_range<D>(tp, wk.y, g0, n);
  const double* A = static_cast<const double*>(tp->u);
  const T* B = static_cast<const T*>(tp->v);
  double part[kRedSlots] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += kThreads)
    part[0] += ldg(A + g0 + i) * (double)ldg(B + g0 + i);
  write_partials(tp->red, tp->m.n_blocks, wk.y, part, 0, 1);
}

// One workgroup per task: red.out[0..NS-1] = totals of partial slots 0..NS-1.
template <int NS>
__global__ void __launch_bounds__(kThreads) k_reduce_store(const Task* __restrict__ tasks) {
  const Task* tp = tasks + blockIdx.x;
  if (!tp->active) return;
  double s0, s1, s2 = 0.0;
  if constexpr (NS == 3) sum_slots3(tp->red.part, tp->m.n_blocks, s0, s1, s2);
  else sum_slots2(tp->red.part, tp->m.n_blocks, 0, 1, s0, s1);
  if (threadIdx.x == 0) {
    tp->red.out[0] = s0;
    tp->red.out[1] = s1;
    if constexpr (NS == 3) tp->red.out[2] = s2;
  }
}

#define PFEM_VEC_LAUNCH(KERNEL, FAM, ...)                                              \
  do {                                                                                \
    if (n_work <= 0) return;                                                          \
    hipEvent_t ev = nullptr;                                                          \
    ctx->timing_begin(FAM, &ev);                                                      \
    dim3 grid(n_work), block(kThreads);                                               \
    if (dim == 2 && prec == PFEM_FP32)                                                \
      hipLaunchKernelGGL((KERNEL<2, float>), grid, block, 0, ctx->stream, __VA_ARGS__);  \
    else if (dim == 2)                                                                \
      hipLaunchKernelGGL((KERNEL<2, double>), grid, block, 0, ctx->stream, __VA_ARGS__); \
    else if (prec == PFEM_FP32)                                                       \
      hipLaunchKernelGGL((KERNEL<3, float>), grid, block, 0, ctx->stream, __VA_ARGS__);  \
    else                                                                              \
      hipLaunchKernelGGL((KERNEL<3, double>), grid, block, 0, ctx->stream, __VA_ARGS__); \
    PFEM_HIP(hipGetLastError());                                                      \
    ctx->timing_end(FAM, ev);                                                         \
  } while (0)

void launch_pcg_init(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                     int n_work, int n_tasks) {
  PFEM_VEC_LAUNCH(k_pcg_init, FAM_UPDATE, tasks, work);
  hipLaunchKernelGGL(k_pcg_init_finish, dim3(n_tasks), dim3(kThreads), 0, ctx->stream, tasks);
  PFEM_HIP(hipGetLastError());
}
void launch_pcg_init_finish(Ctx* ctx, const Task* tasks, int n_tasks) {
  if (n_tasks <= 0) return;
  hipLaunchKernelGGL(k_pcg_init_finish, dim3(n_tasks), dim3(kThreads), 0, ctx->stream, tasks);
  PFEM_HIP(hipGetLastError());
}
void launch_fcg_init(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                     int n_work) {
  PFEM_VEC_LAUNCH(k_fcg_init, FAM_UPDATE, tasks, work);
}
void launch_fcg_init_w(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                       int n_work) {
  PFEM_VEC_LAUNCH(k_fcg_init_w, FAM_UPDATE, tasks, work);
}
void launch_pcg_update(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                       int n_work, int it) {
  PFEM_VEC_LAUNCH(k_pcg_update, FAM_UPDATE, tasks, work, it);
}
void launch_pcg_direction(Ctx* ctx, int dim, int prec, const Task* tasks,
                          const int2* work, int n_work, int it) {
  PFEM_VEC_LAUNCH(k_pcg_direction, FAM_DIRECTION, tasks, work, it);
}
void launch_dot(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                int n_work) {
  PFEM_VEC_LAUNCH(k_dot, FAM_UPDATE, tasks, work);
}
void launch_reduce_store(Ctx* ctx, const Task* tasks, int n_tasks, int n_slots) {
  if (n_tasks <= 0) return;
  if (n_slots == 3)
    hipLaunchKernelGGL(k_reduce_store<3>, dim3(n_tasks), dim3(kThreads), 0, ctx->stream, tasks);
  else
    hipLaunchKernelGGL(k_reduce_store<2>, dim3(n_tasks), dim3(kThreads), 0, ctx->stream, tasks);
  PFEM_HIP(hipGetLastError());
}

__global__ void k_set_scalars(Scalars* sc, double den, double target2, int kmax,
                              int reset_hist, int reset_total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc->den = den;
    sc->target2 = target2;
    sc->kmax = kmax;
    sc->k = 0;
    sc->state = 0;
    if (reset_hist) sc->hist_len = 0;
    if (reset_total) sc->total_k = 0;
  }
}

void launch_set_scalars(Ctx* ctx, Scalars* sc, double den, double target2, int kmax,
                        bool reset_hist, bool reset_total) {
  hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, ctx->stream, sc, den, target2,
                     kmax, reset_hist ? 1 : 0, reset_total ? 1 : 0);
  PFEM_HIP(hipGetLastError());
}

// energies from (value, #inverted) pairs: +inf where any J <= 0.
__global__ void k_energy_out(const double* red, double* out, int n, int stride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = red[(size_t)i * stride + 1] > 0.5 ? __builtin_inf() : red[(size_t)i * stride];
}

void launch_energy_out(Ctx* ctx, const double* red, double* out, int n, int stride) {
  hipLaunchKernelGGL(k_energy_out, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, red, out,
                     n, stride);
  PFEM_HIP(hipGetLastError());
}

// ------------------------------------------------------------ small kernels
static int grid_for(int64_t n) {
  const int64_t g = (n + kThreads - 1) / kThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

template <typename T>
__global__ void k_permute(const int32_t* __restrict__ perm, int64_t n_nodes, int dim,
                          bool to_internal, const T* __restrict__ in, T* __restrict__ out) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_nodes * dim;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = k / dim;
    const int c = (int)(k % dim);
    const int64_t nn = perm[node];   // caller node -> internal node
    if (to_internal) out[nn * dim + c] = in[k];
    else out[k] = in[nn * dim + c];
  }
}

void launch_permute(Ctx* ctx, int prec, int dim, const int32_t* perm, int64_t n_nodes,
                    bool to_internal, const void* in, void* out) {
  const int g = grid_for(n_nodes * dim);
  if (prec == PFEM_FP64)
    hipLaunchKernelGGL(k_permute<double>, dim3(g), dim3(kThreads), 0, ctx->stream, perm,
                       n_nodes, dim, to_internal, (const double*)in, (double*)out);
  else
    hipLaunchKernelGGL(k_permute<float>, dim3(g), dim3(kThreads), 0, ctx->stream, perm,
                       n_nodes, dim, to_internal, (const float*)in, (float*)out);
  PFEM_HIP(hipGetLastError());
}

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    p[k] = v;
}

void launch_fill(Ctx* ctx, int prec, void* p, int64_t n, double value) {
  if (n <= 0) return;
  const int g = grid_for(n);
  if (prec == PFEM_FP64)
    hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(kThreads), 0, ctx->stream,
                       (double*)p, n, value);
  else
    hipLaunchKernelGGL(k_fill<float>, dim3(g), dim3(kThreads), 0, ctx->stream,
                       (float*)p, n, (float)value);
  PFEM_HIP(hipGetLastError());
}

__global__ void k_cast64to32(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    out[k] = (float)in[k];
}
__global__ void k_cast32to64(const float* __restrict__ in, double* __restrict__ out, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    out[k] = (double)in[k];
}

void launch_cast(Ctx* ctx, bool to32, const void* in, void* out, int64_t n) {
  if (n <= 0) return;
  const int g = grid_for(n);
  if (to32)
    hipLaunchKernelGGL(k_cast64to32, dim3(g), dim3(kThreads), 0, ctx->stream,
                       (const double*)in, (float*)out, n);
  else
    hipLaunchKernelGGL(k_cast32to64, dim3(g), dim3(kThreads), 0, ctx->stream,
                       (const float*)in, (double*)out, n);
  PFEM_HIP(hipGetLastError());
}

template <typename T>
__global__ void k_axpy_state(const uint8_t* __restrict__ dmask, const double* __restrict__ ubar,
                             int dim, int64_t n, double* out, const double* base,
                             const T* __restrict__ inc, double s, bool set_dir, double scale) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    double v = base != nullptr ? base[k] : 0.0;
    if (inc != nullptr) v += s * (double)inc[k];
    if (set_dir && ((dmask[k / dim] >> (k % dim)) & 1)) v = scale * ubar[k];
    out[k] = v;
  }
}

void launch_axpy_state(Ctx* ctx, int prec, const MeshDev& m, double* out, const double* base,
                       const void* inc, double s, bool set_dirichlet, double scale) {
  const int64_t n = (int64_t)m.n_nodes * m.dim;
  const int g = grid_for(n);
  if (prec == PFEM_FP64)
    hipLaunchKernelGGL(k_axpy_state<double>, dim3(g), dim3(kThreads), 0, ctx->stream, m.dmask,
                       m.ubar, m.dim, n, out, base, (const double*)inc, s, set_dirichlet, scale);
  else
    hipLaunchKernelGGL(k_axpy_state<float>, dim3(g), dim3(kThreads), 0, ctx->stream, m.dmask,
                       m.ubar, m.dim, n, out, base, (const float*)inc, s, set_dirichlet, scale);
  PFEM_HIP(hipGetLastError());
}

void launch_lift(Ctx* ctx, const MeshDev& m, double* out, const double* base, double scale) {
  launch_axpy_state(ctx, PFEM_FP64, m, out, base, nullptr, 0.0, true, scale);
}

// ------------------------------------------------------- homogenisation
// X^0(IJ) = eps0^(IJ) . X at every node for the six unit strains of App. D
// (11, 22, 33: a one on the diagonal; 12, 13, 23: ones at (p, q) and
// (q, p)); out holds the six fields one after the other, internal order.
__global__ void k_affine6(const double* __restrict__ X, int64_t n_nodes,
                          double* __restrict__ out) {
  const int64_t nd = n_nodes * 3;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < n_nodes;
       n += (int64_t)gridDim.x * blockDim.x) {
    const double x[3] = {X[3 * n], X[3 * n + 1], X[3 * n + 2]};
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 3; ++i) out[k * nd + 3 * n + i] = i == k ? x[k] : 0.0;
    const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
    for (int s = 0; s < 3; ++s) {
      double* o = out + (3 + s) * nd + 3 * n;
      for (int i = 0; i < 3; ++i) o[i] = 0.0;
      o[P[s]] = x[Q[s]];
      o[Q[s]] = x[P[s]];
    }
  }
}

void launch_affine6(Ctx* ctx, const double* X, int64_t n_nodes, double* out) {
  hipLaunchKernelGGL(k_affine6, dim3(grid_for(n_nodes)), dim3(kThreads), 0, ctx->stream, X,
                     n_nodes, out);
  PFEM_HIP(hipGetLastError());
}

// G[k][l] = A_k . B_l for six vectors A_k and six B_l of n entries (stored
// one after the other): every workgroup sums its grid-stride share of the
// 36 products in float64 and stores one partial per product; a one-
// workgroup kernel then adds the partials in workgroup order (no atomics,
// the same result on every run).
__global__ void __launch_bounds__(kThreads)
k_gram6_part(const double* __restrict__ A, const double* __restrict__ B, int64_t n,
             double* __restrict__ part) {
  double v[36];
#pragma unroll
  for (int k = 0; k < 36; ++k) v[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    double a[6], b[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      a[k] = A[k * n + i];
      b[k] = B[k * n + i];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
      for (int l = 0; l < 6; ++l) v[6 * k + l] += a[k] * b[l];
  }
  block_sum_all<36>(v);
  if (threadIdx.x == 0)
    for (int k = 0; k < 36; ++k) part[(size_t)k * gridDim.x + blockIdx.x] = v[k];
}

__global__ void k_gram6_final(const double* __restrict__ part, int n_part,
                              double* __restrict__ out, double scale) {
  const int k = threadIdx.x;
  if (k < 36) {
    double s = 0.0;
    for (int b = 0; b < n_part; ++b) s += part[(size_t)k * n_part + b];
    out[k] = s * scale;
  }
}

int gram6_parts(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 1024)); }

void launch_gram6(Ctx* ctx, const double* A, const double* B, int64_t n, double* part,
                  double* out, double scale) {
  const int g = gram6_parts(n);
  hipLaunchKernelGGL(k_gram6_part, dim3(g), dim3(kThreads), 0, ctx->stream, A, B, n, part);
  hipLaunchKernelGGL(k_gram6_final, dim3(1), dim3(64), 0, ctx->stream, part, g, out, scale);
  PFEM_HIP(hipGetLastError());
}

}  // namespace pfem
