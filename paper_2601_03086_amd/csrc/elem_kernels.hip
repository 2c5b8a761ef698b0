// Element kernels: K.v / Hessian-vector product, internal force, Jacobi
// diagonal and energy on P1 triangles (D = 2) and tetrahedra (D = 3).
//
// Owner-computes scatter (default).  The internal node numbering is cut
// into contiguous blocks of `bn` nodes (compact patches cut from reverse
// Cuthill-McKee bands, or plain RCM runs); elements are sorted by their
// smallest node id.  One workgroup owns one node block: it walks the
// (contiguous) range of sorted elements whose smallest node it owns plus the
// list of earlier blocks' elements that reach into it, evaluates each,
// accumulates the contributions that land on its own nodes in LDS, and
// finally writes every owned DOF exactly once with coalesced stores.  No
// device-wide atomics, no zero-fill of the output, and dot products with the
// output are fused into the write loop.  Elements that straddle two blocks
// are evaluated by both; their gathers hit L2 because consecutive blocks are
// scheduled on the same XCD (work-table remap).  The LDS sums follow the
// order in which the waves reach them, so the last bits may vary from run
// to run; block partial sums are reduced in a fixed order.
//
// Alternatives for comparison: a device-wide atomic scatter over all
// elements, and a colour-by-colour deterministic scatter.
#include <type_traits>

#include "elem_math.h"
#include "fcg_record.h"
#include "owner_common.h"
#include "pfem_internal.h"
#include "reduce.h"

namespace pfem {

template <int D, typename T>
__device__ __forceinline__ void load_nodal(const T* __restrict__ p, int n, T (&o)[D]) {
  if constexpr (D == 2 && sizeof(T) == 4) {
    const pf2 q = ldx(reinterpret_cast<const pf2*>(p), (uint32_t)n);
    o[0] = q.x;
    o[1] = q.y;
  } else if constexpr (D == 2 && sizeof(T) == 8) {
    const pd2 q = ldx(reinterpret_cast<const pd2*>(p), (uint32_t)n);
    o[0] = q.x;
    o[1] = q.y;
  } else {
    const Trip<T> q = ldx(reinterpret_cast<const Trip<T>*>(p), (uint32_t)n);
    o[0] = q.x;
    o[1] = q.y;
    o[2] = q.z;
  }
}

template <int D>
__device__ __forceinline__ void load_conn(const int32_t* __restrict__ conn, int e,
                                          int (&nd)[D + 1]);

// Element e's nodes: in 2D packed (smallest node + two 16-bit offsets, 8
// bytes) when the mesh fits, else plain int32 rows; in 3D always the plain
// 16-byte row (measured: a packed 12-byte row made the 4M-tet K.v 1.4x
// slower in FP32 and the plain row 15% faster in FP64).
// PK = 1: the caller guarantees packed 2D connectivity (no run-time test, so
// no wait at a branch join).
template <int D, typename T, int PK = 0>
__device__ __forceinline__ void load_conn(const MeshDev& m, int e, int (&nd)[D + 1]) {
  if constexpr (D == 2) {
    if (PK == 1 || m.conn_packed) {
      typedef unsigned int pu2 __attribute__((ext_vector_type(2)));
      const pu2 q = ldx(reinterpret_cast<const pu2*>(m.connp), (uint32_t)e);
      nd[0] = (int)q.x;
      nd[1] = (int)(q.x + (q.y & 0xffffu));
      nd[2] = (int)(q.x + (q.y >> 16));
      return;
    }
  }
  load_conn<D>(m.conn, e, nd);
}

template <int D>
__device__ __forceinline__ void load_conn(const int32_t* __restrict__ conn, int e,
                                          int (&nd)[D + 1]) {
  if constexpr (D == 3) {
    const pi4 q = ldx(reinterpret_cast<const pi4*>(conn), (uint32_t)e);
    nd[0] = q.x;
    nd[1] = q.y;
    nd[2] = q.z;
    nd[3] = q.w;
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) nd[a] = ldx(conn, (uint32_t)(e * 3 + a));
  }
}

template <typename T>
__device__ __forceinline__ T mat_mu(const MeshDev& m, int e) {
  if constexpr (sizeof(T) == 4) return ldx(m.mu32, (uint32_t)e); else return ldx(m.mu64, (uint32_t)e);
}
// lambda of element e given its mu: one multiply when the mesh has a
// uniform lambda / mu ratio (one material value per element to stream)
// (branch-free: a uniform mesh re-reads mu, which is already in flight)
template <typename T>
__device__ __forceinline__ T mat_lam(const MeshDev& m, int e, T mu) {
  const T* lam;
  if constexpr (sizeof(T) == 4) lam = m.lam_uniform ? m.mu32 : m.lam32;
  else lam = m.lam_uniform ? m.mu64 : m.lam64;
  return ldx(lam, (uint32_t)e) * (m.lam_uniform ? (T)m.lam_ratio : T(1));
}

// Everything one element needs, gathered before any arithmetic so that all
// of its loads are in flight together.
template <int D, typename T, int OP, bool NL, bool FUSED = false>
struct ElemIn {
  ElemX<D, T> x;
  T u[D + 1][D];   // state (Neo-Hookean) or input of the linear force
  T v[D + 1][D];   // direction of the apply
  T c[OP == OP_HVPC ? D * D + 1 : 1];            // cached {F^-T, ln J}
  T rec[FUSED ? D + 1 : 1][FUSED ? 4 * D : 1];   // fused PCG records
  T mu, lam;
};

template <int D, typename T, int OP, bool NL, bool FUSED = false>
__device__ __forceinline__ void load_elem(const MeshDev& m, const T* __restrict__ U,
                                          const T* __restrict__ V, int mask, int e,
                                          const int (&nd)[D + 1],
                                          ElemIn<D, T, OP, NL, FUSED>& in) {
  load_elem_x<D, T>(m, nd, in.x);
  in.mu = mat_mu<T>(m, e);
  in.lam = mat_lam<T>(m, e, in.mu);
  if constexpr (OP == OP_HVPC) {   // U: the cache, one array of n_elems per value
#pragma unroll
    for (int k = 0; k <= D * D; ++k) in.c[k] = ldx(U, (uint32_t)(k * m.n_elems + e));
  } else if constexpr (NL || OP == OP_FORCE) {
#pragma unroll
    for (int a = 0; a <= D; ++a) load_nodal<D, T>(U, nd[a], in.u[a]);
  }
  if constexpr (FUSED) {
#pragma unroll
    for (int a = 0; a <= D; ++a) load_record<D, T>(V, nd[a], in.rec[a]);
  } else if constexpr (is_apply_op(OP)) {
#pragma unroll
    for (int a = 0; a <= D; ++a) load_nodal<D, T>(V, nd[a], in.v[a]);
    if (mask & PFEM_MASK_IN) {
#pragma unroll
      for (int a = 0; a <= D; ++a) {
        const int bits = ldx(m.dmask, (uint32_t)nd[a]);
#pragma unroll
        for (int i = 0; i < D; ++i)
          if (bits & (1 << i)) in.v[a][i] = T(0);
      }
    }
  }
}

// Fused PCG: the apply direction u' at the element's nodes from their records.
template <int D, typename T, int OP, bool NL>
__device__ __forceinline__ void fcg_direction(ElemIn<D, T, OP, NL, true>& in, T alpha, T beta) {
#pragma unroll
  for (int a = 0; a <= D; ++a)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T s, rn, un;
      fcg_step<T>(in.rec[a][c], in.rec[a][D + c], in.rec[a][2 * D + c], in.rec[a][3 * D + c],
                  alpha, beta, s, rn, un);
      in.v[a][c] = un;
    }
}

// Element output for one op; y[a][i] is the contribution to node a, comp i.
template <int D, typename T, int OP, bool NL, bool FUSED>
__device__ __forceinline__ void element_compute(const MeshDev& m,
                                                const ElemIn<D, T, OP, NL, FUSED>& in,
                                                T (&y)[D + 1][D]) {
  Geo<D, T> g;
  geometry_x<D, T>(m, in.x, g);
  const T mu = in.mu, lam = in.lam;
  const T adet = g.det < T(0) ? -g.det : g.det;
  const T s_sym = T(1) / (T(Fact<D>::v) * adet);       // vol / det^2
  if constexpr (OP == OP_DIAG) {
    T cc[D + 1][D];
#pragma unroll
    for (int i = 0; i < D; ++i) cc[0][i] = T(0);
#pragma unroll
    for (int a = 1; a <= D; ++a)
#pragma unroll
      for (int i = 0; i < D; ++i) {
        cc[a][i] = g.c[a - 1][i];
        cc[0][i] -= g.c[a - 1][i];
      }
    if constexpr (!NL) {
#pragma unroll
      for (int a = 0; a <= D; ++a) {
        T n2 = T(0);
#pragma unroll
        for (int i = 0; i < D; ++i) n2 += cc[a][i] * cc[a][i];
#pragma unroll
        for (int i = 0; i < D; ++i) y[a][i] = s_sym * (mu * n2 + (lam + mu) * cc[a][i] * cc[a][i]);
      }
    } else {
      T Ht[D][D];
      grad_tilde<D, T>(in.u, g, Ht);
      NHState<D, T> st;
      nh_state<D, T>(Ht, T(1) / g.det, st);
      const T coef = lam + mu - lam * st.lnJ;
#pragma unroll
      for (int a = 0; a <= D; ++a) {
        T n2 = T(0);
#pragma unroll
        for (int i = 0; i < D; ++i) n2 += cc[a][i] * cc[a][i];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          T w = T(0);
#pragma unroll
          for (int k = 0; k < D; ++k) w += st.FinvT[i][k] * cc[a][k];
          y[a][i] = s_sym * (mu * n2 + coef * w * w);
        }
      }
    }
  } else if constexpr (!NL) {
    // K v (OP_APPLY) or K u (OP_FORCE, f_ext subtracted by the caller)
    T M[D][D], S[D][D];
    if constexpr (OP == OP_APPLY) grad_tilde<D, T>(in.v, g, M);
    else grad_tilde<D, T>(in.u, g, M);
    linear_stress_tilde<D, T>(M, mu, lam, S);
    scatter_rows<D, T>(S, g, s_sym, y);
  } else {
    NHState<D, T> st;
    if constexpr (OP == OP_HVPC) {   // the tangent needs F^-T and ln J only
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int k = 0; k < D; ++k) st.FinvT[i][k] = in.c[i * D + k];
      st.lnJ = in.c[D * D];
    } else {
      T Ht[D][D];
      grad_tilde<D, T>(in.u, g, Ht);
      nh_state<D, T>(Ht, T(1) / g.det, st);
    }
    if constexpr (OP == OP_FORCE) {
      T P[D][D];
      nh_piola<D, T>(st, mu, lam, P);
      const T s_sgn = (g.det < T(0) ? T(-1) : T(1)) / T(Fact<D>::v);   // vol / det
      scatter_rows<D, T>(P, g, s_sgn, y);
    } else {
      T dF[D][D], dP[D][D];
      grad_tilde<D, T>(in.v, g, dF);
      nh_dpiola<D, T>(st, mu, lam, dF, dP);
      scatter_rows<D, T>(dP, g, s_sym, y);
    }
  }
}

template <int D, typename T, int OP, bool NL>
__device__ __forceinline__ void element_output(const MeshDev& m, const T* __restrict__ U,
                                               const T* __restrict__ V, int mask, int e,
                                               const int (&nd)[D + 1], T (&y)[D + 1][D]) {
  ElemIn<D, T, OP, NL> in;
  load_elem<D, T, OP, NL>(m, U, V, mask, e, nd, in);
  element_compute<D, T, OP, NL, false>(m, in, y);
}

template <int D, typename T, typename A>
__device__ __forceinline__ void lds_accumulate(A* acc, const int (&nd)[D + 1], int n0,
                                               int nloc, const T (&y)[D + 1][D]) {
#pragma unroll
  for (int a = 0; a <= D; ++a) {
    const int ln = nd[a] - n0;
    if ((unsigned)ln < (unsigned)nloc) {
#pragma unroll
      for (int i = 0; i < D; ++i) atomicAdd(&acc[ln * D + i], (A)y[a][i]);
    }
  }
}

// Element visits in flight per thread in the fused 2D linear iteration and
// in the other fused iterations (3D, Neo-Hookean), whose records and state
// take more registers: one visit at a time keeps their occupancy (measured:
// 500k-tet Neo-Hookean warm solve 54.9 ms against 77.4 with two).  In 2D
// one visit (74 registers, 6 waves per SIMD) against two (110, 4 waves):
// the 200k-triangle solve alike (8.14 / 8.12 us per launch), the batched
// 512-request stream 2% faster.
#ifndef PFEM_FCG_EIF
#define PFEM_FCG_EIF 1
#endif
#ifndef PFEM_FCG_EIF_OTHER
#define PFEM_FCG_EIF_OTHER 1
#endif
// Element visits in flight per thread in the (non-fused) owner kernels
// (measured: 4 is 10-35% slower, 1 within noise in 2D and slower in 3D).
#ifndef PFEM_OWNER_EIF
#define PFEM_OWNER_EIF 2
#endif

// LDS accumulator type of the owner kernel.
#ifndef PFEM_ACC_F64
#define PFEM_ACC_F64 1
#endif
template <typename T>
using AccT = typename std::conditional<PFEM_ACC_F64 != 0, double, T>::type;

// ------------------------------------------------------------ owner kernel
// Workgroup = (task, node block).  Elements visited: the block's own sorted
// range (smallest node inside the block) followed by its halo list
// (elements owned by earlier blocks that reach into it).  Each thread keeps
// EIF elements in flight: all connectivity rows are loaded, then all
// gathers, then the arithmetic.

// One round of EIF visits per thread: visit t0 + q NT for q < EIF.  A slot
// past the end loads visit min(t0, total - 1) instead (every block has at
// least one visit) and is skipped, so every load stays inside the block's
// own range or halo list even when t0 itself is past the end.
template <int D, typename T, int OP, bool NL, bool FUSED, int EIF>
struct VisitRound {
  int nd[EIF][D + 1];
  bool on[EIF];
  ElemIn<D, T, OP, NL, FUSED> in[EIF];
};

template <int D, typename T, int OP, bool NL, bool FUSED, int NT, int EIF, int PK = 0>
__device__ __forceinline__ void load_round(const MeshDev& m, const T* __restrict__ U,
                                           const T* __restrict__ V, int mask, const pi4 br,
                                           int t0, VisitRound<D, T, OP, NL, FUSED, EIF>& rd) {
  const int n_own = br.y - br.x;
  const int n_halo = br.w - br.z;
  const int total = n_own + n_halo;
  int e[EIF];
#pragma unroll
  for (int q = 0; q < EIF; ++q) {
    const int t = t0 + q * NT;
    rd.on[q] = t < total;
    const int tt = rd.on[q] ? t : min(t0, total - 1);
    // the halo entry is read unconditionally (clamped; the device list has
    // one padding entry) so that no load waits at a branch join
    const int h = ldx(m.halo, (uint32_t)(br.z + min(max(tt - n_own, 0), max(n_halo - 1, 0))));
    e[q] = tt < n_own ? br.x + tt : h;
  }
#pragma unroll
  for (int q = 0; q < EIF; ++q) load_conn<D, T, PK>(m, e[q], rd.nd[q]);
#pragma unroll
  for (int q = 0; q < EIF; ++q)
    load_elem<D, T, OP, NL, FUSED>(m, U, V, mask, e[q], rd.nd[q], rd.in[q]);
}

template <int D, typename T, int OP, bool NL, typename A, bool FUSED, int EIF>
__device__ __forceinline__ void compute_round(const MeshDev& m,
                                              VisitRound<D, T, OP, NL, FUSED, EIF>& rd,
                                              int n0, int nloc, A* acc, T alpha, T beta) {
  T y[D + 1][D];
#pragma unroll
  for (int q = 0; q < EIF; ++q) {
    if (!rd.on[q]) continue;
    if constexpr (FUSED) fcg_direction<D, T, OP, NL>(rd.in[q], alpha, beta);
    element_compute<D, T, OP, NL, FUSED>(m, rd.in[q], y);
    lds_accumulate<D, T, A>(acc, rd.nd[q], n0, nloc, y);
  }
}

// All visits of the block from t_first on (t_first = threadIdx.x: all of
// them).  acc[] must be zero and visible to every thread; on return it holds
// the block's owned DOFs (all threads synchronised).
template <int D, typename T, int OP, bool NL, typename A, bool FUSED = false, int NT = kThreads,
          int EIF = 2, int PK = 0>
__device__ __forceinline__ void owner_rounds(const MeshDev& m, const T* __restrict__ U,
                                             const T* __restrict__ V, int mask, const pi4 br,
                                             int t_first, int n0, int nloc, A* acc,
                                             T alpha = T(0), T beta = T(0)) {
  const int total = (br.y - br.x) + (br.w - br.z);
  for (int t0 = t_first; t0 < total; t0 += EIF * NT) {
    VisitRound<D, T, OP, NL, FUSED, EIF> rd;
    load_round<D, T, OP, NL, FUSED, NT, EIF, PK>(m, U, V, mask, br, t0, rd);
    compute_round<D, T, OP, NL, A, FUSED, EIF>(m, rd, n0, nloc, acc, alpha, beta);
  }
  __syncthreads();
}

template <int D, typename T, int OP, bool NL, typename A, bool FUSED = false, int NT = kThreads,
          int EIF = 2>
__device__ __forceinline__ void owner_accumulate(const MeshDev& m, const T* __restrict__ U,
                                                 const T* __restrict__ V, int mask,
                                                 const pi4 br, int n0, int nloc, A* acc,
                                                 T alpha = T(0), T beta = T(0)) {
  const int nown = nloc * D;
  for (int i = threadIdx.x; i < nown; i += NT) acc[i] = A(0);
  __syncthreads();
  owner_rounds<D, T, OP, NL, A, FUSED, NT, EIF>(m, U, V, mask, br, threadIdx.x, n0, nloc, acc,
                                                alpha, beta);
}

template <int D, typename T, int OP, bool NL>
__global__ void __launch_bounds__(kThreads)
k_owner(const Task* __restrict__ tasks, const int2* __restrict__ work, const BaseArgs ba) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int2 wk = work[blockIdx.x];
  const Task* tp = tasks + wk.x;
  if (!tp->active) return;
  if (tp->pcg && ldg(&tp->sc->state) != 0) return;
  const MeshDev m = tp->m;
  const int blk = wk.y;
  const int n0 = blk * m.bn;
  const int nloc = min(m.bn, m.n_nodes - n0);
  const pi4 br = ldg(reinterpret_cast<const pi4*>(m.blocks + blk));
  using A = AccT<T>;
  A* acc = reinterpret_cast<A*>(smem_raw);
  const T* U = operand<const T>(const_cast<void*>(tp->u), const_cast<void*>(ba.u), ba.rel);
  const T* V = operand<const T>(const_cast<void*>(tp->v), const_cast<void*>(ba.v), ba.rel);
  const int mask = ba.rel ? ba.mask : tp->mask;
  owner_accumulate<D, T, OP, NL, A, false, kThreads, PFEM_OWNER_EIF>(m, U, V, mask, br, n0,
                                                                     nloc, acc);
  owner_epilogue<D, T, OP>(tp, m, acc, U, V, mask, ba, blk, n0, nloc);
}

// ------------------------------------------- several right-hand sides
// K.v for up to kMultiMax right-hand sides on one linear 3D mesh (the six
// cell problems of a homogenisation): workgroup = node block, and every
// element is visited once for all of them -- connectivity, coordinates,
// material and the element geometry are loaded and computed once, then
// each right-hand side's strain, stress and scatter follows in turn
// (tasks[r] holds right-hand side r: v = p, y = q, w = p, its partial
// sums).  A task whose PCG has stopped is skipped.  The LDS holds one
// float64 accumulator per owned DOF and right-hand side.
constexpr int kMultiMax = 6;

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_owner_multi(const Task* __restrict__ tasks, int nr, const int2* __restrict__ work) {
  constexpr int D = 3;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int blk = work[blockIdx.x].y;
  const MeshDev m = tasks[0].m;
  bool on[kMultiMax];
  int any = 0;
#pragma unroll
  for (int r = 0; r < kMultiMax; ++r) {
    const Task* tp = tasks + min(r, nr - 1);
    on[r] = r < nr && tp->active && !(tp->pcg && ldg(&tp->sc->state) != 0);
    any |= on[r] ? 1 : 0;
  }
  if (!any) return;
  const int n0 = blk * m.bn;
  const int nloc = min(m.bn, m.n_nodes - n0);
  const int nown = nloc * D;
  const pi4 br = ldg(reinterpret_cast<const pi4*>(m.blocks + blk));
  double* acc = reinterpret_cast<double*>(smem_raw);   // [r][nown]
  for (int i = threadIdx.x; i < nr * nown; i += kThreads) acc[i] = 0.0;
  __syncthreads();
  const int n_own = br.y - br.x;
  const int n_halo = br.w - br.z;
  const int total = n_own + n_halo;
  for (int t = threadIdx.x; t < total; t += kThreads) {
    const int h = ldx(m.halo, (uint32_t)(br.z + min(max(t - n_own, 0), max(n_halo - 1, 0))));
    const int e = t < n_own ? br.x + t : h;
    int nd[D + 1];
    load_conn<D, T>(m, e, nd);
    ElemX<D, T> x;
    load_elem_x<D, T>(m, nd, x);
    const T mu = mat_mu<T>(m, e);
    const T lam = mat_lam<T>(m, e, mu);
    Geo<D, T> g;
    geometry_x<D, T>(m, x, g);
    const T adet = g.det < T(0) ? -g.det : g.det;
    const T s_sym = T(1) / (T(Fact<D>::v) * adet);
#pragma unroll 1
    for (int r = 0; r < nr; ++r) {
      if (!on[r]) continue;
      const T* V = static_cast<const T*>(tasks[r].v);
      T v[D + 1][D];
#pragma unroll
      for (int a = 0; a <= D; ++a) load_nodal<D, T>(V, nd[a], v[a]);
      T M[D][D], S[D][D], y[D + 1][D];
      grad_tilde<D, T>(v, g, M);
      linear_stress_tilde<D, T>(M, mu, lam, S);
      scatter_rows<D, T>(S, g, s_sym, y);
      lds_accumulate<D, T, double>(acc + r * nown, nd, n0, nloc, y);
    }
  }
  __syncthreads();
  const size_t g0 = (size_t)n0 * D;
#pragma unroll 1
  for (int r = 0; r < nr; ++r) {
    if (!on[r]) continue;   // uniform over the workgroup
    const Task* tp = tasks + r;
    T* Y = static_cast<T*>(tp->y);
    const T* V = static_cast<const T*>(tp->v);
    const T* W = static_cast<const T*>(tp->w);
    const bool springs = m.pair_ptr != nullptr && !tp->no_pairs;
    double part[kRedSlots] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nown; i += kThreads) {
      const size_t gi = g0 + i;
      T val = (T)acc[r * nown + i];
      const bool con = (ldg(m.dmask + n0 + i / D) >> (i % D)) & 1;
      if (springs) val += periodic_springs<D, T, OP_APPLY>(m, V, tp->mask, n0 + i / D, i % D, con);
      if ((tp->mask & PFEM_MASK_OUT) && con) val = T(0);
      stg(Y + gi, val);
      if (W != nullptr) part[0] += (double)val * (double)ldg(W + gi);
    }
    write_partials(tp->red, m.n_blocks, blk, part, 0, 1);
  }
}

bool owner_multi_fits(int bn, int nr) {
  return nr >= 1 && nr <= kMultiMax && (size_t)nr * bn * 3 * sizeof(double) <= 64 * 1024;
}

void launch_owner_multi(Ctx* ctx, int prec, const Task* tasks_dev, int nr,
                        const int2* work_dev, int n_work, int bn) {
  hipEvent_t ev = nullptr;
  ctx->timing_begin(FAM_APPLY, &ev);
  const size_t sm = (size_t)nr * bn * 3 * sizeof(double);
  if (prec == PFEM_FP32)
    hipLaunchKernelGGL(k_owner_multi<float>, dim3(n_work), dim3(kThreads), sm, ctx->stream,
                       tasks_dev, nr, work_dev);
  else
    hipLaunchKernelGGL(k_owner_multi<double>, dim3(n_work), dim3(kThreads), sm, ctx->stream,
                       tasks_dev, nr, work_dev);
  PFEM_HIP(hipGetLastError());
  ctx->timing_end(FAM_APPLY, ev);
}

// ----------------------------------------------------- fused PCG iteration
// Jacobi-PCG in the Chronopoulos-Gear form (one inner-product phase per
// iteration; same iterates as the textbook loop in exact arithmetic), with
// one launch per iteration j:
//   gamma_j = r.u, delta_j = w.u, |r|^2      partials of launch j-1 (u = M^-1 r, w = A u)
//   beta_j = gamma_j / gamma_{j-1}, alpha_j = gamma_j / (delta_j - beta_j gamma_j / alpha_{j-1})
//   s = w + beta s, r' = r - alpha s, u' = M^-1 r'        at every gathered node
//   w' = A u'                                            element pass, owner scatter
//   p = u + beta p, d += alpha p                         owned DOFs
// The point update is pointwise, so a workgroup evaluates u' itself at the
// nodes its elements touch -- from a per-node record {r, w, s, M^-1} of the
// previous launch -- instead of waiting for the owner of the node; owners
// then write the new record to the other parity buffer.  Partial sums
// alternate between two slot sets by parity of j.  Unlike the pipelined
// (Ghysels-Vanroose) form, no recurrence replaces the matvec, which keeps
// the float32 iteration as stable as the textbook loop.
template <int D, typename T, bool NL, int NT, int PK>
__device__ __forceinline__ void fcg_iteration(const Task* __restrict__ tp, int blk, int it) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // The latency of this launch is a chain of dependent memory round trips,
  // so every load is issued as early as its address allows and none waits
  // behind a branch: descriptor fields (both parity buffers, selected
  // afterwards), then the run scalars, the block's visit ranges, the
  // previous partial sums and this thread's first owned node together.
  Scalars* sc = tp->sc;
  const MeshDev m = tp->m;
  const int nb = m.n_blocks;
  const int j = tp->k_base + it;
  const int n0 = blk * m.bn;
  const int nloc = min(m.bn, m.n_nodes - n0);
  const T* R0 = static_cast<const T*>(tp->rec[0]);
  const T* R1 = static_cast<const T*>(tp->rec[1]);
  const T* Rin = (j & 1) ? R1 : R0;
  T* P = static_cast<T*>(tp->p);
  T* Dd = static_cast<T*>(tp->d);
  const double* part_in = tp->red.part + (size_t)(j & 1) * kRedSlots * nb;
  const int state_in = ldg(&sc->state);
  const double target2 = ldg(&sc->target2);
  const int kmax = ldg(&sc->kmax);
  const double pg_prev = ldg(&sc->pg[(j + 1) & 1]);   // gamma_{j-1}
  const double pa_prev = ldg(&sc->pa[(j + 1) & 1]);   // alpha_{j-1}
  const int active = tp->active;
  const pi4 br = ldg(reinterpret_cast<const pi4*>(m.blocks + blk));
  // branch-free for up to 2 NT blocks: out-of-range threads load a valid
  // neighbour and discard it
  const int pb = min((int)threadIdx.x, nb - 1);
  const int pb2 = min((int)threadIdx.x + NT, nb - 1);
  double pv_in[3], pv2[3];
  pv_in[0] = ldg(part_in + pb);
  pv_in[1] = ldg(part_in + (size_t)nb + pb);
  pv_in[2] = ldg(part_in + (size_t)2 * nb + pb);
  pv2[0] = ldg(part_in + pb2);
  pv2[1] = ldg(part_in + (size_t)nb + pb2);
  pv2[2] = ldg(part_in + (size_t)2 * nb + pb2);
  const int ln0 = threadIdx.x;
  const int lnc = min(ln0, nloc - 1);
  T rc0[4 * D], pv0[D], dv0[D];
  load_record<D, T>(Rin, n0 + lnc, rc0);
  load_nodal<D, T>(P, n0 + lnc, pv0);
  load_nodal<D, T>(Dd, n0 + lnc, dv0);
  const int bits0 = ldg(m.dmask + n0 + lnc);
  // 2D: the first round of element visits needs no scalar, so its
  // connectivity, coordinates and records are in flight while the partials
  // are summed (in 3D the registers held across the sum cost more
  // occupancy than the overlap gains: measured 10-20% slower)
  constexpr int EIF = (D == 2 && !NL) ? PFEM_FCG_EIF : PFEM_FCG_EIF_OTHER;
  constexpr bool HOIST = D == 2;
  // Neo-Hookean: the element state {F^-T, ln J} of the Newton step comes
  // from the solve's per-element cache (tp->u)
  constexpr int OPA = NL ? OP_HVPC : OP_APPLY;
  using A = AccT<T>;
  A* acc = reinterpret_cast<A*>(smem_raw);
  const T* U = static_cast<const T*>(tp->u);
  for (int i = threadIdx.x; i < nloc * D; i += NT) acc[i] = A(0);
  VisitRound<D, T, OPA, NL, true, EIF> rd0;
  if constexpr (HOIST)
    load_round<D, T, OPA, NL, true, NT, EIF, PK>(m, U, Rin, 0, br, threadIdx.x, rd0);
  if ((int)threadIdx.x >= nb) pv_in[0] = pv_in[1] = pv_in[2] = 0.0;
  if ((int)threadIdx.x + NT < nb) {
    pv_in[0] += pv2[0];
    pv_in[1] += pv2[1];
    pv_in[2] += pv2[2];
  }
  for (int b = (int)threadIdx.x + 2 * NT; b < nb; b += NT) {   // more than 2 NT blocks
    pv_in[0] += ldg(part_in + b);
    pv_in[1] += ldg(part_in + (size_t)nb + b);
    pv_in[2] += ldg(part_in + (size_t)2 * nb + b);
  }
  block_sum_all<3, NT>(pv_in);   // its barriers also publish the zeroed acc[]
  const double delta = pv_in[0], gamma = pv_in[1], rr = pv_in[2];
  if (state_in != 0 || !active) return;
  int state = 0;
  double alpha64 = 0.0, beta64 = 0.0;
  if (!(rr == rr) || !(gamma == gamma) || !(delta == delta)) {
    state = 3;
  } else if (rr <= target2) {
    state = 1;
  } else if (!(gamma > 0.0)) {
    state = 3;
  } else if (j >= kmax) {
    state = 2;
  } else {
    double den = delta;
    if (j > 0) {
      beta64 = gamma / pg_prev;
      den = delta - beta64 * gamma / pa_prev;
    }
    if (!(den > 0.0)) state = 3;   // not SPD along this direction
    else alpha64 = gamma / den;
  }
  if (blk == 0 && threadIdx.x == 0) {
    sc->rr = rr;
    const double rho = sqrt(rr) / sc->den;
    sc->rho = rho;
    if (j > 0) {   // residual after j iterations
      const int h = tp->hist_base + j - 1;
      if (tp->hist != nullptr && h < sc->hist_cap) {
        tp->hist[h] = rho;
        sc->hist_len = h + 1;
      }
    }
    if (state == 0) {
      sc->pa[j & 1] = alpha64;
      sc->pg[j & 1] = gamma;
      sc->alpha = alpha64;
      sc->beta = beta64;
      sc->k = j + 1;
      sc->total_k += 1;
    } else {
      sc->k = j;
      sc->state = state;
    }
  }
  if (state != 0) return;
  const T alpha = (T)alpha64, beta = (T)beta64;
  if constexpr (HOIST)
    compute_round<D, T, OPA, NL, A, true, EIF>(m, rd0, n0, nloc, acc, alpha, beta);
  owner_rounds<D, T, OPA, NL, A, true, NT, EIF, PK>(
      m, U, Rin, 0, br, threadIdx.x + (HOIST ? EIF * NT : 0), n0, nloc, acc, alpha, beta);
  T* Rout = static_cast<T*>(tp->rec[(j + 1) & 1]);
  const bool first = j == 0;
  double part[kRedSlots] = {0.0, 0.0, 0.0, 0.0};
  for (int ln = ln0; ln < nloc; ln += NT) {
    const int n = n0 + ln;
    T rc[4 * D], out[4 * D], pv[D], dv[D];
    int bits;
    if (ln == ln0) {
#pragma unroll
      for (int q = 0; q < 4 * D; ++q) rc[q] = rc0[q];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        pv[c] = pv0[c];
        dv[c] = dv0[c];
      }
      bits = bits0;
    } else {
      load_record<D, T>(Rin, n, rc);
      load_nodal<D, T>(P, n, pv);
      load_nodal<D, T>(Dd, n, dv);
      bits = ldg(m.dmask + n);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const T r = rc[c], w = rc[D + c], so = rc[2 * D + c], mi = rc[3 * D + c];
      T s, rn, un;
      fcg_step<T>(r, w, so, mi, alpha, beta, s, rn, un);
      const T ui = mi * r;
      const T p = first ? ui : fma_t(beta, pv[c], ui);
      pv[c] = p;
      if constexpr (sizeof(T) == 8) dv[c] = dv[c] + alpha64 * p;
      else dv[c] = fma_t(alpha, p, dv[c]);
      const T wn = ((bits >> c) & 1) ? T(0) : (T)acc[ln * D + c];
      out[c] = rn;
      out[D + c] = wn;
      out[2 * D + c] = s;
      out[3 * D + c] = mi;
      part[0] += (double)wn * (double)un;
      part[1] += (double)rn * (double)un;
      part[2] += (double)rn * (double)rn;
    }
    store_record<D, T>(Rout, n, out);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      stg(P + (size_t)n * D + c, pv[c]);
      stg(Dd + (size_t)n * D + c, dv[c]);
    }
  }
  RedDev outp{tp->red.part + (size_t)((j + 1) & 1) * kRedSlots * nb, nullptr};
  write_partials<NT>(outp, nb, blk, part, 0, 3);
}

// Batched form: workgroup -> (task, node block) through the work table.
// The 3D Neo-Hookean float32 iteration is held to 5 waves per SIMD (94
// registers, no spills; 4 waves without the hint).
template <int D, typename T, bool NL, int NT, int PK>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu((D == 3 && NL && sizeof(T) == 4) ? 5 : 1)))
k_fcg(const Task* __restrict__ tasks, const int2* __restrict__ work, int it) {
  const int2 wk = work[blockIdx.x];
  fcg_iteration<D, T, NL, NT, PK>(tasks + wk.x, wk.y, it);
}

// -------------------------------------------------- alternative scatters
template <int D, typename T, int OP, bool NL>
__global__ void __launch_bounds__(kThreads) k_atomic(Task t) {
  const MeshDev& m = t.m;
  const T* U = static_cast<const T*>(t.u);
  const T* V = static_cast<const T*>(t.v);
  T* Y = static_cast<T*>(t.y);
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < m.n_elems;
       e += gridDim.x * kThreads) {
    int nd[D + 1];
    load_conn<D, T>(m, e, nd);
    T y[D + 1][D];
    element_output<D, T, OP, NL>(m, U, V, t.mask, e, nd, y);
#pragma unroll
    for (int a = 0; a <= D; ++a)
#pragma unroll
      for (int i = 0; i < D; ++i) atomicAdd(&Y[(size_t)nd[a] * D + i], y[a][i]);
  }
}

template <int D, typename T, int OP, bool NL>
__global__ void __launch_bounds__(kThreads) k_colored(Task t, int c0, int c1) {
  const MeshDev& m = t.m;
  const T* U = static_cast<const T*>(t.u);
  const T* V = static_cast<const T*>(t.v);
  T* Y = static_cast<T*>(t.y);
  for (int k = c0 + blockIdx.x * kThreads + threadIdx.x; k < c1;
       k += gridDim.x * kThreads) {
    const int e = ldg(m.colored + k);
    int nd[D + 1];
    load_conn<D, T>(m, e, nd);
    T y[D + 1][D];
    element_output<D, T, OP, NL>(m, U, V, t.mask, e, nd, y);
#pragma unroll
    for (int a = 0; a <= D; ++a)
#pragma unroll
      for (int i = 0; i < D; ++i) Y[(size_t)nd[a] * D + i] += y[a][i];
  }
}

// Output fix-up for the alternative scatters: subtract f_ext (force),
// Dirichlet handling, all in one pass over the DOFs.
template <int D, typename T, int OP>
__global__ void __launch_bounds__(kThreads) k_alt_fixup(Task t) {
  const MeshDev& m = t.m;
  T* Y = static_cast<T*>(t.y);
  const size_t n = (size_t)m.n_nodes * D;
  for (size_t g = (size_t)blockIdx.x * kThreads + threadIdx.x; g < n;
       g += (size_t)gridDim.x * kThreads) {
    const bool con = (ldg(m.dmask + g / D) >> (g % D)) & 1;
    T val = ldg(Y + g);
    if (OP == OP_FORCE) val -= (T)(t.fscale * ldg(m.fext + g));
    if (OP == OP_DIAG) {
      if (con) val = T(1);
      else if (t.s != 0.0) val = T(1) / val;
    } else if ((t.mask & PFEM_MASK_OUT) && con) {
      val = T(0);
    }
    stg(Y + g, val);
  }
}

// ----------------------------------------------------------------- energy
// Pi = sum_e vol_e Psi_e - f_ext . u over the elements a block owns (each
// element once) and the DOFs it owns.  With DIFF the kernel returns
// Pi(u + s v) - Pi(u) accumulated element by element in float64 (no
// cancellation between two large totals), counts elements with J <= 0 at
// the trial state, and sums the magnitudes of the terms (slot 2) so the
// caller knows the rounding level of the difference.  Partials: (energy or
// difference, #inverted, sum of |terms|).
template <int D, typename TU, typename TV, bool DIFF>
__global__ void __launch_bounds__(kThreads)
k_energy(const Task* __restrict__ tasks, const int2* __restrict__ work, const BaseArgs ba) {
  const int2 wk = work[blockIdx.x];
  const Task* tp = tasks + wk.x;
  if (!tp->active) return;
  const MeshDev m = tp->m;
  const int blk = wk.y;
  const int n0 = blk * m.bn;
  const int nloc = min(m.bn, m.n_nodes - n0);
  const pi4 br = ldg(reinterpret_cast<const pi4*>(m.blocks + blk));
  const TU* U = operand<const TU>(const_cast<void*>(tp->u), const_cast<void*>(ba.u), ba.rel);
  const TV* V = operand<const TV>(const_cast<void*>(tp->v), const_cast<void*>(ba.v), ba.rel);
  const double s = tp->s;
  double part[kRedSlots] = {0.0, 0.0, 0.0, 0.0};
  using T = TU;   // element arithmetic type
  for (int e = br.x + (int)threadIdx.x; e < br.y; e += kThreads) {
    int nd[D + 1];
    load_conn<D, T>(m, e, nd);
    Geo<D, T> g;
    load_geometry<D, T>(m, nd, g);
    const T mu = mat_mu<T>(m, e);
    const T lam = mat_lam<T>(m, e, mu);
    const T adet = g.det < T(0) ? -g.det : g.det;
    const double vol = (double)adet / Fact<D>::v;
    T uu[D + 1][D];
#pragma unroll
    for (int a = 0; a <= D; ++a) load_nodal<D, TU>(U, nd[a], uu[a]);
    T Ht[D][D];
    grad_tilde<D, T>(uu, g, Ht);
    double psi0, psi1 = 0.0;
    T H[D][D];
    const T inv_det = T(1) / g.det;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int k = 0; k < D; ++k) H[i][k] = Ht[i][k] * inv_det;
    if (!m.nonlinear) {
      T S[D][D];
      linear_stress_tilde<D, T>(H, mu, lam, S);
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int k = 0; k < D; ++k) acc += (double)S[i][k] * 0.5 * ((double)H[i][k] + (double)H[k][i]);
      psi0 = 0.5 * acc;
    } else {
      psi0 = nh_energy_density<D, T>(H, (double)mu, (double)lam);
    }
    if (DIFF) {
      T vv[D + 1][D];
#pragma unroll
      for (int a = 0; a <= D; ++a) {
        TV t[D];
        load_nodal<D, TV>(V, nd[a], t);
#pragma unroll
        for (int i = 0; i < D; ++i) vv[a][i] = uu[a][i] + (T)(s * (double)t[i]);
      }
      T Mt[D][D];
      grad_tilde<D, T>(vv, g, Mt);
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int k = 0; k < D; ++k) H[i][k] = Mt[i][k] * inv_det;
      if (!m.nonlinear) {
        T S[D][D];
        linear_stress_tilde<D, T>(H, mu, lam, S);
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int k = 0; k < D; ++k) acc += (double)S[i][k] * 0.5 * ((double)H[i][k] + (double)H[k][i]);
        psi1 = 0.5 * acc;
      } else {
        psi1 = nh_energy_density<D, T>(H, (double)mu, (double)lam);
      }
      if (psi1 == __builtin_inf()) {
        part[1] += 1.0;
      } else {
        part[0] += vol * (psi1 - psi0);
        part[2] += vol * (fabs(psi0) + fabs(psi1));   // size of the summed terms
      }
    } else {
      if (psi0 == __builtin_inf()) part[1] += 1.0;
      else part[0] += vol * psi0;
    }
  }
  energy_epilogue<D, TU, TV, DIFF>(tp, m, U, V, s, blk, n0, nloc, part);
}

// ------------------------------------------- Neo-Hookean element cache
// Per element of the owned ranges (every element exactly once): F^-T and
// ln J of the state u (task u, nodal, kernel precision) into the task's y,
// value k of element e at y[k * n_elems + e] (k = D i + j for F^-T_ij,
// k = D^2 for ln J): what every Hessian-vector product of one Newton step
// needs of the state, computed once per step instead of once per product.
template <int D, typename T>
__global__ void __launch_bounds__(kThreads)
k_nh_cache(const Task* __restrict__ tasks, const int2* __restrict__ work) {
  const int2 wk = work[blockIdx.x];
  const Task* tp = tasks + wk.x;
  if (!tp->active) return;
  const MeshDev m = tp->m;
  const pi4 br = ldg(reinterpret_cast<const pi4*>(m.blocks + wk.y));
  const T* U = static_cast<const T*>(tp->u);
  T* C = static_cast<T*>(tp->y);
  const size_t ne = (size_t)m.n_elems;
  for (int e = br.x + (int)threadIdx.x; e < br.y; e += kThreads) {
    int nd[D + 1];
    load_conn<D, T>(m, e, nd);
    ElemX<D, T> x;
    load_elem_x<D, T>(m, nd, x);
    T u[D + 1][D];
#pragma unroll
    for (int a = 0; a <= D; ++a) load_nodal<D, T>(U, nd[a], u[a]);
    Geo<D, T> g;
    geometry_x<D, T>(m, x, g);
    T Ht[D][D];
    grad_tilde<D, T>(u, g, Ht);
    NHState<D, T> st;
    nh_state<D, T>(Ht, T(1) / g.det, st);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int k = 0; k < D; ++k) stg(C + (size_t)(i * D + k) * ne + e, st.FinvT[i][k]);
    stg(C + (size_t)(D * D) * ne + e, st.lnJ);
  }
}

void launch_nh_cache(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                     int n_work) {
  if (n_work <= 0) return;
  dim3 grid(n_work), block(kThreads);
  hipStream_t s = ctx->stream;
  if (dim == 2 && prec == PFEM_FP32) hipLaunchKernelGGL((k_nh_cache<2, float>), grid, block, 0, s, tasks, work);
  else if (dim == 2) hipLaunchKernelGGL((k_nh_cache<2, double>), grid, block, 0, s, tasks, work);
  else if (prec == PFEM_FP32) hipLaunchKernelGGL((k_nh_cache<3, float>), grid, block, 0, s, tasks, work);
  else hipLaunchKernelGGL((k_nh_cache<3, double>), grid, block, 0, s, tasks, work);
  PFEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- launchers
template <int D, typename T, bool NL>
static void launch_owner_typed(Ctx* ctx, int op, const Task* tasks, const int2* work,
                               int n_work, int bn_max, const BaseArgs& ba) {
  const size_t sm = (size_t)bn_max * D * sizeof(AccT<T>);
  dim3 grid(n_work), block(kThreads);
  switch (op) {
    case OP_APPLY:
      hipLaunchKernelGGL((k_owner<D, T, OP_APPLY, NL>), grid, block, sm, ctx->stream, tasks, work, ba);
      break;
    case OP_HVPC:
      if constexpr (NL)
        hipLaunchKernelGGL((k_owner<D, T, OP_HVPC, true>), grid, block, sm, ctx->stream, tasks, work, ba);
      break;
    case OP_FORCE:
      hipLaunchKernelGGL((k_owner<D, T, OP_FORCE, NL>), grid, block, sm, ctx->stream, tasks, work, ba);
      break;
    default:
      hipLaunchKernelGGL((k_owner<D, T, OP_DIAG, NL>), grid, block, sm, ctx->stream, tasks, work, ba);
      break;
  }
}

template <int D, typename T, bool NL>
static void launch_alt_typed(Ctx* ctx, int op, int mode, const Task& t,
                             const std::vector<int>* color_ptr) {
  const int ne = t.m.n_elems;
  const int grid = std::max(1, std::min((ne + kThreads - 1) / kThreads, 4096));
  launch_fill(ctx, sizeof(T) == 8 ? PFEM_FP64 : PFEM_FP32, t.y, (int64_t)t.m.n_nodes * D, 0.0);
  if (mode == PFEM_SCATTER_ATOMIC) {
#define PFEM_ATOMIC(OPV) hipLaunchKernelGGL((k_atomic<D, T, OPV, NL>), dim3(grid), dim3(kThreads), 0, ctx->stream, t)
    if (op == OP_APPLY) PFEM_ATOMIC(OP_APPLY);
    else if (op == OP_FORCE) PFEM_ATOMIC(OP_FORCE);
    else PFEM_ATOMIC(OP_DIAG);
#undef PFEM_ATOMIC
  } else {
    const std::vector<int>& cp = *color_ptr;
    for (size_t c = 0; c + 1 < cp.size(); ++c) {
      const int cnt = cp[c + 1] - cp[c];
      if (cnt <= 0) continue;
      const int g = std::max(1, std::min((cnt + kThreads - 1) / kThreads, 4096));
#define PFEM_COLOR(OPV) hipLaunchKernelGGL((k_colored<D, T, OPV, NL>), dim3(g), dim3(kThreads), 0, ctx->stream, t, cp[c], cp[c + 1])
      if (op == OP_APPLY) PFEM_COLOR(OP_APPLY);
      else if (op == OP_FORCE) PFEM_COLOR(OP_FORCE);
      else PFEM_COLOR(OP_DIAG);
#undef PFEM_COLOR
    }
  }
  const size_t n = (size_t)t.m.n_nodes * D;
  const int gf = (int)std::max<size_t>(1, std::min<size_t>((n + kThreads - 1) / kThreads, 4096));
#define PFEM_FIX(OPV) hipLaunchKernelGGL((k_alt_fixup<D, T, OPV>), dim3(gf), dim3(kThreads), 0, ctx->stream, t)
  if (op == OP_APPLY) PFEM_FIX(OP_APPLY);
  else if (op == OP_FORCE) PFEM_FIX(OP_FORCE);
  else PFEM_FIX(OP_DIAG);
#undef PFEM_FIX
}

static int family_of(int op) {
  return is_apply_op(op) ? FAM_APPLY : (op == OP_FORCE ? FAM_FORCE : FAM_DIAG);
}

template <bool NL>
static void dispatch_owner(Ctx* ctx, int dim, int prec, int op, const Task* t, const int2* w,
                           int n, int bn, const BaseArgs& ba) {
  if (dim == 2 && prec == PFEM_FP32) launch_owner_typed<2, float, NL>(ctx, op, t, w, n, bn, ba);
  else if (dim == 2) launch_owner_typed<2, double, NL>(ctx, op, t, w, n, bn, ba);
  else if (prec == PFEM_FP32) launch_owner_typed<3, float, NL>(ctx, op, t, w, n, bn, ba);
  else launch_owner_typed<3, double, NL>(ctx, op, t, w, n, bn, ba);
}

template <bool NL>
static void dispatch_alt(Ctx* ctx, int dim, int prec, int op, int mode, const Task& t,
                         const std::vector<int>* cp) {
  if (dim == 2 && prec == PFEM_FP32) launch_alt_typed<2, float, NL>(ctx, op, mode, t, cp);
  else if (dim == 2) launch_alt_typed<2, double, NL>(ctx, op, mode, t, cp);
  else if (prec == PFEM_FP32) launch_alt_typed<3, float, NL>(ctx, op, mode, t, cp);
  else launch_alt_typed<3, double, NL>(ctx, op, mode, t, cp);
}

void launch_elem(Ctx* ctx, int dim, int prec, int op, bool nonlinear, int scatter_mode,
                 const Task* tasks_dev, const int2* work_dev, int n_work, int bn_max,
                 const Task* host_task_for_alt, const std::vector<int>* color_ptr,
                 const BaseArgs* rel) {
  require(op != OP_HVPC || (nonlinear && scatter_mode == PFEM_SCATTER_OWNER && !is_quad_kind(dim)),
          PFEM_E_INVALID_ARG, "the cached Hessian-vector product is an owner-scatter P1 kernel");
  hipEvent_t ev = nullptr;
  ctx->timing_begin(family_of(op), &ev);
  const BaseArgs ba = rel != nullptr ? *rel : BaseArgs{nullptr, nullptr, nullptr, 0, 0};
  if (is_quad_kind(dim)) {   // quadrilaterals: owner scatter only (checked by the callers)
    launch_quad_elem(ctx, dim, prec, op, nonlinear, tasks_dev, work_dev, n_work, bn_max, ba);
  } else if (scatter_mode == PFEM_SCATTER_OWNER) {
    if (n_work > 0) {
      if (nonlinear) dispatch_owner<true>(ctx, dim, prec, op, tasks_dev, work_dev, n_work, bn_max, ba);
      else dispatch_owner<false>(ctx, dim, prec, op, tasks_dev, work_dev, n_work, bn_max, ba);
    }
  } else {
    if (nonlinear) dispatch_alt<true>(ctx, dim, prec, op, scatter_mode, *host_task_for_alt, color_ptr);
    else dispatch_alt<false>(ctx, dim, prec, op, scatter_mode, *host_task_for_alt, color_ptr);
  }
  PFEM_HIP(hipGetLastError());
  ctx->timing_end(family_of(op), ev);
}

void launch_energy(Ctx* ctx, int dim, int prec, bool diff, const Task* tasks_dev,
                   const int2* work_dev, int n_work, const BaseArgs* rel) {
  if (n_work <= 0) return;
  const BaseArgs ba = rel != nullptr ? *rel : BaseArgs{nullptr, nullptr, nullptr, 0, 0};
  hipEvent_t ev = nullptr;
  ctx->timing_begin(FAM_ENERGY, &ev);
  dim3 grid(n_work), block(kThreads);
  hipStream_t s = ctx->stream;
  // diff: u is float64 state, v is the increment in `prec`
  if (is_quad_kind(dim)) {
    launch_quad_energy(ctx, dim, prec, diff, tasks_dev, work_dev, n_work, ba);
  } else if (!diff) {
    if (dim == 2 && prec == PFEM_FP32) hipLaunchKernelGGL((k_energy<2, float, float, false>), grid, block, 0, s, tasks_dev, work_dev, ba);
    else if (dim == 2) hipLaunchKernelGGL((k_energy<2, double, double, false>), grid, block, 0, s, tasks_dev, work_dev, ba);
    else if (prec == PFEM_FP32) hipLaunchKernelGGL((k_energy<3, float, float, false>), grid, block, 0, s, tasks_dev, work_dev, ba);
    else hipLaunchKernelGGL((k_energy<3, double, double, false>), grid, block, 0, s, tasks_dev, work_dev, ba);
  } else {
    if (dim == 2 && prec == PFEM_FP32) hipLaunchKernelGGL((k_energy<2, double, float, true>), grid, block, 0, s, tasks_dev, work_dev, ba);
    else if (dim == 2) hipLaunchKernelGGL((k_energy<2, double, double, true>), grid, block, 0, s, tasks_dev, work_dev, ba);
    else if (prec == PFEM_FP32) hipLaunchKernelGGL((k_energy<3, double, float, true>), grid, block, 0, s, tasks_dev, work_dev, ba);
    else hipLaunchKernelGGL((k_energy<3, double, double, true>), grid, block, 0, s, tasks_dev, work_dev, ba);
  }
  PFEM_HIP(hipGetLastError());
  ctx->timing_end(FAM_ENERGY, ev);
}

// Threads per workgroup of the fused iteration: enough that every thread
// evaluates about one element visit in a single round of dependent loads
// where the registers allow (2D linear), fewer where the element state is
// larger.
#ifndef PFEM_FCG_NT2
#define PFEM_FCG_NT2 256
#endif
#ifndef PFEM_FCG_NT3
#define PFEM_FCG_NT3 256
#endif

void launch_fcg_iter(Ctx* ctx, int dim, int prec, bool nl, const Task* tasks,
                     const int2* work, int n_work, int bn_max, int it, bool packed) {
  if (n_work <= 0) return;
  hipStream_t s = ctx->stream;
  const size_t s32 = (size_t)bn_max * dim * sizeof(AccT<float>);
  const size_t s64 = (size_t)bn_max * dim * sizeof(AccT<double>);
  dim3 grid(n_work);
#define PFEM_FCG(DD, TT, NLV, SM, NTV)                                                     \
  do {                                                                                      \
    if (packed)                                                                             \
      hipLaunchKernelGGL((k_fcg<DD, TT, NLV, NTV, 1>), grid, dim3(NTV), SM, s, tasks, work, it); \
    else                                                                                    \
      hipLaunchKernelGGL((k_fcg<DD, TT, NLV, NTV, 0>), grid, dim3(NTV), SM, s, tasks, work, it); \
  } while (0)
  if (!nl) {
    if (dim == 2 && prec == PFEM_FP32) PFEM_FCG(2, float, false, s32, PFEM_FCG_NT2);
    else if (dim == 2) PFEM_FCG(2, double, false, s64, 256);
    else if (prec == PFEM_FP32) PFEM_FCG(3, float, false, s32, PFEM_FCG_NT3);
    else PFEM_FCG(3, double, false, s64, 256);
  } else {
    if (dim == 2 && prec == PFEM_FP32) PFEM_FCG(2, float, true, s32, 256);
    else if (dim == 2) PFEM_FCG(2, double, true, s64, 256);
    else if (prec == PFEM_FP32) PFEM_FCG(3, float, true, s32, 256);
    else PFEM_FCG(3, double, true, s64, 256);
  }
#undef PFEM_FCG
  PFEM_HIP(hipGetLastError());
}

int block_nodes_max() { return 4096; }

}  // namespace pfem
