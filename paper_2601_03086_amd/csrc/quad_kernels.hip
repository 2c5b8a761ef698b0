// Element kernels on quadrilaterals: Q4 (bilinear, 2 x 2 Gauss points) and
// Q8 (serendipity, 3 x 3), K.v / Hessian-vector product, internal force,
// Jacobi diagonal and energy, linear plane stress / strain and Neo-Hookean
// plane strain (Sec. 'Nonlinear hyperelasticity': the beam and Cook's
// membrane; App. B: isoparametric interpolation, f_int = sum over points of
// w |det J| P dN/dX).
//
// Same owner-computes scatter as the P1 kernels (one workgroup per node
// block, the block's own element range plus its halo list, LDS
// accumulation of the owned DOFs, one coalesced write of every owned DOF)
// and the same epilogues (owner_common.h).  Per element the Gauss points
// run in a loop: at each, the Jacobian of the map from the element's
// coordinates relative to its first node (evaluated in float64, then
// rounded to the kernel type), dN/dX = J^-T dN/dxi, and the point's
// contribution w |det J| S dN_a/dX to every node a.  The constitutive math
// (linear stress, Neo-Hookean state, Piola stress and its derivative) is
// the P1 kernels' own, fed the displacement gradient at the point.
#include "elem_math.h"
#include "owner_common.h"
#include "pfem_internal.h"
#include "reduce.h"

namespace pfem {

namespace {

template <int NV>
struct QuadRule {
  static constexpr int NQ1 = NV == 4 ? 2 : 3;   // points per direction
  static constexpr int NQ = NQ1 * NQ1;
};

// Gauss point k of the 1D rule (2 or 3 points) and its weight.
template <int NQ1>
__device__ __forceinline__ void gauss_1d(int k, double& x, double& w) {
  if constexpr (NQ1 == 2) {
    x = k == 0 ? -0.57735026918962576451 : 0.57735026918962576451;
    w = 1.0;
  } else {
    x = k == 0 ? -0.77459666924148337704 : (k == 1 ? 0.0 : 0.77459666924148337704);
    w = k == 1 ? 8.0 / 9.0 : 5.0 / 9.0;
  }
}

// dN_a/dxi, dN_a/deta at (xi, eta): corners (-1,-1), (1,-1), (1,1), (-1,1),
// then (Q8) the midsides of edges (0,1), (1,2), (2,3), (3,0).
template <int NV, typename T>
__device__ __forceinline__ void shape_derivs(T xi, T eta, T (&dN)[NV][2]) {
  const T cx[4] = {T(-1), T(1), T(1), T(-1)};
  const T cy[4] = {T(-1), T(-1), T(1), T(1)};
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const T p = T(1) + xi * cx[a], q = T(1) + eta * cy[a];
    if constexpr (NV == 4) {
      dN[a][0] = T(0.25) * cx[a] * q;
      dN[a][1] = T(0.25) * cy[a] * p;
    } else {   // N = p q (xi cx + eta cy - 1) / 4
      const T r = xi * cx[a] + eta * cy[a] - T(1);
      dN[a][0] = T(0.25) * cx[a] * q * (r + p);
      dN[a][1] = T(0.25) * cy[a] * p * (r + q);
    }
  }
  if constexpr (NV == 8) {
    dN[4][0] = -xi * (T(1) - eta);
    dN[4][1] = T(-0.5) * (T(1) - xi * xi);
    dN[5][0] = T(0.5) * (T(1) - eta * eta);
    dN[5][1] = -(T(1) + xi) * eta;
    dN[6][0] = -xi * (T(1) + eta);
    dN[6][1] = T(0.5) * (T(1) - xi * xi);
    dN[7][0] = T(-0.5) * (T(1) - eta * eta);
    dN[7][1] = -(T(1) - xi) * eta;
  }
}

// Gauss point q of the element: G[a] = dN_a/dX and the weight w |det J|.
// xr: node coordinates relative to node 0 (a translation does not change J).
template <int NV, typename T>
__device__ __forceinline__ void point_geometry(const T (&xr)[NV][2], int q, T (&G)[NV][2],
                                               T& wdet) {
  constexpr int NQ1 = QuadRule<NV>::NQ1;
  double xi, eta, wx, wy;
  gauss_1d<NQ1>(q / NQ1, xi, wx);
  gauss_1d<NQ1>(q % NQ1, eta, wy);
  T dN[NV][2];
  shape_derivs<NV, T>((T)xi, (T)eta, dN);
  T J[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
#pragma unroll
  for (int a = 1; a < NV; ++a)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < 2; ++k) J[i][k] += xr[a][i] * dN[a][k];
  const T det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const T inv = T(1) / det;
  // J^-1 = [[J11, -J01], [-J10, J00]] / det; G_a,i = sum_k dN_a,k Jinv_k,i
  const T Ji00 = J[1][1] * inv, Ji01 = -J[0][1] * inv;
  const T Ji10 = -J[1][0] * inv, Ji11 = J[0][0] * inv;
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    G[a][0] = dN[a][0] * Ji00 + dN[a][1] * Ji10;
    G[a][1] = dN[a][0] * Ji01 + dN[a][1] * Ji11;
  }
  wdet = (T)(wx * wy) * (det < T(0) ? -det : det);
}

// H_ij = sum_a v_a,i G_a,j
template <int NV, typename T>
__device__ __forceinline__ void point_grad(const T (&v)[NV][2], const T (&G)[NV][2],
                                           T (&H)[2][2]) {
  H[0][0] = H[0][1] = H[1][0] = H[1][1] = T(0);
#pragma unroll
  for (int a = 0; a < NV; ++a)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) H[i][j] += v[a][i] * G[a][j];
}

// y_a,i += w sum_j S_ij G_a,j
template <int NV, typename T>
__device__ __forceinline__ void point_scatter(const T (&S)[2][2], const T (&G)[NV][2], T w,
                                              T (&y)[NV][2]) {
#pragma unroll
  for (int a = 0; a < NV; ++a)
#pragma unroll
    for (int i = 0; i < 2; ++i) y[a][i] += w * (S[i][0] * G[a][0] + S[i][1] * G[a][1]);
}

template <int NV, typename T>
struct QuadIn {
  int nd[NV];
  T xr[NV][2];
  T u[NV][2];
  T v[NV][2];
  T mu, lam;
};

template <int NV, typename T, int OP, bool NL>
__device__ __forceinline__ void quad_load(const MeshDev& m, const T* __restrict__ U,
                                          const T* __restrict__ V, int mask, int e,
                                          QuadIn<NV, T>& in) {
#pragma unroll
  for (int a = 0; a < NV; ++a) in.nd[a] = ldg(m.conn + (size_t)e * NV + a);
  const double x0 = ldg(m.X + (size_t)in.nd[0] * 2), y0 = ldg(m.X + (size_t)in.nd[0] * 2 + 1);
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    in.xr[a][0] = (T)(ldg(m.X + (size_t)in.nd[a] * 2) - x0);
    in.xr[a][1] = (T)(ldg(m.X + (size_t)in.nd[a] * 2 + 1) - y0);
  }
  if (sizeof(T) == 8) {
    in.mu = (T)ldg(m.mu64 + e);
    in.lam = m.lam_uniform ? in.mu * (T)m.lam_ratio : (T)ldg(m.lam64 + e);
  } else {
    in.mu = (T)ldg(m.mu32 + e);
    in.lam = m.lam_uniform ? in.mu * (T)m.lam_ratio : (T)ldg(m.lam32 + e);
  }
  if constexpr (NL || OP == OP_FORCE) {
#pragma unroll
    for (int a = 0; a < NV; ++a)
#pragma unroll
      for (int i = 0; i < 2; ++i) in.u[a][i] = ldg(U + (size_t)in.nd[a] * 2 + i);
  }
  if constexpr (OP == OP_APPLY) {
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      const int bits = (mask & PFEM_MASK_IN) ? (int)ldg(m.dmask + in.nd[a]) : 0;
#pragma unroll
      for (int i = 0; i < 2; ++i)
        in.v[a][i] = (bits >> i) & 1 ? T(0) : ldg(V + (size_t)in.nd[a] * 2 + i);
    }
  }
}

// The element's contributions y[a][i] for one op, summed over its points.
template <int NV, typename T, int OP, bool NL>
__device__ __forceinline__ void quad_compute(const QuadIn<NV, T>& in, T (&y)[NV][2]) {
#pragma unroll
  for (int a = 0; a < NV; ++a) y[a][0] = y[a][1] = T(0);
  const T mu = in.mu, lam = in.lam;
  for (int q = 0; q < QuadRule<NV>::NQ; ++q) {
    T G[NV][2], w;
    point_geometry<NV, T>(in.xr, q, G, w);
    if constexpr (OP == OP_DIAG) {
      if constexpr (!NL) {
#pragma unroll
        for (int a = 0; a < NV; ++a) {
          const T n2 = G[a][0] * G[a][0] + G[a][1] * G[a][1];
#pragma unroll
          for (int i = 0; i < 2; ++i) y[a][i] += w * (mu * n2 + (lam + mu) * G[a][i] * G[a][i]);
        }
      } else {
        T H[2][2];
        point_grad<NV, T>(in.u, G, H);
        NHState<2, T> st;
        nh_state<2, T>(H, T(1), st);
        const T coef = lam + mu - lam * st.lnJ;
#pragma unroll
        for (int a = 0; a < NV; ++a) {
          const T n2 = G[a][0] * G[a][0] + G[a][1] * G[a][1];
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const T wi = st.FinvT[i][0] * G[a][0] + st.FinvT[i][1] * G[a][1];
            y[a][i] += w * (mu * n2 + coef * wi * wi);
          }
        }
      }
    } else if constexpr (!NL) {
      T M[2][2], S[2][2];
      if constexpr (OP == OP_APPLY) point_grad<NV, T>(in.v, G, M);
      else point_grad<NV, T>(in.u, G, M);
      linear_stress_tilde<2, T>(M, mu, lam, S);
      point_scatter<NV, T>(S, G, w, y);
    } else {
      T H[2][2];
      point_grad<NV, T>(in.u, G, H);
      NHState<2, T> st;
      nh_state<2, T>(H, T(1), st);
      T P[2][2];
      if constexpr (OP == OP_FORCE) {
        nh_piola<2, T>(st, mu, lam, P);
      } else {
        T dF[2][2];
        point_grad<NV, T>(in.v, G, dF);
        nh_dpiola<2, T>(st, mu, lam, dF, P);
      }
      point_scatter<NV, T>(P, G, w, y);
    }
  }
}

}  // namespace

template <int NV, typename T, int OP, bool NL>
__global__ void __launch_bounds__(kThreads)
k_owner_quad(const Task* __restrict__ tasks, const int2* __restrict__ work, const BaseArgs ba) {
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
  using A = double;
  A* acc = reinterpret_cast<A*>(smem_raw);
  const T* U = operand<const T>(const_cast<void*>(tp->u), const_cast<void*>(ba.u), ba.rel);
  const T* V = operand<const T>(const_cast<void*>(tp->v), const_cast<void*>(ba.v), ba.rel);
  const int mask = ba.rel ? ba.mask : tp->mask;
  for (int i = threadIdx.x; i < nloc * 2; i += kThreads) acc[i] = A(0);
  __syncthreads();
  const int n_own = br.y - br.x;
  const int total = n_own + (br.w - br.z);
  for (int t = threadIdx.x; t < total; t += kThreads) {
    const int e = t < n_own ? br.x + t : ldg(m.halo + br.z + (t - n_own));
    QuadIn<NV, T> in;
    quad_load<NV, T, OP, NL>(m, U, V, mask, e, in);
    T y[NV][2];
    quad_compute<NV, T, OP, NL>(in, y);
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      const int ln = in.nd[a] - n0;
      if ((unsigned)ln < (unsigned)nloc) {
        atomicAdd(&acc[ln * 2], (A)y[a][0]);
        atomicAdd(&acc[ln * 2 + 1], (A)y[a][1]);
      }
    }
  }
  __syncthreads();
  owner_epilogue<2, T, OP>(tp, m, acc, U, V, mask, ba, blk, n0, nloc);
}

// Strain energy density at a point (float64 accumulation of the kernel-type
// gradient): linear 1/2 sigma : eps, Neo-Hookean as the P1 kernels.
template <typename T>
__device__ __forceinline__ double point_psi(const T (&H)[2][2], T mu, T lam, bool nl) {
  if (!nl) {
    T S[2][2];
    linear_stress_tilde<2, T>(H, mu, lam, S);
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < 2; ++k)
        acc += (double)S[i][k] * 0.5 * ((double)H[i][k] + (double)H[k][i]);
    return 0.5 * acc;
  }
  return nh_energy_density<2, T>(H, (double)mu, (double)lam);
}

// Energy of the elements a block owns (each once) and of its owned DOFs;
// with DIFF the change Pi(u + s v) - Pi(u) point by point (see k_energy).
template <int NV, typename TU, typename TV, bool DIFF>
__global__ void __launch_bounds__(kThreads)
k_energy_quad(const Task* __restrict__ tasks, const int2* __restrict__ work, const BaseArgs ba) {
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
  using T = TU;
  const bool nl = m.nonlinear != 0;
  for (int e = br.x + (int)threadIdx.x; e < br.y; e += kThreads) {
    QuadIn<NV, T> in;
    quad_load<NV, T, OP_FORCE, false>(m, U, nullptr, 0, e, in);   // coordinates, material, u
    T vv[NV][2];
    if (DIFF) {
#pragma unroll
      for (int a = 0; a < NV; ++a)
#pragma unroll
        for (int i = 0; i < 2; ++i)
          vv[a][i] = in.u[a][i] + (T)(s * (double)ldg(V + (size_t)in.nd[a] * 2 + i));
    }
    for (int q = 0; q < QuadRule<NV>::NQ; ++q) {
      T G[NV][2], w;
      point_geometry<NV, T>(in.xr, q, G, w);
      T H[2][2];
      point_grad<NV, T>(in.u, G, H);
      const double psi0 = point_psi<T>(H, in.mu, in.lam, nl);
      if (DIFF) {
        point_grad<NV, T>(vv, G, H);
        const double psi1 = point_psi<T>(H, in.mu, in.lam, nl);
        if (psi1 == __builtin_inf()) {
          part[1] += 1.0;
        } else {
          part[0] += (double)w * (psi1 - psi0);
          part[2] += (double)w * (fabs(psi0) + fabs(psi1));
        }
      } else {
        if (psi0 == __builtin_inf()) part[1] += 1.0;
        else part[0] += (double)w * psi0;
      }
    }
  }
  energy_epilogue<2, TU, TV, DIFF>(tp, m, U, V, s, blk, n0, nloc, part);
}

// ---------------------------------------------------------------- launchers
template <int NV, typename T, bool NL>
static void launch_quad_typed(Ctx* ctx, int op, const Task* tasks, const int2* work, int n_work,
                              int bn_max, const BaseArgs& ba) {
  const size_t sm = (size_t)bn_max * 2 * sizeof(double);
  dim3 grid(n_work), block(kThreads);
  if (op == OP_APPLY)
    hipLaunchKernelGGL((k_owner_quad<NV, T, OP_APPLY, NL>), grid, block, sm, ctx->stream, tasks,
                       work, ba);
  else if (op == OP_FORCE)
    hipLaunchKernelGGL((k_owner_quad<NV, T, OP_FORCE, NL>), grid, block, sm, ctx->stream, tasks,
                       work, ba);
  else
    hipLaunchKernelGGL((k_owner_quad<NV, T, OP_DIAG, NL>), grid, block, sm, ctx->stream, tasks,
                       work, ba);
}

template <int NV>
static void launch_quad_nv(Ctx* ctx, int prec, int op, bool nl, const Task* tasks,
                           const int2* work, int n_work, int bn_max, const BaseArgs& ba) {
  if (prec == PFEM_FP32) {
    if (nl) launch_quad_typed<NV, float, true>(ctx, op, tasks, work, n_work, bn_max, ba);
    else launch_quad_typed<NV, float, false>(ctx, op, tasks, work, n_work, bn_max, ba);
  } else {
    if (nl) launch_quad_typed<NV, double, true>(ctx, op, tasks, work, n_work, bn_max, ba);
    else launch_quad_typed<NV, double, false>(ctx, op, tasks, work, n_work, bn_max, ba);
  }
}

void launch_quad_elem(Ctx* ctx, int kind, int prec, int op, bool nonlinear, const Task* tasks,
                      const int2* work, int n_work, int bn_max, const BaseArgs& ba) {
  if (n_work <= 0) return;
  if (kind == kKindQ4) launch_quad_nv<4>(ctx, prec, op, nonlinear, tasks, work, n_work, bn_max, ba);
  else launch_quad_nv<8>(ctx, prec, op, nonlinear, tasks, work, n_work, bn_max, ba);
}

template <int NV>
static void launch_quad_energy_nv(Ctx* ctx, int prec, bool diff, const Task* tasks,
                                  const int2* work, int n_work, const BaseArgs& ba) {
  dim3 grid(n_work), block(kThreads);
  hipStream_t s = ctx->stream;
  if (!diff) {
    if (prec == PFEM_FP32)
      hipLaunchKernelGGL((k_energy_quad<NV, float, float, false>), grid, block, 0, s, tasks, work, ba);
    else
      hipLaunchKernelGGL((k_energy_quad<NV, double, double, false>), grid, block, 0, s, tasks, work, ba);
  } else {
    // u is the float64 state, v the increment in the kernel precision
    if (prec == PFEM_FP32)
      hipLaunchKernelGGL((k_energy_quad<NV, double, float, true>), grid, block, 0, s, tasks, work, ba);
    else
      hipLaunchKernelGGL((k_energy_quad<NV, double, double, true>), grid, block, 0, s, tasks, work, ba);
  }
}

void launch_quad_energy(Ctx* ctx, int kind, int prec, bool diff, const Task* tasks,
                        const int2* work, int n_work, const BaseArgs& ba) {
  if (n_work <= 0) return;
  if (kind == kKindQ4) launch_quad_energy_nv<4>(ctx, prec, diff, tasks, work, n_work, ba);
  else launch_quad_energy_nv<8>(ctx, prec, diff, tasks, work, n_work, ba);
}

}  // namespace pfem
