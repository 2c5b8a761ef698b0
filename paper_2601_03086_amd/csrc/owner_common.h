// Epilogues shared by the owner-computes element kernels of every element
// family (P1 in elem_kernels.hip, quadrilaterals in quad_kernels.hip): the
// owned-DOF write of K.v / force / diagonal and the owned-DOF terms of the
// energy.
#pragma once

#include "pfem_internal.h"
#include "reduce.h"

namespace pfem {

// Periodic springs at component c of owned node n: the virtual elements of a
// periodic cell, each a spring of stiffness k to a partner node.  Their
// energy 1/2 k |x_n - x_b|^2 adds k sum_b (x_n - x_b) to the apply (input
// X = v) and to the internal force (X = u), and k per partner to the
// diagonal.  With PFEM_MASK_IN an apply reads zero at Dirichlet DOFs.
template <int D, typename T, int OP>
__device__ __forceinline__ T periodic_springs(const MeshDev& m, const T* __restrict__ X, int mask,
                                              int n, int c, bool con) {
  const int q0 = ldg(m.pair_ptr + n), q1 = ldg(m.pair_ptr + n + 1);
  if (OP == OP_DIAG) return (T)(m.pair_k * (double)(q1 - q0));
  const bool mask_in = is_apply_op(OP) && (mask & PFEM_MASK_IN);
  const T xn = (mask_in && con) ? T(0) : ldg(X + (size_t)n * D + c);
  T s = T(0);
  for (int q = q0; q < q1; ++q) {
    const int b = ldg(m.pair_nbr + q);
    const bool cb = mask_in && ((ldg(m.dmask + b) >> c) & 1);
    s += xn - (cb ? T(0) : ldg(X + (size_t)b * D + c));
  }
  return (T)m.pair_k * s;
}

// The block's owned DOFs: acc[] holds the element sums (all threads
// synchronised).  Adds the periodic springs, subtracts the scaled external
// force (OP_FORCE), applies the Dirichlet mask or writes the (inverse)
// diagonal, stores every owned DOF once and writes the block's partials
// (y.w in slot 0, |y|^2 in slot 1; an apply reports slot 0 only: PCG init
// kernels own slots 1 and 2).
template <int D, typename T, int OP, typename A>
__device__ __forceinline__ void owner_epilogue(const Task* __restrict__ tp, const MeshDev& m,
                                               const A* acc, const T* __restrict__ U,
                                               const T* __restrict__ V, int mask,
                                               const BaseArgs& ba, int blk, int n0, int nloc) {
  T* Y = operand<T>(tp->y, ba.y, ba.rel);
  const T* W = static_cast<const T*>(tp->w);
  const double* FE = tp->fext != nullptr ? tp->fext : m.fext;
  const bool springs = m.pair_ptr != nullptr && !tp->no_pairs;
  double part[kRedSlots] = {0.0, 0.0, 0.0, 0.0};
  const size_t g0 = (size_t)n0 * D;
  const int nown = nloc * D;
  for (int i = threadIdx.x; i < nown; i += kThreads) {
    const size_t gi = g0 + i;
    T val = (T)acc[i];
    const bool con = (ldg(m.dmask + n0 + i / D) >> (i % D)) & 1;
    if (OP == OP_FORCE) val -= (T)(tp->fscale * ldg(FE + gi));
    if (springs) val += periodic_springs<D, T, OP>(m, is_apply_op(OP) ? V : U, mask, n0 + i / D,
                                                   i % D, con);
    if (OP == OP_DIAG) {
      if (con) val = T(1);
      else if (tp->s != 0.0) val = T(1) / val;   // inverse diagonal for PCG
    } else if ((mask & PFEM_MASK_OUT) && con) {
      val = T(0);
    }
    stg(Y + gi, val);
    if (W != nullptr) part[0] += (double)val * (double)ldg(W + gi);
    part[1] += (double)val * (double)val;
  }
  write_partials(tp->red, m.n_blocks, blk, part, 0, is_apply_op(OP) ? 1 : 2);
}

// The owned-DOF terms of the energy kernels, then the block's partials
// (energy or difference, #inverted, sum of |terms|): part[] arrives with the
// element sums of the block's own elements.
template <int D, typename TU, typename TV, bool DIFF>
__device__ __forceinline__ void energy_epilogue(const Task* __restrict__ tp, const MeshDev& m,
                                                const TU* __restrict__ U,
                                                const TV* __restrict__ V, double s, int blk,
                                                int n0, int nloc, double (&part)[kRedSlots]) {
  // - f_ext . u   (or - s f_ext . v for the difference), and the energy of
  // the periodic springs, 1/2 k |u_n - u_b|^2 per pair: a quarter from each
  // end's owner
  const size_t g0 = (size_t)n0 * D;
  const double* FE = tp->fext != nullptr ? tp->fext : m.fext;
  const bool springs = m.pair_ptr != nullptr && !tp->no_pairs;
  for (int i = threadIdx.x; i < nloc * D; i += kThreads) {
    const double f = tp->fscale * ldg(FE + g0 + i);
    if (DIFF) {
      const double w = s * f * (double)ldg(V + g0 + i);
      part[0] -= w;
      part[2] += fabs(w);
    } else {
      part[0] -= f * (double)ldg(U + g0 + i);
    }
    if (springs) {
      const int n = n0 + i / D, c = i % D;
      const int q0 = ldg(m.pair_ptr + n), q1 = ldg(m.pair_ptr + n + 1);
      const double un = (double)ldg(U + g0 + i);
      for (int q = q0; q < q1; ++q) {
        const size_t gb = (size_t)ldg(m.pair_nbr + q) * D + c;
        const double du = un - (double)ldg(U + gb);
        const double e0 = 0.25 * m.pair_k * du * du;
        if (DIFF) {
          const double dw = du + s * ((double)ldg(V + g0 + i) - (double)ldg(V + gb));
          const double e1 = 0.25 * m.pair_k * dw * dw;
          part[0] += e1 - e0;
          part[2] += e0 + e1;
        } else {
          part[0] += e0;
        }
      }
    }
  }
  write_partials(tp->red, m.n_blocks, blk, part, 0, DIFF ? 3 : 2);
}

}  // namespace pfem
