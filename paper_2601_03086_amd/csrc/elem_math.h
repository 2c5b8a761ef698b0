// Per-element P1 physics shared by every element kernel (device code).
//
// Geometry (App. B, P1 total-Lagrangian discretisation): with edge vectors
// e_a = X_a - X_0 (a = 1..D) the rows of J^{-1} (J = [e_1 .. e_D]) are the
// shape-function gradients grad N_a = c_a / det J, where c_a are the
// cofactor rows (2D: c_1 = (e2y, -e2x), c_2 = (-e1y, e1x); 3D:
// c_1 = e2 x e3, c_2 = e3 x e1, c_3 = e1 x e2) and grad N_0 = -sum_a grad N_a.
// The element measure is |det J| / D!.  float64 kernels read float64
// coordinates and difference them in float64.  float32 kernels read 32-bit
// fixed-point coordinates (X = lo + q * step over the mesh's bounding box,
// step = extent / (2^32 - 1)): the edge q_a - q_0 is an exact integer, so
// the geometry keeps the relative accuracy of float32 on small elements
// far from the origin, at half the bytes of float64 coordinates.
//
// Every nodal output y_a is formed from the unnormalised c_a; vol/det^2 =
// 1/(D! |det|) and vol/det = sign(det)/D! carry the normalisation, so each
// element needs a single division.
#pragma once

#include <hip/hip_runtime.h>

#include "pfem_internal.h"

namespace pfem {

template <int D>
struct Fact;
template <>
struct Fact<2> { static constexpr double v = 2.0; };
template <>
struct Fact<3> { static constexpr double v = 6.0; };

template <int D, typename T>
struct Geo {
  T c[D][D];   // c[a-1][j]: unnormalised gradient of node a (a = 1..D)
  T det;       // signed det J
};

template <int D>
__device__ __forceinline__ void load_coords(const double* __restrict__ X,
                                            const int (&nd)[D + 1], double (&x)[D + 1][D]) {
  if constexpr (D == 2) {
#pragma unroll
    for (int a = 0; a <= D; ++a) {
      const pd2 q = ldx(reinterpret_cast<const pd2*>(X), (uint32_t)nd[a]);
      x[a][0] = q.x;
      x[a][1] = q.y;
    }
  } else {
#pragma unroll
    for (int a = 0; a <= D; ++a) {
      const Trip<double> q = ldx(reinterpret_cast<const Trip<double>*>(X), (uint32_t)nd[a]);
      x[a][0] = q.x;
      x[a][1] = q.y;
      x[a][2] = q.z;
    }
  }
}

template <int D>
__device__ __forceinline__ void load_coords_q(const uint32_t* __restrict__ Xq,
                                              const int (&nd)[D + 1], uint32_t (&x)[D + 1][D]) {
#pragma unroll
  for (int a = 0; a <= D; ++a) {
    if constexpr (D == 2) {
      typedef unsigned int pu2 __attribute__((ext_vector_type(2)));
      const pu2 q = ldx(reinterpret_cast<const pu2*>(Xq), (uint32_t)nd[a]);
      x[a][0] = q.x;
      x[a][1] = q.y;
    } else {
      const Trip<uint32_t> q = ldx(reinterpret_cast<const Trip<uint32_t>*>(Xq), (uint32_t)nd[a]);
      x[a][0] = q.x;
      x[a][1] = q.y;
      x[a][2] = q.z;
    }
  }
}

template <int D, typename T>
__device__ __forceinline__ void geometry_from_edges(const T (&e)[D][D], Geo<D, T>& g);

// Coordinates of an element as the kernel type reads them.
template <int D, typename T>
struct ElemX {
  double x[D + 1][D];
};
template <int D>
struct ElemX<D, float> {
  uint32_t q[D + 1][D];
};

template <int D, typename T>
__device__ __forceinline__ void load_elem_x(const MeshDev& m, const int (&nd)[D + 1],
                                            ElemX<D, T>& x) {
  if constexpr (sizeof(T) == 4) load_coords_q<D>(m.Xq, nd, x.q);
  else load_coords<D>(m.X, nd, x.x);
}

template <int D, typename T>
__device__ __forceinline__ void geometry_x(const MeshDev& m, const ElemX<D, T>& x,
                                           Geo<D, T>& g) {
  T e[D][D];
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int i = 0; i < D; ++i)
        e[a][i] = (float)((int)x.q[a + 1][i] - (int)x.q[0][i]) * m.qscale[i];   // q < 2^31
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int i = 0; i < D; ++i) e[a][i] = (T)(x.x[a + 1][i] - x.x[0][i]);
  }
  geometry_from_edges<D, T>(e, g);
}

template <int D, typename T>
__device__ __forceinline__ void geometry(const double (&x)[D + 1][D], Geo<D, T>& g) {
  T e[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int i = 0; i < D; ++i)
      e[a][i] = (T)(x[a + 1][i] - x[0][i]);
  geometry_from_edges<D, T>(e, g);
}

template <int D, typename T>
__device__ __forceinline__ void geometry_from_edges(const T (&e)[D][D], Geo<D, T>& g) {
  if constexpr (D == 2) {
    g.c[0][0] = e[1][1];
    g.c[0][1] = -e[1][0];
    g.c[1][0] = -e[0][1];
    g.c[1][1] = e[0][0];
    g.det = e[0][0] * e[1][1] - e[0][1] * e[1][0];
  } else {
    // c_1 = e2 x e3, c_2 = e3 x e1, c_3 = e1 x e2
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T* p = e[(a + 1) % 3];
      const T* q = e[(a + 2) % 3];
      g.c[a][0] = p[1] * q[2] - p[2] * q[1];
      g.c[a][1] = p[2] * q[0] - p[0] * q[2];
      g.c[a][2] = p[0] * q[1] - p[1] * q[0];
    }
    g.det = e[0][0] * g.c[0][0] + e[0][1] * g.c[0][1] + e[0][2] * g.c[0][2];
  }
}

template <int D, typename T>
__device__ __forceinline__ void load_geometry(const MeshDev& m, const int (&nd)[D + 1],
                                              Geo<D, T>& g) {
  ElemX<D, T> x;
  load_elem_x<D, T>(m, nd, x);
  geometry_x<D, T>(m, x, g);
}

// Gradient-like tensor M_ij = sum_{a>=1} (v_a - v_0)_i c_a,j.
template <int D, typename T>
__device__ __forceinline__ void grad_tilde(const T (&v)[D + 1][D],
                                           const Geo<D, T>& g, T (&M)[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) M[i][j] = T(0);
#pragma unroll
  for (int a = 1; a <= D; ++a) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const T dv = v[a][i] - v[0][i];
#pragma unroll
      for (int j = 0; j < D; ++j) M[i][j] += dv * g.c[a - 1][j];
    }
  }
}

// y_a = s * S c_a (a >= 1), y_0 = -sum_a y_a.
template <int D, typename T>
__device__ __forceinline__ void scatter_rows(const T (&S)[D][D], const Geo<D, T>& g,
                                             T s, T (&y)[D + 1][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i) y[0][i] = T(0);
#pragma unroll
  for (int a = 1; a <= D; ++a) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < D; ++j) acc += S[i][j] * g.c[a - 1][j];
      y[a][i] = s * acc;
      y[0][i] -= y[a][i];
    }
  }
}

// ---------------------------------------------------------------- linear
// sigma = mu (M + M^T) + lambda tr(M) I applied to M = sum dv (x) c
// (Sec. 'Linear elastic plate...': sigma = 2 mu eps + lambda tr eps I).
template <int D, typename T>
__device__ __forceinline__ void linear_stress_tilde(const T (&M)[D][D], T mu, T lam,
                                                    T (&S)[D][D]) {
  T tr = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) tr += M[i][i];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j)
      S[i][j] = mu * (M[i][j] + M[j][i]) + (i == j ? lam * tr : T(0));
}

// ------------------------------------------------------------ Neo-Hookean
// Kinematic state of one element: H = grad u, F^{-T}, J - 1 and ln J.
// J - 1 from the invariants of H keeps its relative accuracy at small strain
// in either precision.  Near compression (J < 0.7) ln J and 1/J amplify the
// rounding of J - 1 by 1/J: float32 kernels evaluate J - 1, ln J and 1/J in
// float64 there (the float64 det F / log J rule of the mixed-precision path),
// and in float32 elsewhere, where float32 keeps them to a few ulps.
template <int D, typename T>
struct NHState {
  T H[D][D];
  T FinvT[D][D];
  T j;      // J - 1
  T lnJ;
  bool ok;  // J > 0
};

// J - 1 from the invariants of H (exact identities):
//   2D: tr H + det H;  3D: tr H + ((tr H)^2 - tr H^2)/2 + det H.
template <int D, typename T>
__device__ __forceinline__ T jm1(const T (&h)[D][D]) {
  if constexpr (D == 2) {
    return (h[0][0] + h[1][1]) + (h[0][0] * h[1][1] - h[0][1] * h[1][0]);
  } else {
    const T tr = h[0][0] + h[1][1] + h[2][2];
    T trH2 = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) trH2 += h[i][k] * h[k][i];
    const T det = h[0][0] * (h[1][1] * h[2][2] - h[1][2] * h[2][1]) -
                  h[0][1] * (h[1][0] * h[2][2] - h[1][2] * h[2][0]) +
                  h[0][2] * (h[1][0] * h[2][1] - h[1][1] * h[2][0]);
    return tr + T(0.5) * (tr * tr - trH2) + det;
  }
}

// J - 1, ln J and 1/J of the element (0 and ok = false when J <= 0).
template <int D, typename T>
__device__ __forceinline__ void nh_volumetric(const T (&H)[D][D], T& j, T& lnJ, T& invJ,
                                              bool& ok) {
  j = jm1<D, T>(H);
  if constexpr (sizeof(T) == 4) {
    if (j < -0.3f) {
      // products of two float32 values are exact in float64
      double jd;
      if constexpr (D == 2) {
        jd = ((double)H[0][0] + (double)H[1][1]) +
             ((double)H[0][0] * H[1][1] - (double)H[0][1] * H[1][0]);
      } else {
        const double tr = (double)H[0][0] + (double)H[1][1] + (double)H[2][2];
        // (tr^2 - tr H^2)/2 = sum of the principal 2x2 minors of H
        const double m2 = ((double)H[0][0] * H[1][1] - (double)H[0][1] * H[1][0]) +
                          ((double)H[0][0] * H[2][2] - (double)H[0][2] * H[2][0]) +
                          ((double)H[1][1] * H[2][2] - (double)H[1][2] * H[2][1]);
        const double det =
            (double)H[0][0] * ((double)H[1][1] * H[2][2] - (double)H[1][2] * H[2][1]) -
            (double)H[0][1] * ((double)H[1][0] * H[2][2] - (double)H[1][2] * H[2][0]) +
            (double)H[0][2] * ((double)H[1][0] * H[2][1] - (double)H[1][1] * H[2][0]);
        jd = tr + m2 + det;
      }
      ok = jd > -1.0;
      j = (float)jd;
      // J rounded once from its float64 value: away from J = 1 the float32
      // logarithm and reciprocal of it are accurate to a few ulps
      const float Jf = (float)(1.0 + jd);
      lnJ = ok ? logf(Jf) : 0.0f;
      invJ = ok ? 1.0f / Jf : 0.0f;
      return;
    }
  }
  ok = j > T(-1);
  lnJ = ok ? log1p(j) : T(0);
  invJ = ok ? T(1) / (T(1) + j) : T(0);
}

template <int D, typename T>
__device__ __forceinline__ void nh_state(const T (&Ht)[D][D], T inv_det,
                                         NHState<D, T>& st) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) st.H[i][k] = Ht[i][k] * inv_det;
  T invJ;
  nh_volumetric<D, T>(st.H, st.j, st.lnJ, invJ, st.ok);
  T F[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) F[i][k] = st.H[i][k] + (i == k ? T(1) : T(0));
  // F^{-T} = cof(F) / J
  if constexpr (D == 2) {
    st.FinvT[0][0] = F[1][1] * invJ;
    st.FinvT[0][1] = -F[1][0] * invJ;
    st.FinvT[1][0] = -F[0][1] * invJ;
    st.FinvT[1][1] = F[0][0] * invJ;
  } else {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const T* p = F[(r + 1) % 3];
      const T* q = F[(r + 2) % 3];
      st.FinvT[r][0] = (p[1] * q[2] - p[2] * q[1]) * invJ;
      st.FinvT[r][1] = (p[2] * q[0] - p[0] * q[2]) * invJ;
      st.FinvT[r][2] = (p[0] * q[1] - p[1] * q[0]) * invJ;
    }
  }
}

// First Piola stress P = mu (H + F^{-T} H^T) + lambda ln J F^{-T}
// (= mu (F - F^{-T}) + lambda ln J F^{-T}; App. B internal force).
template <int D, typename T>
__device__ __forceinline__ void nh_piola(const NHState<D, T>& st, T mu, T lam,
                                         T (&P)[D][D]) {
  const T ll = lam * st.lnJ;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T a = T(0);
#pragma unroll
      for (int l = 0; l < D; ++l) a += st.FinvT[i][l] * st.H[k][l];
      P[i][k] = mu * (st.H[i][k] + a) + ll * st.FinvT[i][k];
    }
}

// dP = mu dF + lambda (F^{-T}:dF) F^{-T} + (mu - lambda ln J) F^{-T} dF^T F^{-T}
// (App. B tangent K_mat + K_geo in first-Piola form), dF given unnormalised.
template <int D, typename T>
__device__ __forceinline__ void nh_dpiola(const NHState<D, T>& st, T mu, T lam,
                                          const T (&dF)[D][D], T (&dP)[D][D]) {
  T tr = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) tr += st.FinvT[i][k] * dF[i][k];
  const T c2 = mu - lam * st.lnJ;
  T A[D][D];  // A = dF^T F^{-T}
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T a = T(0);
#pragma unroll
      for (int l = 0; l < D; ++l) a += dF[l][i] * st.FinvT[l][k];
      A[i][k] = a;
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T b = T(0);
#pragma unroll
      for (int l = 0; l < D; ++l) b += st.FinvT[i][l] * A[l][k];
      dP[i][k] = mu * dF[i][k] + lam * tr * st.FinvT[i][k] + c2 * b;
    }
}

// Psi(H) in float64 from the kernel-type H:
//   mu[(tr H - j) + |H|^2/2 + (j - log1p j)] + lambda (log1p j)^2 / 2
// (Sec. 'Nonlinear hyperelasticity' density with I1 - D = 2 tr H + |H|^2,
// ln J = log1p j; tr H - j = -det H in 2D, -(((tr H)^2 - tr H^2)/2 + det H)
// in 3D).  Returns +inf when J <= 0.
template <int D, typename T>
__device__ __forceinline__ double nh_energy_density(const T (&Hk)[D][D], double mu,
                                                    double lam) {
  double H[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) H[i][k] = Hk[i][k];
  double tr = 0.0, h2 = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) tr += H[i][i];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) h2 += H[i][k] * H[i][k];
  double second;  // j - tr H
  if constexpr (D == 2) {
    second = H[0][0] * H[1][1] - H[0][1] * H[1][0];
  } else {
    double trH2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) trH2 += H[i][k] * H[k][i];
    const double det = H[0][0] * (H[1][1] * H[2][2] - H[1][2] * H[2][1]) -
                       H[0][1] * (H[1][0] * H[2][2] - H[1][2] * H[2][0]) +
                       H[0][2] * (H[1][0] * H[2][1] - H[1][1] * H[2][0]);
    second = 0.5 * (tr * tr - trH2) + det;
  }
  const double j = tr + second;
  if (!(j > -1.0)) return __builtin_inf();
  const double l = log1p(j);
  return mu * (-second + 0.5 * h2 + (j - l)) + 0.5 * lam * l * l;
}

}  // namespace pfem
