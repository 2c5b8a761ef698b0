// Coarse space of the two-level preconditioner (host setup).
//
// M^-1 = D^-1 + P (P^T K P)^-1 P^T on the free DOFs, with P spanned on each
// aggregate of nodes by the rigid-body modes of linear elasticity (2D: two
// translations and a rotation; 3D: three and three), zero elsewhere and at
// prescribed DOFs.  The aggregates are groups of G consecutive owner
// blocks of the internal numbering (compact patches), G the smallest group
// that keeps the coarse dimension within kCoarseMax.  Per aggregate the raw
// modes (about its centroid) are orthonormalised over its free DOFs by an
// eigen-decomposition of their 6 x 6 (3 x 3) Gram matrix, dropping the
// directions it does not resolve; the coarse matrix P^T K P is summed
// element by element from float64 element stiffnesses of the linear
// moduli (the Neo-Hookean tangent at the undeformed state), Cholesky-
// factored and inverted, so that the device applies the coarse solve as
// one dense matrix-vector product.
#include <algorithm>
#include <cmath>
#include <functional>
#include <thread>

#include "coarse.h"

namespace pfem {

static void run_threads(int64_t n, const std::function<void(int, int64_t, int64_t)>& f,
                        int nt, int64_t min_n = 4096) {
  if (nt <= 1 || n < min_n) {
    f(0, 0, n);
    return;
  }
  const int64_t chunk = (n + nt - 1) / nt;
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) {
    const int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b < e) th.emplace_back(f, t, b, e);
  }
  for (auto& x : th) x.join();
}

static int host_threads() {
  return (int)std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
}

// Symmetric eigen-decomposition of a small matrix by cyclic Jacobi rotations:
// A (n x n, row-major) = V diag(w) V^T.
static void jacobi_eigen(int n, double* A, double* w, double* V) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double theta = 0.5 * (A[q * n + q] - A[p * n + p]) / apq;
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

// Raw rigid mode j at a point with coordinates y relative to the centroid:
// R[i][j] = component i (2D: translations, rotation (-y1, y0); 3D:
// translations, rotations about x, y, z: (0, -y2, y1), (y2, 0, -y0),
// (-y1, y0, 0)).
static void raw_modes(int D, const double* y, double (*R)[6]) {
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < 6; ++j) R[i][j] = 0.0;
  for (int i = 0; i < D; ++i) R[i][i] = 1.0;
  if (D == 2) {
    R[0][2] = -y[1];
    R[1][2] = y[0];
  } else {
    R[1][3] = -y[2];
    R[2][3] = y[1];
    R[0][4] = y[2];
    R[2][4] = -y[0];
    R[0][5] = -y[1];
    R[1][5] = y[0];
  }
}

int coarse_group(const pfem_mesh* m) {
  const int nrb = m->dim == 2 ? 3 : 6;
  const int64_t need = (int64_t)nrb * m->n_blocks;
  return (int)std::max<int64_t>(1, (need + kCoarseMax - 1) / kCoarseMax);
}

// In-place Cholesky (lower) of a dense SPD matrix, blocked, the panel and
// trailing updates spread over host threads; then A^-1 = L^-T L^-1.
static void spd_inverse(int n, std::vector<double>& A) {
  const int nt = host_threads();
  const int nb = 64;
  for (int k0 = 0; k0 < n; k0 += nb) {
    const int k1 = std::min(n, k0 + nb);
    for (int k = k0; k < k1; ++k) {   // diagonal block and the panel below it
      double d = A[(size_t)k * n + k];
      for (int j = k0; j < k; ++j) d -= A[(size_t)k * n + j] * A[(size_t)k * n + j];
      require(d > 0.0, PFEM_E_BREAKDOWN, "coarse matrix not positive definite");
      const double l = std::sqrt(d);
      A[(size_t)k * n + k] = l;
      run_threads(n - k - 1, [&](int, int64_t b, int64_t e) {
        for (int64_t ii = b; ii < e; ++ii) {
          const int i = k + 1 + (int)ii;
          double s = A[(size_t)i * n + k];
          for (int j = k0; j < k; ++j) s -= A[(size_t)i * n + j] * A[(size_t)k * n + j];
          A[(size_t)i * n + k] = s / l;
        }
      }, nt);
    }
    // trailing update of rows and columns >= k1 by the panel k0..k1
    run_threads(n - k1, [&](int, int64_t b, int64_t e) {
      for (int64_t ii = b; ii < e; ++ii) {
        const int i = k1 + (int)ii;
        for (int j = k1; j <= i; ++j) {
          double s = 0.0;
          for (int k = k0; k < k1; ++k) s += A[(size_t)i * n + k] * A[(size_t)j * n + k];
          A[(size_t)i * n + j] -= s;
        }
      }
    }, nt, 64);
  }
  // L^-1 column by column (independent forward substitutions)
  std::vector<double> Li((size_t)n * n, 0.0);
  run_threads(n, [&](int, int64_t b, int64_t e) {
    for (int64_t c = b; c < e; ++c) {
      for (int i = (int)c; i < n; ++i) {
        double s = i == c ? 1.0 : 0.0;
        for (int k = (int)c; k < i; ++k) s -= A[(size_t)i * n + k] * Li[(size_t)k * n + c];
        Li[(size_t)i * n + c] = s / A[(size_t)i * n + i];
      }
    }
  }, nt, 64);
  // A^-1 = L^-T L^-1: (i, j) = sum_{k >= max(i, j)} Li[k][i] Li[k][j]
  run_threads(n, [&](int, int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i)
      for (int j = 0; j <= i; ++j) {
        double s = 0.0;
        for (int k = (int)i; k < n; ++k) s += Li[(size_t)k * n + i] * Li[(size_t)k * n + j];
        A[(size_t)i * n + j] = s;
      }
  }, nt, 64);
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i];
}

void coarse_build(pfem_mesh* m) {
  std::lock_guard<std::mutex> lk(m->coarse_mu);
  if (m->coarse) return;
  require(m->finalized, PFEM_E_STATE, "mesh not finalized");
  const int D = m->dim, nv = D + 1;
  const int nrb = D == 2 ? 3 : 6;
  auto c = std::make_unique<CoarseHost>();
  c->n_rb = nrb;
  c->G = coarse_group(m);
  const int64_t N = m->n_nodes;
  const int bn = m->bn;
  c->n_agg = (m->n_blocks + c->G - 1) / c->G;
  c->n_c = c->n_agg * nrb;
  auto agg_of = [&](int64_t node) { return (int)((node / bn) / c->G); };
  // centroids (internal coordinates)
  c->cent.assign((size_t)c->n_agg * 3, 0.0);
  std::vector<int64_t> cnt(c->n_agg, 0);
  for (int64_t n = 0; n < N; ++n) {
    const int a = agg_of(n);
    for (int i = 0; i < D; ++i) c->cent[(size_t)a * 3 + i] += m->X_int[n * D + i];
    ++cnt[a];
  }
  for (int a = 0; a < c->n_agg; ++a)
    for (int i = 0; i < D; ++i) c->cent[(size_t)a * 3 + i] /= std::max<int64_t>(cnt[a], 1);
  // per-aggregate orthonormalisation over the free DOFs
  std::vector<double> gram((size_t)c->n_agg * 36, 0.0);
  for (int64_t n = 0; n < N; ++n) {
    const int a = agg_of(n);
    double y[3];
    for (int i = 0; i < D; ++i) y[i] = m->X_int[n * D + i] - c->cent[(size_t)a * 3 + i];
    double R[3][6];
    raw_modes(D, y, R);
    for (int i = 0; i < D; ++i) {
      if ((m->dmask[n] >> i) & 1) continue;
      for (int j = 0; j < nrb; ++j)
        for (int l = 0; l < nrb; ++l) gram[(size_t)a * 36 + j * nrb + l] += R[i][j] * R[i][l];
    }
  }
  c->T.assign((size_t)c->n_agg * nrb * nrb, 0.0);
  for (int a = 0; a < c->n_agg; ++a) {
    double A[36], w[6], V[36];
    std::copy(&gram[(size_t)a * 36], &gram[(size_t)a * 36] + nrb * nrb, A);
    jacobi_eigen(nrb, A, w, V);
    double wmax = 0.0;
    for (int k = 0; k < nrb; ++k) wmax = std::max(wmax, w[k]);
    for (int k = 0; k < nrb; ++k) {
      if (!(w[k] > 1e-12 * wmax) || wmax <= 0.0) continue;   // not resolved: dropped
      const double s = 1.0 / std::sqrt(w[k]);
      for (int j = 0; j < nrb; ++j) c->T[(size_t)a * nrb * nrb + j * nrb + k] = V[j * nrb + k] * s;
    }
  }
  // coarse matrix: sum over elements of (P_e)^T K_e P_e, per-thread copies
  const int nt = host_threads();
  const size_t nc2 = (size_t)c->n_c * c->n_c;
  std::vector<std::vector<double>> Ac(nt);
  run_threads(m->n_elems, [&](int t, int64_t b, int64_t e) {
    std::vector<double>& A = Ac[t];
    A.assign(nc2, 0.0);
    for (int64_t s = b; s < e; ++s) {
      const int32_t* nd = &m->conn_int[s * nv];
      // shape gradients of the P1 element: rows of J^-1, J = [X_a - X_0]
      double J[3][3], Ji[3][3];
      for (int a = 1; a <= D; ++a)
        for (int i = 0; i < D; ++i)
          J[i][a - 1] = m->X_int[(int64_t)nd[a] * D + i] - m->X_int[(int64_t)nd[0] * D + i];
      double det;
      if (D == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        Ji[0][0] = J[1][1] / det;
        Ji[0][1] = -J[0][1] / det;
        Ji[1][0] = -J[1][0] / det;
        Ji[1][1] = J[0][0] / det;
      } else {
        det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
              J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
              J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
      }
      const double vol = std::fabs(det) / (D == 2 ? 2.0 : 6.0);
      double Gr[4][3];
      for (int i = 0; i < D; ++i) Gr[0][i] = 0.0;
      for (int a = 1; a <= D; ++a)
        for (int i = 0; i < D; ++i) {
          Gr[a][i] = Ji[a - 1][i];
          Gr[0][i] -= Ji[a - 1][i];
        }
      const double mu = m->mu_int[s], lam = m->lam_int[s];
      // coarse columns touched: (aggregate, orthonormal mode k) per distinct aggregate
      int aggs[4], na = 0, slot[4];
      for (int a = 0; a < nv; ++a) {
        const int g = agg_of(nd[a]);
        int q = 0;
        while (q < na && aggs[q] != g) ++q;
        if (q == na) aggs[na++] = g;
        slot[a] = q;
      }
      const int ncol = na * nrb;
      // values of each column at the element's DOFs (a, i): column (q, k)
      double Pcol[24][12];
      for (int col = 0; col < ncol; ++col)
        for (int r = 0; r < nv * D; ++r) Pcol[col][r] = 0.0;
      for (int a = 0; a < nv; ++a) {
        const int g = aggs[slot[a]];
        double y[3];
        for (int i = 0; i < D; ++i) y[i] = m->X_int[(int64_t)nd[a] * D + i] - c->cent[(size_t)g * 3 + i];
        double R[3][6];
        raw_modes(D, y, R);
        const double* T = &c->T[(size_t)g * nrb * nrb];
        for (int i = 0; i < D; ++i) {
          if ((m->dmask[nd[a]] >> i) & 1) continue;
          for (int k = 0; k < nrb; ++k) {
            double v = 0.0;
            for (int j = 0; j < nrb; ++j) v += R[i][j] * T[j * nrb + k];
            Pcol[slot[a] * nrb + k][a * D + i] = v;
          }
        }
      }
      // K_e P for every column: (K_e v)_(a,i) = vol sum_b [lam G_a,i (G_b . v_b)
      //   + mu ((G_a . G_b) v_b,i + G_a . v_b G_b,i)]
      double KP[24][12];
      for (int col = 0; col < ncol; ++col) {
        double divv = 0.0;           // sum_b G_b . v_b  (trace of grad v)
        double Gv[3][3] = {};        // grad v: Gv[i][j] = sum_b v_b,i G_b,j
        for (int b2 = 0; b2 < nv; ++b2)
          for (int i = 0; i < D; ++i) {
            const double vb = Pcol[col][b2 * D + i];
            divv += vb * Gr[b2][i];
            for (int j = 0; j < D; ++j) Gv[i][j] += vb * Gr[b2][j];
          }
        // stress of the strain sym(grad v): sigma = lam tr I + mu (Gv + Gv^T)
        double S[3][3];
        for (int i = 0; i < D; ++i)
          for (int j = 0; j < D; ++j) S[i][j] = mu * (Gv[i][j] + Gv[j][i]) + (i == j ? lam * divv : 0.0);
        for (int a = 0; a < nv; ++a)
          for (int i = 0; i < D; ++i) {
            double v = 0.0;
            for (int j = 0; j < D; ++j) v += S[i][j] * Gr[a][j];
            KP[col][a * D + i] = vol * v;
          }
      }
      for (int c1 = 0; c1 < ncol; ++c1) {
        const int row = aggs[c1 / nrb] * nrb + c1 % nrb;
        for (int c2 = 0; c2 < ncol; ++c2) {
          const int colg = aggs[c2 / nrb] * nrb + c2 % nrb;
          double v = 0.0;
          for (int r = 0; r < nv * D; ++r) v += Pcol[c1][r] * KP[c2][r];
          A[(size_t)row * c->n_c + colg] += v;
        }
      }
    }
  }, nt);
  std::vector<double> A(nc2, 0.0);
  for (auto& At : Ac) {
    if (At.empty()) continue;
    for (size_t i = 0; i < nc2; ++i) A[i] += At[i];
    std::vector<double>().swap(At);
  }
  // dropped directions and aggregates without free DOFs: identity rows
  for (int i = 0; i < c->n_c; ++i)
    if (!(A[(size_t)i * c->n_c + i] > 0.0)) {
      for (int j = 0; j < c->n_c; ++j) A[(size_t)i * c->n_c + j] = A[(size_t)j * c->n_c + i] = 0.0;
      A[(size_t)i * c->n_c + i] = 1.0;
    }
  spd_inverse(c->n_c, A);
  // B = T A_c^-1 T^T (T block diagonal, one nrb x nrb block per aggregate):
  // the coarse correction in raw-mode coordinates, y = B (R^T r), so the
  // device needs neither T nor the orthonormal coordinates
  const int n = c->n_c;
  std::vector<double> C((size_t)n * n);
  run_threads(c->n_agg, [&](int, int64_t b, int64_t e) {
    for (int64_t a = b; a < e; ++a) {
      const double* Ta = &c->T[(size_t)a * nrb * nrb];
      for (int k = 0; k < nrb; ++k) {        // C = A_c^-1 T^T, rows of aggregate a
        const double* arow = &A[(size_t)(a * nrb + k) * n];
        double* crow = &C[(size_t)(a * nrb + k) * n];
        for (int g = 0; g < c->n_agg; ++g) {
          const double* Tg = &c->T[(size_t)g * nrb * nrb];
          for (int l = 0; l < nrb; ++l) {
            double v = 0.0;
            for (int q = 0; q < nrb; ++q) v += arow[g * nrb + q] * Tg[l * nrb + q];
            crow[g * nrb + l] = v;
          }
        }
      }
      for (int j = 0; j < nrb; ++j) {        // B = T C, rows of aggregate a
        double* brow = &A[(size_t)(a * nrb + j) * n];
        for (int col = 0; col < n; ++col) {
          double v = 0.0;
          for (int k = 0; k < nrb; ++k) v += Ta[j * nrb + k] * C[(size_t)(a * nrb + k) * n + col];
          brow[col] = v;
        }
      }
    }
  }, host_threads());
  c->B.swap(A);
  m->coarse = std::move(c);
}

void coarse_upload(pfem_mesh* m, Ctx* ctx) {
  coarse_build(m);
  std::lock_guard<std::mutex> lk(m->coarse_mu);
  if (m->dev.coarse_B64 != nullptr) return;
  const CoarseHost& c = *m->coarse;
  const int D = m->dim;
  std::vector<double> rel64(m->X_int.size());
  std::vector<float> rel32(m->X_int.size());
  for (int64_t n = 0; n < m->n_nodes; ++n) {
    const int a = (int)((n / m->bn) / c.G);
    for (int i = 0; i < D; ++i) {
      rel64[n * D + i] = m->X_int[n * D + i] - c.cent[(size_t)a * 3 + i];
      rel32[n * D + i] = (float)rel64[n * D + i];
    }
  }
  std::vector<float> b32(c.B.begin(), c.B.end());
  auto up = [&](void** p, const void* src, size_t bytes) {
    PFEM_HIP(hipMalloc(p, std::max<size_t>(bytes, 8)));
    PFEM_HIP(hipMemcpy(*p, src, bytes, hipMemcpyHostToDevice));
    m->dev.bytes += (int64_t)std::max<size_t>(bytes, 8);
  };
  (void)ctx;
  up((void**)&m->dev.coarse_rel64, rel64.data(), rel64.size() * 8);
  up((void**)&m->dev.coarse_rel32, rel32.data(), rel32.size() * 4);
  up((void**)&m->dev.coarse_B32, b32.data(), b32.size() * 4);
  up((void**)&m->dev.coarse_B64, c.B.data(), c.B.size() * 8);
}

int64_t coarse_device_bytes(const pfem_mesh* m) {
  const int nrb = m->dim == 2 ? 3 : 6;
  const int64_t G = coarse_group(m);
  const int64_t n_agg = (m->n_blocks + G - 1) / G;
  const int64_t nc = n_agg * nrb;
  return m->n_dof() * 12 + nc * nc * 12 + 4 * 8;
}

}  // namespace pfem
