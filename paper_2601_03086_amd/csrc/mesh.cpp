// Mesh validation, bit-exact preprocessing and device upload.
//
// Preprocessing rules (the paper fixes no ordering; these tie-broken rules
// make every preprocessing result reproducible bit for bit):
//  * reverse Cuthill-McKee on the node graph (nodes adjacent when they share
//    an element): each connected component starts at the unvisited node of
//    smallest degree (ties: smallest caller id); a dequeued node appends its
//    unvisited neighbours ordered by (degree, caller id); the visiting order
//    is reversed at the end;
//  * node blocks (default numbering): the RCM order is cut into bands of
//    k * bn consecutive positions, k = max(1, min(round(w N / (L bn)),
//    floor(32768 / bn))) with L the number of breadth-first levels of the
//    search (summed over components) and w the largest integer with
//    w^d <= bn, halves rounded up (a band stays within 32768 positions, so
//    element node offsets fit 16 bits on ordinary meshes); each band
//    is cut into blocks of bn nodes by recursive coordinate bisection: a set
//    of more than bn nodes is ordered along its axis of largest extent
//    (smallest axis on ties) by (coordinate, RCM position) and split after
//    bn * floor(ceil(n / bn) / 2) nodes; a set of at most bn nodes is a
//    block, kept in RCM order.  Blocks become compact patches instead of
//    slivers of one RCM level, so far fewer elements straddle two blocks;
//  * elements sorted by the ascending tuple of their new node ids, ties by
//    caller element index (so the smallest node id is non-decreasing);
//  * colours by first fit in decreasing priority (fmix32(k ^ 0x9E3779B9), k)
//    with k the sorted position and fmix32 the MurmurHash3 finaliser;
//  * free DOFs ranked by increasing caller DOF index.
#include "mesh.h"
#include "coarse.h"

#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>
#include <thread>

namespace pfem {

uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Lame parameters (Sec. 'Nonlinear hyperelasticity': lambda = nu E /
// ((1+nu)(1-2nu)), mu = E / (2(1+nu))); plane stress uses the textbook
// lambda* = E nu / (1 - nu^2) = 2 mu lambda / (lambda + 2 mu).
void lame_from_params(int model, int param_kind, double p0, double p1, double* mu,
                      double* lam) {
  if (param_kind == PFEM_PARAM_E_NU) {
    const double E = p0, nu = p1;
    *mu = E / (2.0 * (1.0 + nu));
    if (model == PFEM_LIN_PLANE_STRESS)
      *lam = E * nu / (1.0 - nu * nu);
    else
      *lam = nu * E / ((1.0 + nu) * (1.0 - 2.0 * nu));
  } else {
    *mu = p0;
    *lam = p1;
    if (model == PFEM_LIN_PLANE_STRESS) *lam = 2.0 * p0 * p1 / (p1 + 2.0 * p0);
  }
}

static void prepare_device_images(pfem_mesh* m);

// Reference-coordinate derivatives dN_a/dxi, dN_a/deta of the Q4 (nv = 4)
// or Q8 serendipity (nv = 8) shape functions: corners (-1,-1), (1,-1),
// (1,1), (-1,1), then the midsides of edges (0,1), (1,2), (2,3), (3,0).
static void quad_shape_derivs(int nv, double xi, double eta, double (&dN)[8][2]) {
  static const double cx[4] = {-1, 1, 1, -1}, cy[4] = {-1, -1, 1, 1};
  for (int a = 0; a < 4; ++a) {
    const double p = 1 + xi * cx[a], q = 1 + eta * cy[a];
    if (nv == 4) {
      dN[a][0] = 0.25 * cx[a] * q;
      dN[a][1] = 0.25 * cy[a] * p;
    } else {   // N = p q (xi cx + eta cy - 1) / 4
      const double r = xi * cx[a] + eta * cy[a] - 1;
      dN[a][0] = 0.25 * cx[a] * q * (r + p);
      dN[a][1] = 0.25 * cy[a] * p * (r + q);
    }
  }
  if (nv == 8) {
    dN[4][0] = -xi * (1 - eta);            dN[4][1] = -0.5 * (1 - xi * xi);
    dN[5][0] = 0.5 * (1 - eta * eta);      dN[5][1] = -(1 + xi) * eta;
    dN[6][0] = -xi * (1 + eta);            dN[6][1] = 0.5 * (1 - xi * xi);
    dN[7][0] = -0.5 * (1 - eta * eta);     dN[7][1] = -(1 - xi) * eta;
  }
}

// Jacobian determinants of a quadrilateral at its corners and 3 x 3 Gauss
// points; false if they are not all of one sign, or one is tiny against the
// longest corner distance squared (a degenerate or folded element).
static bool quad_ok(const pfem_mesh* m, const int32_t* c) {
  static const double cxi[4] = {-1, 1, 1, -1}, ceta[4] = {-1, -1, 1, 1};
  const double g = std::sqrt(0.6);
  double pts[13][2];
  int np = 0;
  for (int a = 0; a < 4; ++a) {
    pts[np][0] = cxi[a];
    pts[np++][1] = ceta[a];
  }
  for (int i = -1; i <= 1; ++i)
    for (int j = -1; j <= 1; ++j) {
      pts[np][0] = i * g;
      pts[np++][1] = j * g;
    }
  double lmax = 0.0;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < a; ++b) {
      const double dx = m->coords[c[a] * 2] - m->coords[c[b] * 2];
      const double dy = m->coords[c[a] * 2 + 1] - m->coords[c[b] * 2 + 1];
      lmax = std::max(lmax, std::sqrt(dx * dx + dy * dy));
    }
  int sign = 0;
  for (int p = 0; p < np; ++p) {
    double dN[8][2];
    quad_shape_derivs(m->nv, pts[p][0], pts[p][1], dN);
    double J[2][2] = {{0, 0}, {0, 0}};
    for (int a = 0; a < m->nv; ++a)
      for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 2; ++k) J[i][k] += m->coords[(size_t)c[a] * 2 + i] * dN[a][k];
    const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    if (!(std::isfinite(det) && std::fabs(det) > 1e-12 * lmax * lmax)) return false;
    const int s = det > 0 ? 1 : -1;
    if (sign != 0 && s != sign) return false;
    sign = s;
  }
  return true;
}

// Block count above which the automatic block size grows (see finalize).
constexpr int64_t kBlocksSoftMax = 512;

static void validate(const pfem_mesh* m) {
  const int D = m->dim;
  const int nv = m->nv;
  require(m->model >= 0, PFEM_E_STATE, "material not set");
  std::vector<char> used(m->n_nodes, 0);
  for (int64_t e = 0; e < m->n_elems; ++e) {
    const int32_t* c = &m->conn[e * nv];
    // (messages are built only when a check fails: this loop runs per element)
    for (int a = 0; a < nv; ++a) {
      if (!(c[a] >= 0 && c[a] < m->n_nodes))
        throw Error{PFEM_E_INVALID_MESH,
                    "element " + std::to_string(e) + " references node out of range"};
      used[c[a]] = 1;
      for (int b = 0; b < a; ++b)
        if (c[a] == c[b])
          throw Error{PFEM_E_INVALID_MESH, "element " + std::to_string(e) + " repeats a node"};
    }
    if (m->elem != PFEM_ELEM_P1) {
      if (!quad_ok(m, c))
        throw Error{PFEM_E_INVALID_MESH,
                    "element " + std::to_string(e) + " is degenerate or folded"};
      continue;
    }
    // degeneracy: |det J| against the longest edge^D
    double ev[3][3] = {};
    double lmax = 0.0;
    for (int a = 0; a < D; ++a) {
      double l2 = 0.0;
      for (int i = 0; i < D; ++i) {
        ev[a][i] = m->coords[(size_t)c[a + 1] * D + i] - m->coords[(size_t)c[0] * D + i];
        l2 += ev[a][i] * ev[a][i];
      }
      lmax = std::max(lmax, std::sqrt(l2));
    }
    double det;
    if (D == 2)
      det = ev[0][0] * ev[1][1] - ev[0][1] * ev[1][0];
    else
      det = ev[0][0] * (ev[1][1] * ev[2][2] - ev[1][2] * ev[2][1]) -
            ev[0][1] * (ev[1][0] * ev[2][2] - ev[1][2] * ev[2][0]) +
            ev[0][2] * (ev[1][0] * ev[2][1] - ev[1][1] * ev[2][0]);
    if (!(std::isfinite(det) && std::fabs(det) > 1e-12 * std::pow(lmax, D)))
      throw Error{PFEM_E_INVALID_MESH, "element " + std::to_string(e) + " is degenerate"};
  }
  for (int64_t n = 0; n < m->n_nodes; ++n)
    if (!used[n])
      throw Error{PFEM_E_INVALID_MESH, "node " + std::to_string(n) + " belongs to no element"};
  for (double v : m->coords)
    require(std::isfinite(v), PFEM_E_INVALID_MESH, "non-finite coordinate");
  for (size_t i = 0; i < m->mu.size(); ++i)
    require(std::isfinite(m->mu[i]) && std::isfinite(m->lam[i]), PFEM_E_INVALID_ARG,
            "non-finite material parameter");
}

// f(begin, end) over [0, n) in contiguous chunks on up to 16 host threads
// (serially below 65536 items); f must only write its own items.
static void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& f) {
  const int64_t nt = std::min<int64_t>(16, std::max(1u, std::thread::hardware_concurrency()));
  if (n < 65536 || nt == 1) {
    f(0, n);
    return;
  }
  const int64_t chunk = (n + nt - 1) / nt;
  std::vector<std::thread> th;
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b < e) th.emplace_back(f, b, e);
  }
  for (auto& x : th) x.join();
}

// ----------------------------------------------------------------- RCM
static void node_graph(const pfem_mesh* m, std::vector<int64_t>& ptr,
                       std::vector<int32_t>& nbr) {
  const int nv = m->nv;
  const int64_t N = m->n_nodes;
  std::vector<int64_t> cnt(N + 1, 0);
  for (int64_t e = 0; e < m->n_elems; ++e)
    for (int a = 0; a < nv; ++a) cnt[m->conn[e * nv + a] + 1] += nv - 1;
  for (int64_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
  std::vector<int32_t> raw(cnt[N]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t e = 0; e < m->n_elems; ++e)
    for (int a = 0; a < nv; ++a)
      for (int b = 0; b < nv; ++b)
        if (a != b) raw[fill[m->conn[e * nv + a]]++] = m->conn[e * nv + b];
  ptr.assign(N + 1, 0);
  nbr.clear();
  nbr.reserve(raw.size() / 2);
  for (int64_t i = 0; i < N; ++i) {
    auto b = raw.begin() + cnt[i], en = raw.begin() + cnt[i + 1];
    std::sort(b, en);
    auto last = std::unique(b, en);
    nbr.insert(nbr.end(), b, last);
    ptr[i + 1] = (int64_t)nbr.size();
  }
}

// Cuthill-McKee visiting order; returns the number of breadth-first levels
// summed over the components.
static int64_t cuthill_mckee(const pfem_mesh* m, std::vector<int32_t>& q) {
  std::vector<int64_t> ptr;
  std::vector<int32_t> nbr;
  node_graph(m, ptr, nbr);
  const int64_t N = m->n_nodes;
  std::vector<int32_t> deg(N);
  for (int64_t i = 0; i < N; ++i) deg[i] = (int32_t)(ptr[i + 1] - ptr[i]);
  std::vector<int32_t> starts(N);
  std::iota(starts.begin(), starts.end(), 0);
  std::stable_sort(starts.begin(), starts.end(),
                   [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
  std::vector<char> vis(N, 0);
  std::vector<int32_t> level(N, 0);
  q.clear();
  q.reserve(N);
  std::vector<int32_t> tmp;
  int64_t si = 0, n_levels = 0;
  size_t head = 0;
  while ((int64_t)q.size() < N) {
    while (vis[starts[si]]) ++si;
    const int32_t s = starts[si];
    vis[s] = 1;
    q.push_back(s);
    int32_t depth = 0;
    while (head < q.size()) {
      const int32_t v = q[head++];
      depth = std::max(depth, level[v]);
      tmp.clear();
      for (int64_t k = ptr[v]; k < ptr[v + 1]; ++k)
        if (!vis[nbr[k]]) tmp.push_back(nbr[k]);
      std::sort(tmp.begin(), tmp.end(), [&](int32_t a, int32_t b) {
        return deg[a] != deg[b] ? deg[a] < deg[b] : a < b;
      });
      for (int32_t w : tmp) {
        vis[w] = 1;
        level[w] = level[v] + 1;
        q.push_back(w);
      }
    }
    n_levels += depth + 1;
  }
  return n_levels;
}

// Recursive coordinate bisection of nodes[b, e) into blocks of bn nodes, in
// place (rules in the header comment).  pos: RCM position of each node.
static void bisect_blocks(int32_t* b, int32_t* e, const double* X, int D,
                          const std::vector<int32_t>& pos, int bn) {
  const int64_t n = e - b;
  if (n <= bn) {
    std::sort(b, e, [&](int32_t x, int32_t y) { return pos[x] < pos[y]; });
    return;
  }
  double lo[3], hi[3];
  for (int i = 0; i < D; ++i) lo[i] = hi[i] = X[(int64_t)b[0] * D + i];
  for (const int32_t* v = b; v != e; ++v)
    for (int i = 0; i < D; ++i) {
      const double c = X[(int64_t)*v * D + i];
      lo[i] = std::min(lo[i], c);
      hi[i] = std::max(hi[i], c);
    }
  int ax = 0;
  for (int i = 1; i < D; ++i)
    if (hi[i] - lo[i] > hi[ax] - lo[ax]) ax = i;
  const int64_t parts = (n + bn - 1) / bn;
  const int64_t left = (int64_t)bn * (parts / 2);
  // the left set is unique under the strict order (coordinate, position)
  std::nth_element(b, b + left, e, [&](int32_t x, int32_t y) {
    const double cx = X[(int64_t)x * D + ax], cy = X[(int64_t)y * D + ax];
    return cx != cy ? cx < cy : pos[x] < pos[y];
  });
  bisect_blocks(b, b + left, X, D, pos, bn);
  bisect_blocks(b + left, e, X, D, pos, bn);
}

// new_id[caller node] = internal node (RCM, or node blocks cut from RCM bands).
static void number_nodes(pfem_mesh* m, int bn, bool blocks,
                         std::vector<int32_t>& new_id) {
  const int64_t N = m->n_nodes;
  std::vector<int32_t> q;
  const int64_t n_levels = cuthill_mckee(m, q);
  std::reverse(q.begin(), q.end());            // q[position] = caller node (RCM)
  m->band_blocks = 0;
  if (blocks) {
    std::vector<int32_t> pos(N);
    for (int64_t i = 0; i < N; ++i) pos[q[i]] = (int32_t)i;
    int64_t w = 1;
    auto ipow = [&](int64_t x) { int64_t r = 1; for (int i = 0; i < m->dim; ++i) r *= x; return r; };
    while (ipow(w + 1) <= bn) ++w;
    const int64_t k = std::max<int64_t>(
        1, std::min<int64_t>((2 * w * N + n_levels * bn) / (2 * n_levels * bn), 32768 / bn));
    const int64_t band = k * bn;
    m->band_blocks = (int)k;
    for (int64_t b0 = 0; b0 < N; b0 += band)
      bisect_blocks(q.data() + b0, q.data() + std::min(N, b0 + band), m->coords.data(),
                    m->dim, pos, bn);
  }
  new_id.assign(N, 0);
  for (int64_t i = 0; i < N; ++i) new_id[q[i]] = (int32_t)i;
}

static int64_t bandwidth(const pfem_mesh* m, const int32_t* numbering) {
  const int nv = m->nv;
  int64_t bw = 0;
  for (int64_t e = 0; e < m->n_elems; ++e) {
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    for (int a = 0; a < nv; ++a) {
      const int32_t v = numbering ? numbering[m->conn[e * nv + a]] : m->conn[e * nv + a];
      lo = std::min(lo, v);
      hi = std::max(hi, v);
    }
    bw = std::max<int64_t>(bw, hi - lo);
  }
  return bw;
}

void mesh_finalize_host(pfem_mesh* m, int block_nodes) {
  validate(m);
  const int D = m->dim;
  const int nv = m->nv;
  const int64_t N = m->n_nodes, NE = m->n_elems;
  // 0. nodes per owner block
  int bn = block_nodes;
  if (bn <= 0) {
    // N/4000 (2D) or N/750 (3D) nodes, a multiple of 32, at least 224 (2D) or
    // 64 (3D), at most 1024: measured optimum of the owner kernels on compact
    // blocks (enough workgroups to fill the chip, few halo revisits, LDS for
    // enough resident workgroups).  Also at least N/512: every workgroup of a
    // PCG vector launch and of the fused iteration sums the partials of all
    // blocks, work that grows as the square of the block count (fused FP32
    // iteration on a 2M-triangle plate: 62.5 us with 3915 blocks, 41.7 with
    // 1958, 35.7 with 979)
    const int64_t per = D == 2 ? 4000 : 750, lo = D == 2 ? 224 : 64;
    const int64_t want = std::max(N / per, (N + kBlocksSoftMax - 1) / kBlocksSoftMax);
    bn = (int)std::min<int64_t>(1024, std::max<int64_t>(lo, (want + 31) / 32 * 32));
  }
  require(bn <= block_nodes_max(), PFEM_E_INVALID_ARG, "block_nodes too large");
  // the element kernels address mesh and solver arrays with 32-bit byte
  // offsets; the largest per-node array is the FP64 fused-PCG record (4 d
  // doubles), the largest per-element one the 16-byte 3D connectivity row
  require(N * 32 * D < (int64_t(1) << 32) && NE * 16 < (int64_t(1) << 32), PFEM_E_INVALID_MESH,
          "mesh too large: at most " + std::to_string((int64_t(1) << 32) / (32 * D) - 1) +
              " nodes and 268435455 elements per mesh");
  // 1. node numbering
  number_nodes(m, bn, m->node_order == PFEM_ORDER_BLOCKS, m->perm);
  m->bw_in = bandwidth(m, nullptr);
  m->bw_int = bandwidth(m, m->perm.data());
  // 2. element order
  std::vector<int32_t> keys((size_t)NE * nv);
  for (int64_t e = 0; e < NE; ++e) {
    int32_t* k = &keys[e * nv];
    for (int a = 0; a < nv; ++a) k[a] = m->perm[m->conn[e * nv + a]];
    std::sort(k, k + nv);
  }
  m->elem_order.resize(NE);
  std::iota(m->elem_order.begin(), m->elem_order.end(), 0);
  std::sort(m->elem_order.begin(), m->elem_order.end(), [&](int32_t a, int32_t b) {
    const int32_t* ka = &keys[(size_t)a * nv];
    const int32_t* kb = &keys[(size_t)b * nv];
    for (int i = 0; i < nv; ++i)
      if (ka[i] != kb[i]) return ka[i] < kb[i];
    return a < b;
  });
  // internal connectivity (node order inside the element kept)
  m->conn_int.resize((size_t)NE * nv);
  for (int64_t s = 0; s < NE; ++s)
    for (int a = 0; a < nv; ++a)
      m->conn_int[s * nv + a] = m->perm[m->conn[(size_t)m->elem_order[s] * nv + a]];
  // 3. colouring
  std::vector<int64_t> n2e_ptr(N + 1, 0);
  for (int64_t s = 0; s < NE; ++s)
    for (int a = 0; a < nv; ++a) n2e_ptr[m->conn_int[s * nv + a] + 1]++;
  for (int64_t i = 0; i < N; ++i) n2e_ptr[i + 1] += n2e_ptr[i];
  std::vector<int32_t> n2e(n2e_ptr[N]);
  {
    std::vector<int64_t> fill(n2e_ptr.begin(), n2e_ptr.end() - 1);
    for (int64_t s = 0; s < NE; ++s)
      for (int a = 0; a < nv; ++a) n2e[fill[m->conn_int[s * nv + a]]++] = (int32_t)s;
  }
  // Greedy first fit in decreasing priority, computed as Jones-Plassmann
  // rounds (same colours): in each round every uncoloured element none of
  // whose uncoloured neighbours has a higher priority takes the smallest
  // colour its (already coloured, all higher-priority) neighbours leave free.
  // Such elements are pairwise non-adjacent, so a round runs in parallel
  // and sweeps the elements in their sorted (cache-friendly) order.
  std::vector<uint32_t> h(NE);
  for (int64_t k = 0; k < NE; ++k) h[k] = fmix32((uint32_t)k ^ 0x9E3779B9u);
  auto higher = [&](int32_t f, int32_t e) { return h[f] != h[e] ? h[f] > h[e] : f > e; };
  m->color.assign(NE, -1);
  std::vector<int32_t> active(NE), next;
  std::iota(active.begin(), active.end(), 0);
  std::vector<char> ready;
  int32_t* col = m->color.data();
  while (!active.empty()) {
    const int64_t na = (int64_t)active.size();
    ready.assign(na, 0);
    parallel_for(na, [&](int64_t b, int64_t e) {
      for (int64_t i = b; i < e; ++i) {
        const int32_t el = active[i];
        bool ok = true;
        for (int a = 0; a < nv && ok; ++a) {
          const int32_t n = m->conn_int[(size_t)el * nv + a];
          for (int64_t k = n2e_ptr[n]; k < n2e_ptr[n + 1]; ++k) {
            const int32_t f = n2e[k];
            if (f != el && col[f] < 0 && higher(f, el)) {
              ok = false;
              break;
            }
          }
        }
        ready[i] = ok;
      }
    });
    parallel_for(na, [&](int64_t b, int64_t e) {
      std::vector<int32_t> stamp(64, -1);
      for (int64_t i = b; i < e; ++i) {
        if (!ready[i]) continue;
        const int32_t el = active[i];
        for (int a = 0; a < nv; ++a) {
          const int32_t n = m->conn_int[(size_t)el * nv + a];
          for (int64_t k = n2e_ptr[n]; k < n2e_ptr[n + 1]; ++k) {
            const int32_t c = col[n2e[k]];   // never an element of this round
            if (c >= 0) {
              if ((size_t)c >= stamp.size()) stamp.resize(2 * (size_t)c + 2, -1);
              stamp[c] = el;
            }
          }
        }
        int32_t c = 0;
        while ((size_t)c < stamp.size() && stamp[c] == el) ++c;
        col[el] = c;
      }
    });
    next.clear();
    for (int64_t i = 0; i < na; ++i)
      if (!ready[i]) next.push_back(active[i]);
    const int64_t done = na - (int64_t)next.size();
    active.swap(next);
    if (!active.empty() && done < 1024) {
      // few elements per round (a node of very high degree, e.g. a fan):
      // finish with the plain greedy in decreasing priority, same colours.
      // Nodes of degree > 256 keep a bit set of the colours already used
      // around them, so an element next to such a hub costs O(colours / 64)
      // instead of a scan of the hub's whole element list.
      std::sort(active.begin(), active.end(), [&](int32_t a, int32_t b) { return higher(a, b); });
      auto set_bit = [](std::vector<uint64_t>& b, int32_t c) {
        if ((size_t)(c >> 6) >= b.size()) b.resize((size_t)(c >> 6) + 1, 0);
        b[c >> 6] |= uint64_t(1) << (c & 63);
      };
      const int64_t hub_deg = 256;
      std::vector<std::vector<uint64_t>> hub_used;
      std::vector<int32_t> hub_id(N, -1);
      for (int64_t n = 0; n < N; ++n)
        if (n2e_ptr[n + 1] - n2e_ptr[n] > hub_deg) {
          hub_id[n] = (int32_t)hub_used.size();
          hub_used.emplace_back();
          for (int64_t k = n2e_ptr[n]; k < n2e_ptr[n + 1]; ++k)
            if (col[n2e[k]] >= 0) set_bit(hub_used.back(), col[n2e[k]]);
        }
      std::vector<uint64_t> used;
      for (int32_t el : active) {
        used.assign(used.size(), 0);
        for (int a = 0; a < nv; ++a) {
          const int32_t n = m->conn_int[(size_t)el * nv + a];
          if (hub_id[n] >= 0) {
            const std::vector<uint64_t>& hb = hub_used[hub_id[n]];
            if (used.size() < hb.size()) used.resize(hb.size(), 0);
            for (size_t w = 0; w < hb.size(); ++w) used[w] |= hb[w];
            continue;
          }
          for (int64_t k = n2e_ptr[n]; k < n2e_ptr[n + 1]; ++k)
            if (col[n2e[k]] >= 0) set_bit(used, col[n2e[k]]);
        }
        int32_t c = 0;
        while ((size_t)(c >> 6) < used.size() && ((used[c >> 6] >> (c & 63)) & 1)) ++c;
        col[el] = c;
        for (int a = 0; a < nv; ++a) {
          const int32_t n = m->conn_int[(size_t)el * nv + a];
          if (hub_id[n] >= 0) set_bit(hub_used[hub_id[n]], c);
        }
      }
      active.clear();
    }
  }
  int ncol = 0;
  for (int64_t k = 0; k < NE; ++k) ncol = std::max(ncol, col[k] + 1);
  m->n_colors = ncol;
  m->color_ptr.assign(ncol + 1, 0);
  for (int64_t s = 0; s < NE; ++s) m->color_ptr[m->color[s] + 1]++;
  for (int c = 0; c < ncol; ++c) m->color_ptr[c + 1] += m->color_ptr[c];
  m->colored.resize(NE);
  {
    std::vector<int> fill(m->color_ptr.begin(), m->color_ptr.end() - 1);
    for (int64_t s = 0; s < NE; ++s) m->colored[fill[m->color[s]]++] = (int32_t)s;
  }
  // 4. free-DOF map and Dirichlet data
  const int64_t ndof = N * D;
  std::vector<char> con(ndof, 0);
  std::vector<double> dv(ndof, 0.0);
  for (size_t i = 0; i < m->dnode.size(); ++i) {
    const int64_t g = (int64_t)m->dnode[i] * D + m->dcomp[i];
    con[g] = 1;
    dv[g] = m->dval[i];
  }
  m->free_index.assign(ndof, -1);
  int64_t rank = 0;
  for (int64_t g = 0; g < ndof; ++g)
    if (!con[g]) m->free_index[g] = (int32_t)rank++;
  m->n_free = rank;
  m->dmask.assign(N, 0);
  m->ubar_int.assign(ndof, 0.0);
  for (int64_t n = 0; n < N; ++n)
    for (int c = 0; c < D; ++c)
      if (con[n * D + c]) {
        m->dmask[m->perm[n]] |= (uint8_t)(1u << c);
        m->ubar_int[(int64_t)m->perm[n] * D + c] = dv[n * D + c];
      }
  // 5. external force (App. B: t |facet| / n_f on each node of a linear
  // facet; a Q8 edge integrates its quadratic shape functions)
  std::vector<double> fext(ndof, 0.0);
  const int nfn = m->facet_nodes();
  for (int64_t f = 0; f < m->n_facets; ++f) {
    const int32_t* fn = &m->facets[f * nfn];
    const double* t = &m->traction[f * D];
    if (nfn == 3 && D == 2) {
      // nodes (end, end, middle): N = s(s-1)/2, s(s+1)/2, 1 - s^2 on
      // s in [-1, 1]; 3 Gauss points along the edge
      const double gs[3] = {-std::sqrt(0.6), 0.0, std::sqrt(0.6)};
      const double gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
      double w[3] = {0, 0, 0};
      for (int q = 0; q < 3; ++q) {
        const double sq = gs[q];
        const double N[3] = {0.5 * sq * (sq - 1), 0.5 * sq * (sq + 1), 1 - sq * sq};
        const double dN[3] = {sq - 0.5, sq + 0.5, -2 * sq};
        double tx = 0, ty = 0;
        for (int a = 0; a < 3; ++a) {
          tx += dN[a] * m->coords[(size_t)fn[a] * 2];
          ty += dN[a] * m->coords[(size_t)fn[a] * 2 + 1];
        }
        const double ds = std::sqrt(tx * tx + ty * ty);
        for (int a = 0; a < 3; ++a) w[a] += gw[q] * ds * N[a];
      }
      for (int a = 0; a < 3; ++a)
        for (int i = 0; i < 2; ++i) fext[(int64_t)fn[a] * 2 + i] += t[i] * w[a];
      continue;
    }
    double meas;
    if (D == 2) {
      const double dx = m->coords[fn[1] * 2] - m->coords[fn[0] * 2];
      const double dy = m->coords[fn[1] * 2 + 1] - m->coords[fn[0] * 2 + 1];
      meas = std::sqrt(dx * dx + dy * dy);
    } else {
      double a[3], b[3];
      for (int i = 0; i < 3; ++i) {
        a[i] = m->coords[fn[1] * 3 + i] - m->coords[fn[0] * 3 + i];
        b[i] = m->coords[fn[2] * 3 + i] - m->coords[fn[0] * 3 + i];
      }
      const double cx = a[1] * b[2] - a[2] * b[1];
      const double cy = a[2] * b[0] - a[0] * b[2];
      const double cz = a[0] * b[1] - a[1] * b[0];
      meas = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
    }
    for (int a = 0; a < D; ++a)
      for (int i = 0; i < D; ++i) fext[(int64_t)fn[a] * D + i] += t[i] * meas / D;
  }
  m->fext_int.assign(ndof, 0.0);
  double fn2 = 0.0;
  for (int64_t n = 0; n < N; ++n)
    for (int c = 0; c < D; ++c) {
      m->fext_int[(int64_t)m->perm[n] * D + c] = fext[n * D + c];
      fn2 += fext[n * D + c] * fext[n * D + c];
    }
  m->fext_norm = std::sqrt(fn2);
  // 6. internal coordinates and materials
  m->X_int.resize(ndof);
  for (int64_t n = 0; n < N; ++n)
    for (int c = 0; c < D; ++c) m->X_int[(int64_t)m->perm[n] * D + c] = m->coords[n * D + c];
  m->mu_int.resize(NE);
  m->lam_int.resize(NE);
  for (int64_t s = 0; s < NE; ++s) {
    m->mu_int[s] = m->mu[m->elem_order[s]];
    m->lam_int[s] = m->lam[m->elem_order[s]];
  }
  // 7. owner node blocks
  m->bn = bn;
  m->n_blocks = (int)((N + bn - 1) / bn);
  const int nb = m->n_blocks;
  // owned range of block b: elements whose smallest node lies in b (the
  // sort makes it contiguous); halo of b: elements owned by an earlier
  // block that have a node in b, in increasing sorted position.
  std::vector<int> own_begin(nb + 1, (int)NE);
  std::vector<std::vector<int32_t>> halo(nb);
  for (int64_t s = NE - 1; s >= 0; --s) {
    int32_t mn = m->conn_int[s * nv];
    for (int a = 1; a < nv; ++a) mn = std::min(mn, m->conn_int[s * nv + a]);
    own_begin[mn / bn] = (int)s;
  }
  for (int b = nb - 1; b >= 0; --b)   // blocks that own nothing start where the next starts
    if (own_begin[b] > own_begin[b + 1]) own_begin[b] = own_begin[b + 1];
  for (int64_t s = 0; s < NE; ++s) {
    int bl[4];
    int32_t mn = m->conn_int[s * nv];
    for (int a = 1; a < nv; ++a) mn = std::min(mn, m->conn_int[s * nv + a]);
    const int ob = mn / bn;
    int nbl = 0;
    for (int a = 0; a < nv; ++a) {
      const int b = m->conn_int[s * nv + a] / bn;
      if (b == ob) continue;
      bool seen = false;
      for (int k = 0; k < nbl; ++k) seen |= bl[k] == b;
      if (!seen) bl[nbl++] = b;
    }
    for (int k = 0; k < nbl; ++k) halo[bl[k]].push_back((int32_t)s);
  }
  m->blocks.assign(nb, make_int4(0, 0, 0, 0));
  m->halo.clear();
  m->owner_visits = 0;
  for (int b = 0; b < nb; ++b) {
    const int h0 = (int)m->halo.size();
    m->halo.insert(m->halo.end(), halo[b].begin(), halo[b].end());
    m->blocks[b] = make_int4(own_begin[b], own_begin[b + 1], h0, (int)m->halo.size());
    m->owner_visits += (own_begin[b + 1] - own_begin[b]) + (int64_t)halo[b].size();
    require(own_begin[b + 1] > own_begin[b] || !halo[b].empty(), PFEM_E_INVALID_MESH,
            "internal: node block touched by no element");
  }
  // work table: consecutive blocks on the same XCD (workgroup i runs on
  // XCD i % 8 when dispatched round-robin)
  m->work.resize(nb);
  {
    int cnt[8], pre[8];
    for (int k = 0; k < 8; ++k) cnt[k] = (nb - k + 7) / 8;
    pre[0] = 0;
    for (int k = 1; k < 8; ++k) pre[k] = pre[k - 1] + std::max(cnt[k - 1], 0);
    for (int i = 0; i < nb; ++i) m->work[i] = make_int2(0, pre[i % 8] + i / 8);
  }
  prepare_device_images(m);
  m->finalized = true;
}

// Host images of the device arrays that are not plain copies, prepared once
// at finalize so that an upload (a server admitting a request) only copies.
static void prepare_device_images(pfem_mesh* m) {
  const int D = m->dim;
  m->mu32.assign(m->mu_int.begin(), m->mu_int.end());
  m->lam32.assign(m->lam_int.begin(), m->lam_int.end());
  // 31-bit fixed-point coordinates over the bounding box (float32 kernels):
  // 0 <= q < 2^31, so the difference of any two fits a signed 32-bit integer
  // (an element spanning more than half the box must not wrap around)
  m->xq.assign(m->X_int.size(), 0u);
  for (int i = 0; i < 3; ++i) m->qscale[i] = 1.f;
  for (int i = 0; i < D; ++i) {
    double lo = 0.0, hi = 0.0;
    for (int64_t n = 0; n < m->n_nodes; ++n) {
      const double v = m->X_int[n * D + i];
      if (n == 0 || v < lo) lo = v;
      if (n == 0 || v > hi) hi = v;
    }
    const double step = hi > lo ? (hi - lo) / 2147483647.0 : 1.0;
    m->qscale[i] = (float)step;
    for (int64_t n = 0; n < m->n_nodes; ++n) {
      const double t = std::round((m->X_int[n * D + i] - lo) / step);
      m->xq[n * D + i] = (uint32_t)std::min(std::max(t, 0.0), 2147483647.0);
    }
  }
  // packed 2D connectivity: smallest node first, 16-bit offsets of the
  // other two (3D kernels read the plain 16-byte rows)
  const int nv = m->nv;
  bool packable = D == 2 && m->elem == PFEM_ELEM_P1;
  m->connp.assign(packable ? (size_t)m->n_elems * 2 : 0, 0u);
  for (int64_t s = 0; packable && s < m->n_elems; ++s) {
    const int32_t* c = &m->conn_int[s * nv];
    int amin = 0;
    for (int a = 1; a < nv; ++a)
      if (c[a] < c[amin]) amin = a;
    uint32_t off[2];
    for (int k = 1; k < nv; ++k) {
      const int64_t dlt = (int64_t)c[(amin + k) % nv] - c[amin];
      if (dlt > 65535) packable = false;
      off[k - 1] = (uint32_t)dlt;
    }
    uint32_t* o = &m->connp[s * 2];
    o[0] = (uint32_t)c[amin];
    o[1] = (off[0] & 0xffffu) | ((off[1] & 0xffffu) << 16);
  }
  if (!packable) {
    m->connp.clear();
    m->connp.shrink_to_fit();
  }
  m->halo_pad = m->halo;   // one padding entry: clamped reads
  m->halo_pad.push_back(0);
  // periodic springs: partners of every internal node, sorted (CSR)
  m->pair_ptr.clear();
  m->pair_nbr.clear();
  if (!m->pairs.empty()) {
    const int64_t np = (int64_t)m->pairs.size() / 2;
    m->pair_ptr.assign(m->n_nodes + 1, 0);
    for (int64_t q = 0; q < np; ++q) {
      ++m->pair_ptr[m->perm[m->pairs[2 * q]] + 1];
      ++m->pair_ptr[m->perm[m->pairs[2 * q + 1]] + 1];
    }
    for (int64_t n = 0; n < m->n_nodes; ++n) m->pair_ptr[n + 1] += m->pair_ptr[n];
    m->pair_nbr.assign(m->pair_ptr[m->n_nodes], 0);
    std::vector<int32_t> fill(m->pair_ptr.begin(), m->pair_ptr.end() - 1);
    for (int64_t q = 0; q < np; ++q) {
      const int32_t a = m->perm[m->pairs[2 * q]], b = m->perm[m->pairs[2 * q + 1]];
      m->pair_nbr[fill[a]++] = b;
      m->pair_nbr[fill[b]++] = a;
    }
    for (int64_t n = 0; n < m->n_nodes; ++n)
      std::sort(m->pair_nbr.begin() + m->pair_ptr[n], m->pair_nbr.begin() + m->pair_ptr[n + 1]);
  }
  // volume of the cell the coordinates span (homogenisation divides by it)
  m->cell_volume = 1.0;
  for (int i = 0; i < D; ++i) {
    double lo = 0.0, hi = 0.0;
    for (int64_t n = 0; n < m->n_nodes; ++n) {
      const double v = m->X_int[n * D + i];
      if (n == 0 || v < lo) lo = v;
      if (n == 0 || v > hi) hi = v;
    }
    m->cell_volume *= hi - lo;
  }
  // uniform lambda / mu ratio (uniform Poisson ratio): kernels stream mu only
  m->lam_uniform = false;
  m->lam_ratio = 0.0;
  if (m->n_elems > 0 && m->mu_int[0] != 0.0) {
    const double r = m->lam_int[0] / m->mu_int[0];
    bool uni = std::isfinite(r);
    for (int64_t s = 0; uni && s < m->n_elems; ++s)
      uni = std::fabs(m->lam_int[s] - r * m->mu_int[s]) <= 2e-15 * std::fabs(m->lam_int[s]);
    if (uni) {
      m->lam_uniform = true;
      m->lam_ratio = r;
    }
  }
}

// --------------------------------------------------------------- device
template <typename T>
static T* upload(const std::vector<T>& v, int64_t& bytes) {
  T* p = nullptr;
  const size_t n = std::max<size_t>(v.size(), 1) * sizeof(T);
  PFEM_HIP(hipMalloc((void**)&p, n));
  if (!v.empty()) PFEM_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  bytes += (int64_t)n;
  return p;
}

void mesh_upload(pfem_mesh* m, Ctx* ctx) {
  require(m->finalized, PFEM_E_STATE, "mesh not finalized");
  if (m->uploaded) return;
  PFEM_HIP(hipSetDevice(ctx->device));
  MeshDevBuffers& d = m->dev;
  d.bytes = 0;
  const bool packable = !m->connp.empty();
  try {
    d.X = upload(m->X_int, d.bytes);
    d.Xq = upload(m->xq, d.bytes);
    d.connp = upload(m->connp, d.bytes);
    d.conn = upload(m->conn_int, d.bytes);
    d.mu32 = upload(m->mu32, d.bytes);
    d.lam32 = upload(m->lam32, d.bytes);
    d.mu64 = upload(m->mu_int, d.bytes);
    d.lam64 = upload(m->lam_int, d.bytes);
    d.dmask = upload(m->dmask, d.bytes);
    d.blocks = upload(m->blocks, d.bytes);
    d.halo = upload(m->halo_pad, d.bytes);
    d.fext = upload(m->fext_int, d.bytes);
    d.ubar = upload(m->ubar_int, d.bytes);
    d.colored = upload(m->colored, d.bytes);
    d.perm = upload(m->perm, d.bytes);
    d.work = upload(m->work, d.bytes);
    if (!m->pair_ptr.empty()) {
      d.pair_ptr = upload(m->pair_ptr, d.bytes);
      d.pair_nbr = upload(m->pair_nbr, d.bytes);
    }
  } catch (...) {
    mesh_release_device(m);
    throw;
  }
  MeshDev& md = m->md;
  md.X = d.X;
  md.Xq = d.Xq;
  md.connp = d.connp;
  md.conn_packed = packable ? 1 : 0;
  for (int i = 0; i < 3; ++i) md.qscale[i] = m->qscale[i];
  md.conn = d.conn;
  md.mu32 = d.mu32;
  md.lam32 = d.lam32;
  md.mu64 = d.mu64;
  md.lam64 = d.lam64;
  md.dmask = d.dmask;
  md.blocks = d.blocks;
  md.halo = d.halo;
  md.fext = d.fext;
  md.ubar = d.ubar;
  md.colored = d.colored;
  md.pair_ptr = d.pair_ptr;
  md.pair_nbr = d.pair_nbr;
  md.pair_k = m->pair_ptr.empty() ? 0.0 : m->pair_k;
  md.n_nodes = (int32_t)m->n_nodes;
  md.n_elems = (int32_t)m->n_elems;
  md.n_blocks = m->n_blocks;
  md.bn = m->bn;
  md.dim = m->dim;
  md.nv = m->nv;
  md.model = m->model;
  md.nonlinear = m->nonlinear ? 1 : 0;
  // uniform lambda / mu ratio (uniform Poisson ratio): kernels stream mu only
  md.lam_uniform = m->lam_uniform ? 1 : 0;
  md.lam_ratio = m->lam_uniform ? m->lam_ratio : 0.0;
  ctx_ref(ctx);
  m->ctx = ctx;
  m->uploaded = true;
}

void CallScratch::ensure(int64_t nd, int nb) {
  if (nd <= n_dof && nb <= n_blocks && in64 != nullptr) return;
  release();
  PFEM_HIP(hipMalloc(&in64, nd * 8));
  PFEM_HIP(hipMalloc(&v64, nd * 8));
  PFEM_HIP(hipMalloc(&out64, nd * 8));
  PFEM_HIP(hipMalloc(&zero64, nd * 8));
  PFEM_HIP(hipMemset(zero64, 0, nd * 8));
  PFEM_HIP(hipMalloc((void**)&part, (size_t)std::max(nb, 1) * kRedSlots * 8));
  PFEM_HIP(hipMalloc((void**)&out, kRedSlots * 8));
  n_dof = nd;
  n_blocks = nb;
}

void CallScratch::release() {
  if (in64) (void)hipFree(in64);
  if (v64) (void)hipFree(v64);
  if (out64) (void)hipFree(out64);
  if (zero64) (void)hipFree(zero64);
  if (part) (void)hipFree(part);
  if (out) (void)hipFree(out);
  in64 = v64 = out64 = zero64 = nullptr;
  part = nullptr;
  out = nullptr;
  n_dof = 0;
  n_blocks = 0;
}

void mesh_release_device(pfem_mesh* m) {
  const bool held = m->uploaded;
  if (held && m->ctx != nullptr && m->ctx->stream != nullptr)
    (void)hipStreamSynchronize(m->ctx->stream);
  m->solve_state.reset();
  m->scratch.release();
  MeshDevBuffers& d = m->dev;
  void* ptrs[] = {d.X, d.Xq, d.conn, d.connp, d.mu32, d.lam32, d.mu64, d.lam64, d.dmask, d.blocks,
                  d.halo, d.fext, d.ubar, d.colored, d.perm, d.work, d.pair_ptr,
                  d.pair_nbr, d.coarse_rel64, d.coarse_rel32, d.coarse_B32, d.coarse_B64};
  for (void* p : ptrs)
    if (p != nullptr) (void)hipFree(p);
  d = MeshDevBuffers{};
  m->md = MeshDev{};
  m->uploaded = false;
  if (held) {
    ctx_unref(m->ctx);
    m->ctx = nullptr;
  }
}

int64_t mesh_device_bytes(const pfem_mesh* m) {
  const int64_t N = m->n_nodes, NE = m->n_elems, D = m->dim;
  auto r = [](int64_t b) { return std::max<int64_t>(b, 1); };
  return r(N * D * 8) + r(N * D * 4) + r(NE * m->nv * 4) +
         r(D == 2 && m->elem == PFEM_ELEM_P1 ? NE * 8 : 0) + 2 * r(NE * 4) + 2 * r(NE * 8) + r(N) +
         r((int64_t)m->n_blocks * 16) + r(((int64_t)m->halo.size() + 1) * 4) + 2 * r(N * D * 8) +
         r(NE * 4) + r(N * 4) + r((int64_t)m->n_blocks * 8) +
         (m->pair_ptr.empty() ? 0 : r((N + 1) * 4) + r((int64_t)m->pair_nbr.size() * 4));
}

int64_t solve_bytes(const pfem_mesh* m, int prec, bool fused_pcg, bool two_level) {
  const int64_t nd = m->n_dof();
  const int64_t s = prec == PFEM_FP64 ? 8 : 4;
  int64_t b = 3 * nd * 8 + (6 + (fused_pcg ? 9 : 0)) * nd * s +
              (int64_t)m->n_blocks * 2 * kRedSlots * 8 + 4096 + (int64_t)8 * 65536 +
              nh_cache_values(m) * s;
  if (two_level) {   // the solve's own arrays and the mesh's coarse arrays
    const int64_t G = coarse_group(m);
    const int64_t n_agg = (m->n_blocks + G - 1) / G;
    const int64_t n_c = n_agg * (m->dim == 2 ? 3 : 6);
    b += (int64_t)m->n_blocks * 48 + n_agg * 48 + 8 * (n_c / kCoarseRows + 1) + 1024 +
         coarse_device_bytes(m);
  }
  return b;
}

int64_t nh_cache_values(const pfem_mesh* m) {
  if (!m->nonlinear || m->elem != PFEM_ELEM_P1) return 0;
  return (int64_t)(m->dim * m->dim + 1) * m->n_elems;
}

bool krylov_fused(const pfem_solve_opts& o, const pfem_mesh* m) {
  if (o.krylov != PFEM_KRYLOV_AUTO) return o.krylov == PFEM_KRYLOV_FUSED;
  if (o.precond == PFEM_PRECOND_TWO_LEVEL) return false;   // classic loop only
  if (m->elem != PFEM_ELEM_P1) return false;                // quadrilaterals: classic loop
  // Measured warm FP32 solves to 1e-8 with the automatic owner blocks
  // (fused against classic, ms): plates with holes 200k triangles 55 / 82,
  // 600k 173 / 209, 1M 308 / 449, 2M 822 / 1003 -- the fused form needs
  // up to 20% more products on the plates but saves two launches and two
  // vector passes per iteration; Neo-Hookean boxes 515k tets 65 / 75, 1M
  // tets 133 / 134; linear boxes 515k 48 / 53, 1M 105 / 104.  Fused in 2D
  // at every size, in 3D up to 800k tetrahedra (beyond, a tie).
  const int64_t limit = m->dim == 2 ? INT64_MAX : 800000;
  // periodic springs are applied by the owner kernels only (classic loop)
  return o.prec == PFEM_FP32 && m->n_elems <= limit && m->pairs.empty();
}

}  // namespace pfem

pfem_mesh::~pfem_mesh() = default;
