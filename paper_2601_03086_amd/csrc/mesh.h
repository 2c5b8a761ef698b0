// Mesh handle: caller input, bit-exact preprocessing, device arrays.
#pragma once

#include <memory>
#include <mutex>
#include <vector>

#include "pfem_internal.h"

namespace pfem {

struct CoarseHost {
  int n_rb = 0;              // rigid modes per aggregate (3 in 2D, 6 in 3D)
  int G = 1;                 // owner blocks per aggregate
  int n_agg = 0, n_c = 0;    // aggregates, coarse DOFs (n_agg * n_rb)
  std::vector<double> cent;  // n_agg * 3 centroids (internal coordinates)
  std::vector<double> T;     // n_agg * n_rb * n_rb: column k = raw-mode coefficients of
                             // the aggregate's orthonormal coarse DOF k (0: dropped)
  std::vector<double> B;     // n_c * n_c, row-major: T (P^T K P)^-1 T^T, the coarse
                             // correction in raw-mode coordinates
};

// Device-resident solver state for one solve (one slot).
struct SolveState {
  int prec = PFEM_FP32;
  int64_t n_dof = 0;
  int n_blocks = 0;
  double* x64 = nullptr;    // current state (caller's solution, internal order)
  double* g64 = nullptr;    // float64 gradient / residual at x64
  double* aux64 = nullptr;  // lifted state / scratch
  void* d = nullptr;        // Krylov correction
  void* r = nullptr;
  void* p = nullptr;
  void* q = nullptr;
  void* minv = nullptr;
  void* u32 = nullptr;      // float32 copy of the state (FP32 Neo-Hookean HVP)
  void* nhc = nullptr;      // Neo-Hookean P1: per-element {F^-T, ln J} of the Newton
                            // state, (dim^2 + 1) arrays of n_elems (kernel precision)
  bool fused = false;       // fused PCG records present
  void* rec[2] = {nullptr, nullptr};   // fused PCG: {r, w, s, M^-1} per node, by parity
  void* tmp = nullptr;
  double* part = nullptr;   // 2 * kRedSlots * n_blocks (two slot sets)
  Scalars* sc = nullptr;
  double* hist = nullptr;
  int64_t hist_cap = 0;
  // two-level preconditioner: restriction partials, coarse correction,
  // coarse partials of r.M^-1 r, and the descriptor the kernels read
  double* rc_part = nullptr;
  double* tl_y = nullptr;
  double* gc_part = nullptr;
  TwoLevelDev* tl_dev = nullptr;
  int64_t bytes = 0;
  void alloc(int prec, int64_t n_dof, int n_blocks, int64_t hist_cap, bool nonlinear,
             bool fused_pcg, int64_t nh_cache_values);
  // Adds the two-level arrays for the mesh's coarse space (uploaded).
  void alloc_two_level(const pfem_mesh* m);
  void release();
  ~SolveState() { release(); }
};

struct MeshDevBuffers {
  double* X = nullptr;
  uint32_t* Xq = nullptr;
  int32_t* conn = nullptr;
  uint32_t* connp = nullptr;
  float* mu32 = nullptr;
  float* lam32 = nullptr;
  double* mu64 = nullptr;
  double* lam64 = nullptr;
  uint8_t* dmask = nullptr;
  int4* blocks = nullptr;
  int32_t* halo = nullptr;
  double* fext = nullptr;
  double* ubar = nullptr;
  int32_t* colored = nullptr;
  int32_t* perm = nullptr;
  int2* work = nullptr;      // single-mesh work table (XCD-remapped)
  int32_t* pair_ptr = nullptr;
  int32_t* pair_nbr = nullptr;
  // two-level preconditioner (uploaded on first use)
  double* coarse_rel64 = nullptr;  // node coordinates relative to their aggregate's centroid
  float* coarse_rel32 = nullptr;
  float* coarse_B32 = nullptr;     // raw-mode coarse correction matrix
  double* coarse_B64 = nullptr;
  int64_t bytes = 0;
};

// Scratch for kernel-level calls (lazily allocated, reused).
struct CallScratch {
  void* in64 = nullptr;
  void* v64 = nullptr;
  void* out64 = nullptr;
  void* zero64 = nullptr;   // all-zero state (K = K_T(0))
  double* part = nullptr;
  double* out = nullptr;
  int64_t n_dof = 0;
  int n_blocks = 0;
  void ensure(int64_t n_dof, int n_blocks);
  void release();
};

}  // namespace pfem

struct pfem_mesh {
  pfem::Ctx* ctx = nullptr;
  int dim = 0;
  int elem = PFEM_ELEM_P1;          // element family (PFEM_ELEM_*)
  int nv = 0;                       // nodes per element
  int64_t n_nodes = 0, n_elems = 0;
  std::vector<double> coords;       // caller order
  std::vector<int32_t> conn;        // caller order
  int model = -1;
  bool nonlinear = false;
  std::vector<double> mu, lam;      // caller element order
  std::vector<int32_t> dnode;
  std::vector<int8_t> dcomp;
  std::vector<double> dval;
  std::vector<int32_t> facets;
  std::vector<double> traction;
  int64_t n_facets = 0;
  std::vector<int32_t> pairs;       // periodic node pairs (caller ids), 2 per pair
  double pair_k = 0.0;              // spring stiffness of every pair

  int node_order = PFEM_ORDER_BLOCKS;
  bool finalized = false;
  // preprocessing (bit-exact hooks)
  std::vector<int32_t> perm;        // caller node -> internal node
  std::vector<int32_t> elem_order;  // sorted position -> caller element
  std::vector<int32_t> color;       // per sorted element
  std::vector<int32_t> free_index;  // caller DOF -> free rank or -1
  std::vector<int> color_ptr;       // colour CSR
  std::vector<int32_t> colored;     // sorted element ids grouped by colour
  std::vector<int4> blocks;         // (own begin, own end, halo begin, halo end)
  std::vector<int32_t> halo;        // halo element lists of all blocks
  std::vector<int2> work;           // single-mesh work table
  int bn = 0, n_blocks = 0, n_colors = 0;
  int band_blocks = 0;   // owner blocks per RCM band (block numbering; 0 under plain RCM)
  int64_t n_free = 0, bw_in = 0, bw_int = 0, owner_visits = 0;
  double fext_norm = 0.0;
  // internal-order arrays
  std::vector<double> X_int;
  std::vector<int32_t> conn_int;
  std::vector<double> mu_int, lam_int;
  std::vector<uint8_t> dmask;
  std::vector<double> fext_int, ubar_int;
  // device images prepared on the host at finalize, so an upload only copies
  std::vector<uint32_t> xq;         // 31-bit fixed-point coordinates (float32 kernels)
  float qscale[3] = {1.f, 1.f, 1.f};
  std::vector<uint32_t> connp;      // packed 2D connectivity (empty: not packable)
  std::vector<float> mu32, lam32;
  std::vector<int32_t> halo_pad;    // halo lists + one padding entry (clamped reads)
  bool lam_uniform = false;         // lambda = lam_ratio * mu on every element
  double lam_ratio = 0.0;
  std::vector<int32_t> pair_ptr, pair_nbr;   // spring partners per internal node (CSR)
  double cell_volume = 0.0;         // volume of the coordinates' bounding box

  // device
  bool uploaded = false;
  pfem::MeshDevBuffers dev;
  pfem::MeshDev md{};
  pfem::CallScratch scratch;
  std::unique_ptr<pfem::SolveState> solve_state;   // cached for pfem_solve
  std::unique_ptr<pfem::CoarseHost> coarse;        // two-level preconditioner (built on use)
  std::mutex coarse_mu;
  ~pfem_mesh();

  int64_t n_dof() const { return n_nodes * dim; }
  // nodes of a Neumann facet: an edge (2D), a triangle (3D), a 3-node edge (Q8)
  int facet_nodes() const { return elem == PFEM_ELEM_Q8 ? 3 : dim; }
  // what the element launches dispatch on (pfem::elem_kind)
  int kind() const { return pfem::elem_kind(dim, elem); }
};

struct pfem_ctx {
  pfem::Ctx* c = nullptr;
};

namespace pfem {
void mesh_finalize_host(pfem_mesh* m, int block_nodes);
void mesh_upload(pfem_mesh* m, Ctx* ctx);
void mesh_release_device(pfem_mesh* m);
int64_t mesh_device_bytes(const pfem_mesh* m);
int64_t solve_bytes(const pfem_mesh* m, int prec, bool fused_pcg, bool two_level);
// Values of the per-element Neo-Hookean cache of a solve on m (0: none).
int64_t nh_cache_values(const pfem_mesh* m);
// Whether a solve with these options runs the fused (one launch per
// iteration) PCG.
bool krylov_fused(const pfem_solve_opts& o, const pfem_mesh* m);
void lame_from_params(int model, int param_kind, double p0, double p1, double* mu,
                      double* lam);
uint32_t fmix32(uint32_t h);
}  // namespace pfem
