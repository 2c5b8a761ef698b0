// Mesh handle: caller input, bit-exact preprocessing, device arrays.
#pragma once

#include <memory>
#include <vector>

#include "pfem_internal.h"

namespace pfem {

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
  bool fused = false;       // fused PCG records present
  void* rec[2] = {nullptr, nullptr};   // fused PCG: {r, w, s, M^-1} per node, by parity
  void* tmp = nullptr;
  double* part = nullptr;   // 2 * kRedSlots * n_blocks (two slot sets)
  Scalars* sc = nullptr;
  double* hist = nullptr;
  int64_t hist_cap = 0;
  int64_t bytes = 0;
  void alloc(int prec, int64_t n_dof, int n_blocks, int64_t hist_cap, bool nonlinear,
             bool fused_pcg);
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

  // device
  bool uploaded = false;
  pfem::MeshDevBuffers dev;
  pfem::MeshDev md{};
  pfem::CallScratch scratch;
  std::unique_ptr<pfem::SolveState> solve_state;   // cached for pfem_solve

  int64_t n_dof() const { return n_nodes * dim; }
};

struct pfem_ctx {
  pfem::Ctx* c = nullptr;
};

namespace pfem {
void mesh_finalize_host(pfem_mesh* m, int block_nodes);
void mesh_upload(pfem_mesh* m, Ctx* ctx);
void mesh_release_device(pfem_mesh* m);
int64_t mesh_device_bytes(const pfem_mesh* m);
int64_t solve_bytes(const pfem_mesh* m, int prec, bool fused_pcg);
// Whether a solve with these options runs the fused (one launch per
// iteration) PCG.
bool krylov_fused(const pfem_solve_opts& o, const pfem_mesh* m);
void lame_from_params(int model, int param_kind, double p0, double p1, double* mu,
                      double* lam);
uint32_t fmix32(uint32_t h);
}  // namespace pfem
