// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pfem.h"

namespace pfem {

constexpr int kThreads = 256;       // threads per workgroup (4 wave64s)
constexpr int kRedSlots = 4;        // partial sums per block per reduction

// ------------------------------------------------------------------ errors
struct Error {
  pfem_status code;
  std::string msg;
};
void set_error(const std::string& msg);
const char* last_error_cstr();

#define PFEM_HIP(call)                                                       \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      throw ::pfem::Error{PFEM_E_DEVICE,                                     \
                          std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

inline void require(bool ok, pfem_status code, const std::string& msg) {
  if (!ok) throw Error{code, msg};
}
// literal messages: no string is built unless the check fails (hot loops)
inline void require(bool ok, pfem_status code, const char* msg) {
  if (!ok) throw Error{code, std::string(msg)};
}

// Native vector types: HIP's float2/double2/int4 wrappers copy through
// generic references, which would turn a global load back into a flat one.
typedef float pf2 __attribute__((ext_vector_type(2)));
typedef float pf4 __attribute__((ext_vector_type(4)));
typedef double pd2 __attribute__((ext_vector_type(2)));
typedef int pi4 __attribute__((ext_vector_type(4)));
// three consecutive 4-byte values (a 3D node's coordinates or DOFs), loaded
// as one 12-byte access
template <typename T>
struct Trip {
  T x, y, z;
};

// ------------------------------------------------------- device descriptors
// Everything a kernel needs to know about one finalized mesh (POD).
struct MeshDev {
  const double* X;        // n_nodes * dim, internal node order
  const uint32_t* Xq;     // n_nodes * dim 31-bit fixed-point coordinates (float32 kernels):
                          // X = lo + q * qscale, per dimension
  const int32_t* conn;    // n_elems * nv, sorted element order, internal ids
  const uint32_t* connp;  // packed 2D connectivity (conn_packed): per element
                          // the smallest node, then the 16-bit offsets of the
                          // other two in one word; node order inside the
                          // element rotated so the smallest comes first
  const float* mu32;      // n_elems
  const float* lam32;     // n_elems
  const double* mu64;     // n_elems
  const double* lam64;    // n_elems
  const uint8_t* dmask;   // n_nodes, bit c set when component c is Dirichlet
  const int4* blocks;     // n_blocks: (first owned elem, end owned, halo begin, halo end)
  const int32_t* halo;    // elements owned by earlier blocks that touch a block
  const double* fext;     // n_dof, internal order
  const double* ubar;     // n_dof, final Dirichlet values, 0 on free DOFs
  const int32_t* colored; // n_elems: sorted element ids grouped by colour
  int32_t n_nodes, n_elems, n_blocks, bn;
  int32_t dim, model, nonlinear;
  int32_t lam_uniform;    // 1: lambda = lam_ratio * mu on every element (lam arrays unread)
  int32_t conn_packed;    // 1: kernels read connp (every offset fits 16 bits)
  int32_t nv;             // nodes per element (conn row length)
  double lam_ratio;
  float qscale[3];        // fixed-point coordinate step per dimension
  // periodic springs (virtual elements of a periodic cell): node n's
  // partners are pair_nbr[pair_ptr[n] .. pair_ptr[n+1]), each joined to it
  // by a spring of stiffness pair_k; pair_ptr == nullptr: no springs
  const int32_t* pair_ptr;
  const int32_t* pair_nbr;
  double pair_k;
};

// Partial sums of one task: slot k of block b at part[k * n_blocks + b].
// The kernel after the producing one (or a one-workgroup reduction kernel)
// sums them in block order, so no workgroup waits for another and no fence
// is needed.
struct RedDev {
  double* part;           // kRedSlots * n_blocks partial sums
  double* out;            // reduced sums land here (kRedSlots doubles)
};

// Per-slot scalars of the Krylov state machine (device-resident).  Values a
// kernel reads while its own block 0 may update them are double-buffered by
// iteration parity (rz2).
struct Scalars {
  double rz2[2];          // r.M^-1 r after an even / odd number of iterations
  double pq, rr, alpha, beta;
  double rho;             // latest |r| / den
  double den;             // |r_f(lifted)| (denominator of the relative residual)
  double target2;         // stop when |r|^2 <= target2
  double bnorm;           // |r| at inner start
  double red[kRedSlots];  // outputs of one-workgroup reductions
  double pa[2], pg[2];    // fused PCG: alpha_j and gamma_j by parity of j
  double lsred[2];        // line search: slope g.d (first trial)
  int32_t k;              // Krylov iterations done in the current inner solve
  int32_t kmax;           // cap for the current inner solve
  int32_t state;          // 0 running, 1 converged, 2 max-iter, 3 breakdown
  int32_t hist_len, hist_cap, total_k, pad0, pad1;
};

// Two-level preconditioner state of one solve (device memory): the mesh's
// coarse arrays and the solve's restriction partials and coarse correction.
struct TwoLevelDev {
  const void* rel;        // n_nodes * dim coordinates relative to the aggregate centroid
                          // (kernel precision)
  const void* B;          // n_c * n_c raw-mode coarse correction T A_c^-1 T^T (kernel
                          // precision), row-major, symmetric
  double* rc_part;        // n_blocks * 6: per owner block, raw-mode sums of the residual
  double* y;              // n_agg * 6: raw-mode coefficients of the coarse correction
  double* gc_part;        // n_chunks partials of (R^T r) . y
  int32_t nrb, G, n_agg, n_c, n_chunks, pad;
};
// Element kernel families: P1 meshes launch by their dimension (2, 3);
// quadrilateral meshes by these codes (their nodes per element).
constexpr int kKindQ4 = 4;
constexpr int kKindQ8 = 8;
inline int elem_kind(int dim, int elem) {
  return elem == PFEM_ELEM_Q4 ? kKindQ4 : elem == PFEM_ELEM_Q8 ? kKindQ8 : dim;
}
inline bool is_quad_kind(int kind) { return kind == kKindQ4 || kind == kKindQ8; }
constexpr int kCoarseRows = 8;   // rows of B per workgroup of the coarse solve
// Largest coarse dimension: the device applies the coarse inverse as one
// dense matrix-vector product per iteration.
constexpr int kCoarseMax = 1536;

// One unit of work for a launch: a mesh plus operand pointers.
struct Task {
  MeshDev m;
  const void* u;          // state (Neo-Hookean) / input of force, energy, diag
  const void* v;          // direction (HVP), increment (line search)
  void* y;                // output vector (owned nodes written)
  const void* w;          // dot partner of y (or nullptr)
  RedDev red;
  Scalars* sc;            // Krylov scalars (PCG launches)
  double* hist;           // residual history (PCG launches)
  const void* minv;       // inverse Jacobi diagonal (PCG launches)
  void* r;                // Krylov residual (PCG launches)
  void* p;                // search direction (PCG launches)
  void* d;                // correction accumulated by PCG (PCG launches)
  double s;               // step length (line search); inverse flag (diagonal)
  double fscale;          // load factor applied to f_ext (load steps)
  int32_t mask;           // PFEM_MASK_* bits
  int32_t active;         // 0: every workgroup of this task returns at once
  int32_t k_base;         // Krylov iterations done before this chunk (PCG)
  int32_t hist_base;      // history index of iteration 0 of this inner solve (PCG)
  int32_t pcg;            // 1: PCG apply (returns at once unless state == 0)
  int32_t no_pairs;       // 1: elements only, without the mesh's periodic springs
  const double* fext;     // external force of this task (nullptr: the mesh's)
  const TwoLevelDev* tl;  // two-level preconditioner (nullptr: Jacobi)
  // Fused PCG: per-node records {r, w, s, M^-1} (4 * dim values, kernel
  // precision) by iteration parity -- launch j gathers rec[j & 1] and its
  // owners write rec[(j + 1) & 1] -- and a scratch vector for the start.
  void* rec[2];
  void* tmp;
};

// Relocatable operands.  With rel != 0 the u, v, y fields of every task of
// a launch hold element offsets instead of pointers, and the base pointers
// and the mask come with the launch: a batch of meshes keeps one persistent
// device task table instead of uploading one per call.
struct BaseArgs {
  const void* u;
  const void* v;
  void* y;
  int32_t rel;
  int32_t mask;
};

template <typename T>
__host__ __device__ inline T* operand(void* field, void* base, int rel) {
  return rel ? static_cast<T*>(base) + reinterpret_cast<uintptr_t>(field) : static_cast<T*>(field);
}

// Element-kernel operations.
// OP_HVPC: the Neo-Hookean Hessian-vector product with the element state
// {F^-T, ln J} read from a per-element cache (the task's u) instead of
// evaluated from the nodal state (P1 meshes, owner scatter).
enum ElemOp { OP_APPLY = 0, OP_FORCE = 1, OP_DIAG = 2, OP_HVPC = 3 };
constexpr bool is_apply_op(int op) { return op == OP_APPLY || op == OP_HVPC; }

// Kernel timing families (pfem_ctx_kernel_time).
enum Family { FAM_APPLY = 0, FAM_FORCE = 1, FAM_ENERGY = 2, FAM_DIAG = 3,
              FAM_UPDATE = 4, FAM_DIRECTION = 5, FAM_FUSED = 6, FAM_COUNT = 7 };

// ----------------------------------------------------- launch descriptors
struct Ctx;
// Staging ring: small launch descriptors go host(pinned) -> device here.
class ArgRing {
 public:
  void init(size_t bytes, hipStream_t s);
  void release();
  // Copies `n` bytes to device memory valid for launches enqueued next.
  void* put(const void* src, size_t n);
 private:
  static constexpr int kSeg = 8;
  char* host_ = nullptr;
  char* dev_ = nullptr;
  size_t cap_ = 0, off_ = 0;
  int seg_ = 0;
  hipEvent_t ev_[kSeg] = {};
  bool used_[kSeg] = {};
  hipStream_t stream_ = nullptr;
};

struct Ctx {
  std::atomic<int> refs{1};   // handle + every uploaded mesh / batch
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  ArgRing ring;
  int timing = 0;          // bitmask of timed families
  int sample_every = 1;    // time one launch in this many per family
  int64_t fam_seen[FAM_COUNT] = {};
  int64_t fam_launches[FAM_COUNT] = {};
  double fam_ms[FAM_COUNT] = {};
  // launches that did work (timed or not; launches of a group that returned
  // at once because every solve in it had converged are not counted) and
  // their algorithmic bytes: for the K.v / HVP apply and the fused PCG
  // iteration of solves, while the family is timed
  int64_t fam_run[FAM_COUNT] = {};
  double fam_alg_bytes[FAM_COUNT] = {};
  struct Timed {
    int fam;
    hipEvent_t a, b;
    int64_t key;          // launch group (-1: none)
    int it;               // iteration index inside the group
    int count;            // launches between the two events
  };
  std::vector<Timed> pending;
  std::vector<hipEvent_t> event_pool;
  int64_t cur_key = -1;   // tag for the launches being enqueued
  int cur_it = 0;
  int64_t next_key = 0;
  void timing_begin(int fam, hipEvent_t* a);
  void timing_end(int fam, hipEvent_t a);
  // One event pair around `count` consecutive launches of one family (no
  // sampling): the average per launch excludes the event overhead.
  void timing_begin_run(int fam, hipEvent_t* a);
  void timing_end_run(int fam, hipEvent_t a, int count);
  void drain_timing();
  // Forget timed launches of group `key` with iteration index >= keep (and
  // runs that include one): they returned at once because their solve had
  // already converged.
  void drop_noop(int64_t key, int keep);
};

// Contexts live until their handle and every mesh or batch using them are
// released, whatever order the caller destroys them in.
void ctx_ref(Ctx* c);
void ctx_unref(Ctx* c);

// ---------------------------------------------------------------- launchers
// All launchers enqueue on ctx->stream.  `tasks_dev` points to n_tasks Task
// structs in device memory; `work_dev` to n_work (task, block) pairs.
void launch_elem(Ctx* ctx, int dim, int prec, int op, bool nonlinear, int scatter_mode,
                 const Task* tasks_dev, const int2* work_dev, int n_work,
                 int bn_max, const Task* host_task_for_alt,
                 const std::vector<int>* color_ptr, const BaseArgs* rel = nullptr);
// K.v for nr (<= 6) right-hand sides on one linear 3D mesh, every element
// visited once for all of them: tasks_dev[r] carries right-hand side r (all
// on the same mesh); work_dev is the mesh's own work table.  Usable when
// owner_multi_fits(bn, nr) (the accumulators fit 64 KB of LDS).
bool owner_multi_fits(int bn, int nr);
void launch_owner_multi(Ctx* ctx, int prec, const Task* tasks_dev, int nr,
                        const int2* work_dev, int n_work, int bn);
// Records, with `device` current, the device address of the allocation-free
// entry point's scratch array (once per device; pfem_ctx_create calls it).
void noalloc_init(int device);
void launch_energy(Ctx* ctx, int dim, int prec, bool diff,
                   const Task* tasks_dev, const int2* work_dev, int n_work,
                   const BaseArgs* rel = nullptr);
// Quadrilateral element kernels (kind kKindQ4 / kKindQ8; owner scatter),
// called by launch_elem / launch_energy.
void launch_quad_elem(Ctx* ctx, int kind, int prec, int op, bool nonlinear, const Task* tasks,
                      const int2* work, int n_work, int bn_max, const BaseArgs& ba);
void launch_quad_energy(Ctx* ctx, int kind, int prec, bool diff, const Task* tasks,
                        const int2* work, int n_work, const BaseArgs& ba);
// PCG vector passes over owned node blocks.
void launch_pcg_init(Ctx* ctx, int dim, int prec, const Task* tasks_dev,
                     const int2* work_dev, int n_work, int n_tasks);
void launch_pcg_update(Ctx* ctx, int dim, int prec, const Task* tasks_dev,
                       const int2* work_dev, int n_work, int it);
void launch_pcg_direction(Ctx* ctx, int dim, int prec, const Task* tasks_dev,
                          const int2* work_dev, int n_work, int it);
// Fused PCG (one element launch per iteration).  init: r = -g into rec[0]
// (s = 0, M^-1 copied), p = u = M^-1 r, d = 0, partials (r.u, r.r) in slots
// 1, 2; the caller then applies tmp = A p (partial in slot 0), calls
// init_w (w of rec[0] = tmp) and the classic init_finish.
void launch_fcg_init(Ctx* ctx, int dim, int prec, const Task* tasks_dev,
                     const int2* work_dev, int n_work);
void launch_fcg_init_w(Ctx* ctx, int dim, int prec, const Task* tasks_dev,
                       const int2* work_dev, int n_work);
void launch_pcg_init_finish(Ctx* ctx, const Task* tasks_dev, int n_tasks);
// Two-level preconditioned PCG (classic loop): the start r = -g with the
// restriction partials, the coarse solve over (task, chunk) work items,
// p = M^-1 r; each iteration's update with restriction partials, coarse
// solve, and the direction p = M^-1 r + beta p.
void launch_tl_init(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                    int n_work);
void launch_tl_coarse(Ctx* ctx, int prec, const Task* tasks, const int2* cwork, int n_cwork,
                      int init);
void launch_tl_prolong_init(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                            int n_work);
void launch_tl_update(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                      int n_work, int it);
void launch_tl_direction(Ctx* ctx, int dim, int prec, const Task* tasks, const int2* work,
                         int n_work, int it);
// packed: every task of the launch has packed connectivity (see MeshDev).
// Neo-Hookean P1: F^-T and ln J of every element of each task's state u
// into its y (the cache that OP_HVPC reads); owner work table.
void launch_nh_cache(Ctx* ctx, int dim, int prec, const Task* tasks_dev, const int2* work_dev,
                     int n_work);
void launch_fcg_iter(Ctx* ctx, int dim, int prec, bool nonlinear, const Task* tasks_dev,
                     const int2* work_dev, int n_work, int bn_max, int it, bool packed);
// One workgroup per task: red.out[0..n_slots-1] = sums of partial slots
// 0..n_slots-1 (n_slots 2 or 3).
void launch_reduce_store(Ctx* ctx, const Task* tasks_dev, int n_tasks, int n_slots = 2);
// out[i] = energy of reduction i (red[i * stride]), +inf where red[i * stride + 1]
// (elements with J <= 0) is nonzero.
void launch_energy_out(Ctx* ctx, const double* red, double* out, int n, int stride);
void launch_dot(Ctx* ctx, int dim, int prec, const Task* tasks_dev,
                const int2* work_dev, int n_work);
void launch_set_scalars(Ctx* ctx, Scalars* sc, double den, double target2, int kmax,
                        bool reset_hist, bool reset_total);
// Misc vector kernels (grid-stride, single vector).
void launch_permute(Ctx* ctx, int prec, int dim, const int32_t* perm,
                    int64_t n_nodes, bool to_internal, const void* in, void* out);
void launch_fill(Ctx* ctx, int prec, void* p, int64_t n, double value);
// Homogenisation: the six affine fields eps0^(IJ) . X of a 3D mesh (FP64
// coordinates, internal order, six fields one after the other), and the 6 x 6
// Gram matrix out[6 k + l] = scale A_k . B_l of six n-vectors each, through
// gram6_parts(n) float64 partials per product.
void launch_affine6(Ctx* ctx, const double* X, int64_t n_nodes, double* out);
int gram6_parts(int64_t n);
void launch_gram6(Ctx* ctx, const double* A, const double* B, int64_t n, double* part,
                  double* out, double scale);
void launch_cast(Ctx* ctx, bool to32, const void* in, void* out, int64_t n);
// x64 = base64 + s * inc (inc precision `prec`), then Dirichlet DOFs of the
// result set to scale * ubar (when set_dirichlet).
void launch_axpy_state(Ctx* ctx, int prec, const MeshDev& m, double* out,
                       const double* base, const void* inc, double s,
                       bool set_dirichlet, double scale);
// out = scale * ubar on Dirichlet DOFs, keep others of `base` (or 0 if base null)
void launch_lift(Ctx* ctx, const MeshDev& m, double* out, const double* base,
                 double scale);

// Device-side access through the global address space: pointers read from
// descriptor structs are generic, and generic (flat) accesses make the
// compiler wait on both the vector and the LDS/scalar counters.
#if defined(__HIP_DEVICE_COMPILE__)
#define PFEM_GLOBAL __attribute__((address_space(1)))
#else
#define PFEM_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ T ldg(const T* p) {
  return *(const PFEM_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ void stg(T* p, T v) {
  *(PFEM_GLOBAL T*)p = v;
}
// Element i of a device array through a 32-bit byte offset (mesh arrays
// stay below 4 GiB, checked at upload): with a uniform base pointer the
// load takes the scalar-base + 32-bit-offset form and needs no 64-bit
// address arithmetic per lane.
template <typename T>
__device__ __forceinline__ T ldx(const T* base, uint32_t i) {
  return *(const PFEM_GLOBAL T*)((const PFEM_GLOBAL char*)base + i * (uint32_t)sizeof(T));
}

// Host-side helpers.
int block_nodes_max();  // largest block size the kernels accept

}  // namespace pfem
