/*
 * pfem.h -- C ABI of the P1 finite-element physics library for MI355X (gfx950).
 *
 * What the library computes (arXiv 2601.03086, "Pretrain Finite Element
 * Method"):
 *   - the total potential Pi(u) = sum_e vol_e Psi(grad u) - f_ext . u used as
 *     the physics-informed loss (Sec. 'Linear elastic plate with arbitrary
 *     holes' and Sec. 'Nonlinear hyperelasticity', loss equations);
 *   - its gradient f_int(u) - f_ext (App. B, total-Lagrangian internal
 *     force) and its Hessian-vector product (App. B, K_mat + K_geo), applied
 *     matrix-free;
 *   - warm-started iterative solves (Sec. 'Warm-start', iteration and
 *     stopping equations; App. B): Jacobi-preconditioned CG for linear
 *     elasticity and Newton-Krylov with load steps for Neo-Hookean
 *     hyperelasticity, whose initial guess U0 may come from a network;
 *   - a serving loop that admits solve requests by device-memory footprint
 *     and advances all live requests together (continuous batching).
 *
 * Elements are P1 triangles (dim 2) and tetrahedra (dim 3).
 *
 * Conventions
 *   - Every function returns pfem_status: 0 OK, > 0 completed with a
 *     warning, < 0 error.  On error outputs are unspecified and
 *     pfem_last_error() returns a message (thread-local, valid until the
 *     next call on the same thread).  No C++ exception crosses the ABI.
 *   - Indices are 0-based int32.  A DOF index is g = node * dim + comp in
 *     the CALLER's node numbering unless a call takes PFEM_LAYOUT_INTERNAL,
 *     in which case vectors are in the library's internal node order (see
 *     pfem_mesh_set_node_order and pfem_mesh_query_int(PFEM_Q_PERM)).
 *   - Input arrays are caller-owned and copied during the call.  Handles are
 *     library-owned and released with the matching *_destroy.  Output
 *     buffers are caller-owned.
 *   - Pointers documented as "device" must point to memory of the context's
 *     device; "host" pointers to ordinary host memory.
 *   - A context binds one device and one HIP stream; all device work of the
 *     handles created from it is ordered on that stream.  Calls on one
 *     context must be serialised by the caller (the server object is the
 *     exception: submit/poll/result/cancel may be called from any thread).
 */
#ifndef PFEM_H
#define PFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pfem_status;
enum {
  PFEM_OK = 0,
  PFEM_NOT_CONVERGED = 1,     /* max iterations reached, or (linear) the true residual
                                 stalled above tol; outputs hold the last iterate */
  PFEM_SKIPPED_FINE = 2,      /* guess already below tol_fine: no iteration run */
  PFEM_E_INVALID_ARG = -1,
  PFEM_E_INVALID_MESH = -2,   /* bad index, degenerate element, orphan node ... */
  PFEM_E_OOM = -3,
  PFEM_E_DEVICE = -4,         /* a HIP runtime call failed */
  PFEM_E_BREAKDOWN = -5,      /* p.Ap <= 0 or NaN in a linear solve */
  PFEM_E_INVERTED = -6,       /* an element has J <= 0 at the evaluated state */
  PFEM_E_LINESEARCH = -7,     /* no admissible Armijo step */
  PFEM_E_CANCELLED = -8,
  PFEM_E_STATE = -9           /* call not valid in the handle's current state */
};

/* Constitutive models.  Linear: sigma = 2 mu eps + lambda tr(eps) I with
 * eps = sym grad u (plane stress replaces lambda by 2 mu lambda/(lambda+2 mu)).
 * Neo-Hookean: Psi = 1/2 lambda (ln J)^2 - mu ln J + 1/2 mu (I1 - dim). */
enum {
  PFEM_LIN_PLANE_STRESS = 0,
  PFEM_LIN_PLANE_STRAIN = 1,
  PFEM_LIN_3D = 2,
  PFEM_NH_PLANE_STRAIN = 3,
  PFEM_NH_3D = 4
};

/* Material parameter kinds for pfem_mesh_set_material. */
enum { PFEM_PARAM_E_NU = 0, PFEM_PARAM_LAME = 1 };

/* Arithmetic of the element kernels: FP64 throughout, or FP32 element math
 * with FP64 reductions, FP64 outer residuals and FP64 log J. */
enum { PFEM_FP64 = 0, PFEM_FP32 = 1 };

/* Scatter strategy of the element kernels (kernel-level calls). */
enum {
  PFEM_SCATTER_OWNER = 0,     /* node blocks own their outputs; LDS accumulation */
  PFEM_SCATTER_COLORED = 1,   /* colour by colour, deterministic */
  PFEM_SCATTER_ATOMIC = 2     /* device-wide atomic adds */
};

/* Vector layout for kernel-level calls. */
enum { PFEM_LAYOUT_USER = 0, PFEM_LAYOUT_INTERNAL = 1 };

/* Masking flags for kernel-level calls (bitwise or). */
enum {
  PFEM_MASK_NONE = 0,
  PFEM_MASK_OUT = 1,          /* zero the output at Dirichlet DOFs */
  PFEM_MASK_IN = 2            /* treat the input direction as zero at Dirichlet DOFs */
};

/* Integer query hooks (bit-exact preprocessing results). */
enum {
  PFEM_Q_PERM = 0,            /* n_nodes: internal id of each caller node */
  PFEM_Q_ELEM_ORDER = 1,      /* n_elems: caller element index at each sorted position */
  PFEM_Q_COLOR = 2,           /* n_elems: colour of each sorted element */
  PFEM_Q_FREE_INDEX = 3,      /* n_nodes*dim: rank among free DOFs (caller numbering) or -1 */
  PFEM_Q_BLOCKS = 4,          /* 3*n_blocks: per node block (first touching elem,
                                 first owned elem, end elem) in sorted order */
  PFEM_Q_AGGREGATE = 5        /* n_nodes: coarse aggregate of each caller node (the
                                 two-level preconditioner's partition) */
};

typedef struct pfem_ctx pfem_ctx;
typedef struct pfem_mesh pfem_mesh;
typedef struct pfem_batch pfem_batch;
typedef struct pfem_server pfem_server;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * run on, or NULL for a library-owned stream (default priority). */
pfem_status pfem_ctx_create(int device, void* hip_stream, pfem_ctx** out);
/* Release the handle (NULL is a no-op).  Meshes and batches made on it
 * keep the device context alive; its stream is synchronised and its
 * resources freed when the last of them is destroyed (a server runs on a
 * stream of its own).  A caller-supplied stream is never destroyed. */
void pfem_ctx_destroy(pfem_ctx* ctx);
/* Message of the last error on this thread ("" if none).  Kept per thread,
 * not per context: calls without a context (host-only meshes) and the
 * server calls, which any thread may make, report through it too. */
const char* pfem_last_error(void);
/* Library version string. */
const char* pfem_version(void);

/* Kernel timing: every launch of a timed kernel family on the context is
 * bracketed by HIP events on the context stream and its elapsed time is
 * accumulated per family.  Families: 0 = K.v / Hessian-vector apply,
 * 1 = internal force, 2 = energy, 3 = Jacobi diagonal, 4 = PCG vector
 * update, 5 = direction update, 6 = fused PCG iteration (matvec and
 * vector updates in one launch; timed per chunk of consecutive launches,
 * chunks that ran past convergence discarded).  `family_mask`: bit f times
 * family f (0 = off).  Reading synchronises the stream. */
pfem_status pfem_ctx_set_timing(pfem_ctx* ctx, int family_mask);
/* Time only every `every`-th launch of each per-launch timed family
 * (default 1), so that the event pairs barely perturb a long sequence. */
pfem_status pfem_ctx_set_timing_sample(pfem_ctx* ctx, int every);
/* Launches timed and their summed duration (ms) for one family since the
 * last reset; launches, total_ms: host, may be NULL.  Synchronises the
 * stream.  PFEM_E_INVALID_ARG for a family outside 0..6. */
pfem_status pfem_ctx_kernel_time(pfem_ctx* ctx, int family, int64_t* launches,
                                 double* total_ms);
/* Launches and algorithmic bytes of one family since the last reset.
 * launches_timed / total_ms: as pfem_ctx_kernel_time.  launches_run: the
 * launches of the family that did work and whose time is in total_ms (a
 * launch of a PCG chunk after every solve in it has converged returns at
 * once and is not counted; a fused chunk, timed as one run, counts only
 * when every one of its launches did work).  alg_bytes: what those
 * launches had to move at least, summed over every solve they advanced and
 * every iteration each one ran
 * (K.v / Hessian-vector apply: 4 (d+1) N_e connectivity + s N_e material +
 * d s N_n coordinates + d s N_n input + d s N_n output, plus d s N_n of
 * state u for Neo-Hookean meshes; fused PCG iteration: the same
 * connectivity, material and coordinates + 11 d s N_n of node records and
 * vectors ({r, w, s, M^-1} read, {r, w, s} written, p and d read and
 * written), plus d s N_n of state u for Neo-Hookean meshes; s = 4 or 8 by
 * precision).  Counted for the apply (0)
 * and fused (6) families of solves while the family is timed; 0 for the
 * others and for kernel-level calls.  So alg_bytes / launches_run is the
 * average per launch and alg_bytes / total_ms the achieved algorithmic
 * bandwidth when every launch is timed (sampling 1). */
typedef struct {
  int64_t launches_timed;
  double total_ms;
  int64_t launches_run;
  double alg_bytes;
} pfem_kernel_stats;
pfem_status pfem_ctx_kernel_stats(pfem_ctx* ctx, int family, pfem_kernel_stats* out);
/* Zero every family's counters (pending timings are collected first). */
pfem_status pfem_ctx_reset_timing(pfem_ctx* ctx);
/* Block until all work queued on the context stream has finished. */
pfem_status pfem_ctx_synchronize(pfem_ctx* ctx);

/* ------------------------------------------------------------------- mesh */

/* Create a mesh (App. B discretisation; Sec. 'Pretraining': the mesh the
 * point cloud comes from).  coords: host, n_nodes*dim float64, node-major.
 * conn: host, n_elems*(dim+1) int32.  Either orientation is accepted.
 * `ctx` may be NULL for a host-only mesh (preprocessing and queries work;
 * device calls return PFEM_E_STATE) -- the server uploads such meshes when
 * it admits them. */
pfem_status pfem_mesh_create(pfem_ctx* ctx, int dim, int64_t n_nodes,
                             const double* coords, int64_t n_elems,
                             const int32_t* conn, pfem_mesh** out);
/* Element families.  PFEM_ELEM_P1: linear triangles (2D) / tetrahedra (3D),
 * one point per element (what pfem_mesh_create builds).  PFEM_ELEM_Q4:
 * bilinear quadrilaterals, 2 x 2 Gauss points; PFEM_ELEM_Q8: 8-node
 * serendipity quadrilaterals, 3 x 3 Gauss points (Sec. 'Nonlinear
 * hyperelasticity': the beam on a Q4 mesh and Cook's membrane on a Q8 mesh;
 * App. B: the isoparametric interpolation X = N_I X_I, u = N_I u_I). */
enum { PFEM_ELEM_P1 = 0, PFEM_ELEM_Q4 = 1, PFEM_ELEM_Q8 = 2 };
/* Create a 2D quadrilateral mesh.  elem: PFEM_ELEM_Q4 or PFEM_ELEM_Q8.
 * coords: host, n_nodes*2 float64.  conn: host, n_elems*4 (Q4) or n_elems*8
 * (Q8) int32: the corners in order around the element (either
 * orientation), then for Q8 the midside nodes of edges (0,1), (1,2), (2,3),
 * (3,0).  Neumann facets of a Q8 mesh are its 3-node edges (pfem_mesh_
 * set_neumann).  Quadrilateral meshes run every element kernel with the
 * owner scatter; the fused PCG, the two-level preconditioner and the
 * coloured / atomic scatters are refused (PFEM_E_INVALID_ARG) -- automatic
 * Krylov selection picks the classic loop.  Errors as pfem_mesh_create;
 * PFEM_E_INVALID_ARG for another elem. */
pfem_status pfem_mesh_create_quad(pfem_ctx* ctx, int elem, int64_t n_nodes,
                                  const double* coords, int64_t n_elems,
                                  const int32_t* conn, pfem_mesh** out);
/* Per-element material (both parameters given per element: a uniform one is
 * an array of n_elems equal values).  model: PFEM_LIN_* / PFEM_NH_*.  param_kind:
 * PFEM_PARAM_E_NU (p0 = Young's modulus, p1 = Poisson ratio; Lame
 * parameters per Sec. 'Nonlinear hyperelasticity') or PFEM_PARAM_LAME
 * (p0 = mu, p1 = lambda).  p0, p1: host, n_elems float64 each.
 * PFEM_E_INVALID_ARG (and no material kept) unless every element has
 * mu > 0 and dim * lambda + 2 mu > 0 (lambda* in plane stress): the
 * stiffness is then SPD.  Non-finite parameters (nu = 0.5, nu = -1) are
 * reported by pfem_mesh_finalize.  PFEM_E_STATE after finalize. */
pfem_status pfem_mesh_set_material(pfem_mesh* m, int model, int param_kind,
                                   const double* p0, const double* p1);
/* Dirichlet set: n triples (node, comp, final value); host arrays.  Values
 * are the final-load values; load steps scale them.  Dirichlet overrides
 * Neumann at shared DOFs. */
pfem_status pfem_mesh_set_dirichlet(pfem_mesh* m, int64_t n, const int32_t* node,
                                    const int8_t* comp, const double* value);
/* Neumann set: n_facets boundary facets (edges in 2D: 2 nodes; triangles in
 * 3D: 3 nodes; on a Q8 mesh 3-node edges: the two ends, then the middle
 * node) each with a constant traction (dim values); host arrays.  f_ext is
 * the consistent load t int N_a dGamma (App. B, f_ext integral): t |facet|
 * / n_f on each node of a linear facet; on a Q8 edge the quadratic shape
 * functions integrated along the edge with 3 Gauss points (t L/6, t L/6,
 * 2 t L/3 on a straight edge with a centred middle node). */
pfem_status pfem_mesh_set_neumann(pfem_mesh* m, int64_t n_facets,
                                  const int32_t* facet_nodes, const double* traction);
/* Periodic springs (App. D: the virtual elements PFEM uses to impose the
 * periodic boundary conditions of a unit cell, a penalty): n_pairs node
 * pairs (host, 2 int32 each, caller ids), each joined by a spring of
 * stiffness `stiffness` whose energy 1/2 k |u_a - u_b|^2 joins the
 * potential.  Every owner-scatter kernel includes them (K.v, force,
 * energy, diagonal); the fused PCG and the coloured / atomic scatters do
 * not and refuse such meshes.  Linear models only (checked at finalize).
 * n_pairs = 0 clears.  Must be called before pfem_mesh_finalize
 * (PFEM_E_STATE after); PFEM_E_INVALID_ARG for a node out of range, a pair
 * of one node, or a stiffness that is not finite and > 0. */
pfem_status pfem_mesh_set_periodic(pfem_mesh* m, int64_t n_pairs, const int32_t* pairs,
                                   double stiffness);
/* Internal node numbering (not in the paper, which names no ordering; it
 * decides how many elements straddle two owner blocks and so how often the
 * element kernels evaluate an element):
 *   PFEM_ORDER_BLOCKS (default): reverse Cuthill-McKee, cut into bands about
 *     as many breadth-first levels thick as a block is wide, each band cut
 *     into compact blocks of block_nodes nodes by recursive coordinate
 *     bisection;
 *   PFEM_ORDER_RCM: reverse Cuthill-McKee alone (blocks are runs of RCM
 *     positions).
 * Must be called before pfem_mesh_finalize (PFEM_E_STATE after); an unknown
 * value is PFEM_E_INVALID_ARG. */
enum { PFEM_ORDER_BLOCKS = 0, PFEM_ORDER_RCM = 1 };
pfem_status pfem_mesh_set_node_order(pfem_mesh* m, int order);
/* Validate and preprocess: node numbering, element sort, colouring,
 * free-DOF map, node blocks; upload to the device when the mesh has a
 * context.  block_nodes: nodes per owner block (0 = automatic). */
pfem_status pfem_mesh_finalize(pfem_mesh* m, int block_nodes);

typedef struct {
  int32_t dim, model;
  int64_t n_nodes, n_elems, n_dof, n_free;
  int32_t n_colors, n_blocks, block_nodes;
  int64_t bandwidth_in, bandwidth_internal;   /* max |i-j| over element node pairs:
                                                caller and internal numbering */
  int64_t owner_elem_visits;                /* sum over blocks of touched range lengths */
  int64_t device_bytes;                     /* mesh arrays resident on the device */
  int64_t solve_bytes_fp32, solve_bytes_fp64;   /* extra device bytes of one solve */
  double f_ext_norm;
  int32_t band_blocks;                      /* owner blocks per RCM band of the block
                                               numbering (0 under PFEM_ORDER_RCM) */
  int32_t elem;                             /* PFEM_ELEM_* */
  int32_t nodes_per_elem;                   /* dim+1 (P1), 4 (Q4), 8 (Q8) */
} pfem_mesh_info;
/* Sizes and preprocessing statistics of a mesh; out: host.  Fields that
 * preprocessing sets (free DOFs, colours, blocks, bandwidths, device
 * bytes) are 0 before pfem_mesh_finalize. */
pfem_status pfem_mesh_get_info(const pfem_mesh* m, pfem_mesh_info* out);
/* Copy a preprocessing array (see PFEM_Q_*) into out (host, the first
 * min(cap, length) entries); *n (host) receives the full length.  out may
 * be NULL to ask for the length only, n may be NULL.  PFEM_E_STATE before
 * pfem_mesh_finalize; PFEM_E_INVALID_ARG for an unknown query or cap < 0. */
pfem_status pfem_mesh_query_int(const pfem_mesh* m, int which, int32_t* out,
                                int64_t cap, int64_t* n);
/* Device bytes a solve of this mesh in precision prec (PFEM_FP64 /
 * PFEM_FP32, automatic Krylov formulation) occupies: the mesh arrays plus
 * one solve's state -- what a server charges against its memory budget
 * when it admits the request and has to upload the mesh (Sec.
 * 'Warm-start': many warm-started solves on one device).  bytes: host.
 * PFEM_E_STATE before pfem_mesh_finalize. */
pfem_status pfem_mesh_footprint(const pfem_mesh* m, int prec, int64_t* bytes);
/* Build the coarse space of the two-level preconditioner on the host (see
 * PFEM_PRECOND_TWO_LEVEL) now rather than at the first solve that asks for
 * it: aggregates, orthonormal rigid modes, P^T K P and its inverse.  Needs
 * no device; thread-safe per mesh; a no-op when built.  n_coarse (host, may
 * be NULL) receives the coarse dimension.  PFEM_E_STATE before
 * pfem_mesh_finalize. */
pfem_status pfem_mesh_prepare_coarse(pfem_mesh* m, int32_t* n_coarse);
/* Upload a finalized host-only mesh (created with ctx NULL) to ctx's
 * device, so kernel-level and batched calls can use it; a no-op for a mesh
 * already resident on ctx, PFEM_E_STATE for one resident on another
 * context.  A server that is handed a resident mesh uses its arrays in
 * place and charges nothing for them. */
pfem_status pfem_mesh_upload(pfem_mesh* m, pfem_ctx* ctx);
/* Free the mesh's device arrays; the mesh stays finalized and host-only
 * (a no-op for a mesh that is not resident).  It must not be in a live
 * batch or a server request that has not been collected. */
pfem_status pfem_mesh_release_device(pfem_mesh* m);
/* Free the mesh and its device arrays (NULL is a no-op).  It must not be in
 * a live batch or a server request that has not been collected. */
void pfem_mesh_destroy(pfem_mesh* m);

/* Convert a vector between the caller's and the internal node order.
 * to_internal = 1: in caller order -> out internal; 0: the reverse.
 * prec selects float64 (PFEM_FP64) or float32 (PFEM_FP32) elements.
 * in, out: device, n_dof entries, must not alias. */
pfem_status pfem_permute(pfem_mesh* m, int prec, int to_internal,
                         const void* in, void* out);

/* ------------------------------------------------------ kernel-level calls
 * All vectors are device pointers of n_dof entries in `prec` (float64 or
 * float32), in the layout given.  Mesh must be finalized with a context.
 * Device pointers only, by design: these calls sit inside device-resident
 * loops (the differentiable energy's forward / backward / double backward,
 * Krylov iterations of a caller, benchmarks), where a host round trip per
 * call would cost more than the kernel; a host caller copies in once or
 * uses pfem_solve, which takes host or device vectors.  The scatter
 * strategy is chosen per call (finalize prepares owner blocks and colours
 * for all of them). */

/* y = K v (linear models) or y = K_T(u) v (Neo-Hookean; u ignored for linear
 * models and may be NULL).  App. B: incremental internal force
 * (K_geo + K_mat) dU.  scatter: PFEM_SCATTER_*; mask: PFEM_MASK_* bits. */
pfem_status pfem_hvp(pfem_mesh* m, int prec, int layout, int scatter, int mask,
                     const void* u, const void* v, void* y);
/* y = K v: pfem_hvp at u = 0. */
pfem_status pfem_apply_K(pfem_mesh* m, int prec, int layout, int scatter,
                         int mask, const void* v, void* y);
/* g = dPi/du = f_int(u) - f_ext (App. B: f_int,iI = int dN_I/dX_J P_iJ dV0). */
pfem_status pfem_force(pfem_mesh* m, int prec, int layout, int mask,
                       const void* u, void* g);
/* Pi(u) = sum_e vol_e Psi_e(u) - f_ext . u, reduced in float64 in a fixed
 * order; energy_dev: device, 1 float64.  Elements with J <= 0 give +inf. */
pfem_status pfem_energy(pfem_mesh* m, int prec, int layout, const void* u,
                        double* energy_dev);
/* pfem_energy without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and result as
 * pfem_energy; its block partial sums, reduced sums and (layout
 * PFEM_LAYOUT_USER) the permuted state live in one library-owned device
 * array of 16 MiB per GPU, created when the library is loaded and held
 * until the process ends (its address on a device is looked up when the
 * first context on that device is created).  Needs 256 + round256(32 *
 * n_blocks) bytes, plus round256(n_dof * 8 or 4) in user layout (about
 * 2M float64 DOFs); a larger mesh gets PFEM_E_INVALID_ARG and nothing runs.
 * Nothing in the array has to start at zero: every call writes what it
 * reads.  All calls on one GPU share the array, so calls that overlap in
 * time on one GPU (several contexts or streams, several host threads) race
 * and must be ordered by the caller.  No hipMalloc, hipFree or other
 * allocating routine is called. */
pfem_status pfem_energy_noalloc(pfem_mesh* m, int prec, int layout, const void* u,
                                double* energy_dev);
/* diag(K_T(u)) (Jacobi preconditioner of the warm-start PCG); Dirichlet DOFs
 * get 1. */
pfem_status pfem_diag(pfem_mesh* m, int prec, int layout, const void* u, void* d);

/* ------------------------------------------------------- batched calls
 * A batch groups finalized meshes (same context) so each element kernel
 * runs once over all of them (one launch, one work table).  Vectors are
 * concatenated in batch order in INTERNAL layout: mesh i occupies
 * [offset_i, offset_i + n_dof_i) with offsets from pfem_batch_offsets. */
/* meshes: host array of n finalized meshes uploaded on ctx's device, all of
 * one dimension (linear and Neo-Hookean may mix; a mesh may appear in
 * several batches).  The batch references the meshes: they must outlive it.
 * PFEM_E_INVALID_ARG for n <= 0, a mesh of another context or mixed
 * dimensions; PFEM_E_STATE for a mesh that is not finalized or has no
 * device context. */
pfem_status pfem_batch_create(pfem_ctx* ctx, int32_t n, pfem_mesh* const* meshes,
                              pfem_batch** out);
/* Free the batch's tables after its queued work (NULL is a no-op); the
 * meshes are not touched. */
void pfem_batch_destroy(pfem_batch* b);
/* offsets: host, n+1 int64 entries (offsets[n] = total DOFs). */
pfem_status pfem_batch_offsets(const pfem_batch* b, int64_t* offsets);
/* Per-mesh total potential Pi_i(u_i) (the pretraining loss of each sample).
 * u: device, concatenated, float64 or float32 per prec; energies_dev:
 * device, n float64.  An element with J <= 0 makes its mesh's energy +inf. */
pfem_status pfem_batch_energy(pfem_batch* b, int prec, const void* u,
                              double* energies_dev);
/* g = dPi/du = f_int(u) - f_ext per mesh (the loss gradient).  u, g: device,
 * concatenated, prec's type; mask as for pfem_force. */
pfem_status pfem_batch_force(pfem_batch* b, int prec, int mask, const void* u,
                             void* g);
/* y = K_T(u) v per mesh (K v for linear meshes).  u, v, y: device,
 * concatenated, prec's type, y must not alias u or v; mask as for
 * pfem_hvp. */
pfem_status pfem_batch_hvp(pfem_batch* b, int prec, int mask, const void* u,
                           const void* v, void* y);

/* --------------------------------------------------------------- solves */
/* PCG formulations (same Krylov iterates in exact arithmetic):
 * CLASSIC  three launches per iteration (apply; update; direction), the
 *          textbook recurrences (Saad, Alg. 9.1);
 * FUSED    one launch per iteration: the Chronopoulos-Gear form, whose two
 *          inner products come from one phase, with the pointwise vector
 *          update evaluated by every workgroup at the nodes it gathers, so
 *          the element pass and all vector updates share a kernel (one
 *          extra matvec per inner solve, w = A u at the start);
 * AUTO     FUSED in FP32 mode on triangle meshes of any size and on
 *          tetrahedral meshes up to 800k elements, CLASSIC otherwise, in
 *          FP64 mode, on quadrilaterals and with periodic springs. */
enum { PFEM_KRYLOV_AUTO = 0, PFEM_KRYLOV_CLASSIC = 1, PFEM_KRYLOV_FUSED = 2 };

/* Preconditioner of the PCG solves (the paper's CG names none; §5.6 notes
 * that a stronger one complements the warm start):
 * JACOBI     M^-1 = D^-1, the diagonal of K (or of K_T(u));
 * TWO_LEVEL  M^-1 = D^-1 + P (P^T K P)^-1 P^T, P the rigid-body modes of
 *            linear elasticity on aggregates of consecutive owner blocks
 *            (PFEM_Q_AGGREGATE), orthonormalised per aggregate over its free
 *            DOFs; P^T K P from the linear moduli (the Neo-Hookean tangent
 *            at rest), built on the host and inverted once per mesh (at
 *            most 1536 coarse DOFs), applied with the classic PCG loop. */
enum { PFEM_PRECOND_JACOBI = 0, PFEM_PRECOND_TWO_LEVEL = 1 };

/* Options of a solve.  pfem_solve and pfem_server_submit return
 * PFEM_E_INVALID_ARG for a tol that is not finite and > 0, an unknown prec,
 * krylov or precond, the fused formulation with the two-level
 * preconditioner, or an inner_rtol outside {0} U (0, 0.5]. */
typedef struct {
  double tol;           /* relative residual target |r_f| / |r_f(lifted)| (App. B) */
  double tol_fine;      /* skip iterating if the guess is already below (Sec. 'Warm-start'); 0 = off */
  int32_t max_iter;     /* cap on K.v products in all Krylov loops of the solve;
                           <= 0: 10 * n_free + 1000 * load steps (1 if linear) */
  int32_t n_load_steps; /* Neo-Hookean: load steps N_f (warm start jumps to N_f); < 1 means 1 */
  int32_t max_newton;   /* per load step; <= 0 means 50 */
  int32_t prec;         /* PFEM_FP64 or PFEM_FP32 (FP32 Krylov, FP64 outer residual) */
  int32_t record_history;
  double inner_rtol;    /* FP32 mode: residual reduction per refinement sweep;
                           0 = automatic (1e-4 for FUSED, 1e-3 for CLASSIC) */
  int32_t krylov;       /* PFEM_KRYLOV_*: PCG formulation of the inner solves */
  int32_t precond;      /* PFEM_PRECOND_*; TWO_LEVEL uses the classic loop (AUTO) and
                           refuses PFEM_KRYLOV_FUSED */
} pfem_solve_opts;

typedef struct {
  pfem_status status;
  int32_t kv_count;          /* K.v / HVP products in Krylov loops */
  int32_t pcg_iters;
  int32_t newton_iters;      /* summed over load steps */
  int32_t load_steps_done;
  int32_t residual_evals;    /* FP64 residual (internal force) evaluations */
  int32_t outer_sweeps;      /* refinement sweeps / PCG restarts */
  int32_t line_search_evals;
  double rel_residual_initial;
  double rel_residual_final;
  int64_t history_len;
  double t_device_ms;        /* wall time of the solve on the context stream */
} pfem_solve_report;

/* Fill opts with defaults (tol 1e-8, FP32 mode, history on). */
void pfem_solve_opts_default(pfem_solve_opts* o);

/* Solve for the displacement field (Sec. 'Warm-start': U^(0) = u0, stop at
 * the relative-residual tolerance).  u0: NULL (zero start; Neo-Hookean runs
 * all load steps) or n_dof float64 (warm start; Neo-Hookean starts at the
 * final load step).  u0/u_out are device pointers if ptr_is_device else
 * host; caller numbering.  Dirichlet DOFs of u_out hold the prescribed
 * values.  history: host, history_cap float64 relative residuals (may be
 * NULL; entry 0 is the initial guess's, then one per Krylov iteration of
 * every inner loop in order, truncated to history_cap).  rep: host (may be
 * NULL).  Returns when the solve has ended (the context stream is
 * synchronised).  A linear solve whose true residual fails to halve over
 * three refinement sweeps in a row (tol below the accuracy the FP64
 * residual evaluation attains on the mesh) ends with PFEM_NOT_CONVERGED and
 * rel_residual_final at that level instead of running to max_iter.
 * Status: PFEM_OK, PFEM_SKIPPED_FINE, PFEM_NOT_CONVERGED,
 * or a solver failure (PFEM_E_BREAKDOWN, PFEM_E_INVERTED,
 * PFEM_E_LINESEARCH) -- all of these still fill u_out (the last iterate),
 * history and rep; argument, state and device errors leave the outputs
 * unspecified. */
pfem_status pfem_solve(pfem_mesh* m, const double* u0, const pfem_solve_opts* o,
                       double* u_out, int ptr_is_device, double* history,
                       int64_t history_cap, pfem_solve_report* rep);

/* Homogenised elasticity tensor of a periodic cell (App. D; Sec. 'Three-
 * dimensional solid mechanics homogenization').  The mesh: 3D, linear
 * (PFEM_LIN_3D), periodic springs set, and one node held at zero by the
 * Dirichlet set (its 3 components), which removes the rigid translations.
 * For each of the six unit macroscopic strains eps0^(IJ), (IJ) = 11, 22,
 * 33, 12, 13, 23 (ones at (p, q) and (q, p) for the shears), the
 * fluctuation X^v solves (K + P) X^v = F^(IJ), F^(IJ) the element loads of
 * the uniform stress E : eps0^(IJ), to o->tol (relative residual; o->prec
 * as for pfem_solve; the classic PCG); the six solves run together, every
 * element launch covering all of them.  Then
 * E^H_(IJ)(KL) = 1/|Omega| sum_e vol_e (eps0 - eps^v)^(IJ) : E_e :
 * (eps0 - eps^v)^(KL), |Omega| the volume of the mesh's bounding box.
 * u0: NULL (zero starts) or 6 n_dof float64 warm starts of the six
 * fluctuations (case k at [k n_dof, (k+1) n_dof)); x_out: 6 n_dof float64,
 * the fluctuations in the same layout; both device pointers if
 * ptr_is_device, else host; caller numbering.  eh: host, 36 float64, E^H
 * row-major in the case order above.  reps: host array of 6 reports or
 * NULL.  Returns the most severe of the six statuses (outputs filled as
 * for pfem_solve); argument and state errors as for pfem_solve. */
pfem_status pfem_homogenize(pfem_mesh* m, const double* u0, const pfem_solve_opts* o,
                            double* x_out, int ptr_is_device, double* eh,
                            pfem_solve_report* reps);

/* --------------------------------------------------------------- serving
 * Many warm-started solves on one device (Sec. 'Warm-start': the network is
 * pretrained once and its predictions start the solves of the deployment;
 * each solve is the same as pfem_solve's).  Requests of uneven size share
 * the device under a memory budget and are advanced together. */
/* Create a server on ctx's device: at most max_slots live solves whose
 * device footprint sums to at most hbm_budget_bytes.  Each live request is
 * charged its solve state; a mesh the server uploads is charged once, while
 * the server holds it for one or more live requests (a mesh resident on a
 * caller's context is used in place and not charged).  A worker thread
 * admits queued requests in arrival order as slots and memory free up (the
 * head of the queue waits), keeps each live solve's state on the device and
 * advances all live solves together, one batched launch per kernel family
 * per step, so requests that arrive while others run overlap with them. */
pfem_status pfem_server_create(pfem_ctx* ctx, int64_t hbm_budget_bytes,
                               int32_t max_slots, pfem_server** out);
/* Queue a solve.  `m` must be finalized (a host-only mesh is fine); the
 * server keeps a reference, so the caller must not destroy the mesh, nor
 * upload or release its device arrays, before the result is collected.
 * u0: host n_dof float64 or NULL (copied).  req_id must be unique among
 * requests not yet collected.  Returns PFEM_E_OOM if the solve state alone
 * exceeds the budget; a request that needs the mesh uploaded and can never
 * fit with it ends with PFEM_E_OOM when it reaches the head of the queue. */
pfem_status pfem_server_submit(pfem_server* s, pfem_mesh* m, const double* u0,
                               const pfem_solve_opts* o, int64_t req_id);
/* Completed request ids not yet reported (non-blocking). */
pfem_status pfem_server_poll(pfem_server* s, int64_t* done_ids, int64_t cap,
                             int64_t* n_done);
/* Collect a completed request: u_out host n_dof float64 (may be NULL); times
 * in seconds since the server started (submit, admission, completion).
 * Releases the request.  PFEM_E_STATE while the request is queued or live
 * (nothing is released; call again later), PFEM_E_INVALID_ARG for an
 * unknown or already collected id; otherwise the request's own status if
 * it is an error (a device failure inside the worker ends every live
 * request with that error), else PFEM_OK. */
pfem_status pfem_server_result(pfem_server* s, int64_t req_id, double* u_out,
                               pfem_solve_report* rep, double* t_submit,
                               double* t_admit, double* t_done);
/* Cancel a queued or live request (its result reports PFEM_E_CANCELLED). */
pfem_status pfem_server_cancel(pfem_server* s, int64_t req_id);
typedef struct {
  int64_t submitted, completed, live, queued, peak_live;
  int64_t bytes_in_use, peak_bytes, budget;
  int64_t steps, launches;
  double admit_s, tick_s, complete_s;   /* worker host seconds: admitting requests
                                           (uploads, solver state), engine steps,
                                           completing them (download, frees) */
} pfem_server_stats;
/* Counters of the server (a consistent snapshot; out: host): requests
 * submitted / completed / live / queued, the most live at once, device
 * bytes in use, their peak and the budget, worker steps and launches, and
 * where the worker's time went. */
pfem_status pfem_server_get_stats(pfem_server* s, pfem_server_stats* out);
/* Kernel timing of the server's own stream: the families of
 * pfem_ctx_set_timing (bitmask; 0 = off), every launch timed.  Counters are
 * zeroed and the mask takes effect at the worker's next step. */
pfem_status pfem_server_set_timing(pfem_server* s, int family_mask);
/* Counters of one family since the last pfem_server_set_timing, as
 * pfem_ctx_kernel_stats, up to the worker's last completed step. */
pfem_status pfem_server_kernel_stats(pfem_server* s, int family, pfem_kernel_stats* out);
/* Stop the worker (live requests are cancelled) and free everything. */
void pfem_server_destroy(pfem_server* s);

#ifdef __cplusplus
}
#endif
#endif /* PFEM_H */
