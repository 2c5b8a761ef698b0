// C ABI: argument checking, error translation and call orchestration.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "mesh.h"
#include "coarse.h"
#include "solver.h"

using namespace pfem;

struct pfem_batch {
  Ctx* ctx = nullptr;
  std::vector<pfem_mesh*> meshes;
  std::vector<int64_t> offsets;       // DOF offsets (n + 1)
  int dim = 0;
  int kind = 0;                       // element kernel family (pfem::elem_kind)
  int bn_max = 0;
  int n_work = 0;
  int2* work = nullptr;               // persistent device work table (all meshes)
  int n_work_kind[2] = {0, 0};        // linear / Neo-Hookean sub-tables
  int2* work_kind[2] = {nullptr, nullptr};
  double* part = nullptr;             // per mesh: n_blocks * kRedSlots
  double* outs = nullptr;             // per mesh: kRedSlots
  std::vector<int64_t> part_off;
  // persistent task tables with relocatable operands (u, v, y = DOF offset
  // of each mesh), with and without partial sums
  pfem::Task* tasks_red = nullptr;
  pfem::Task* tasks_plain = nullptr;
};

#define PFEM_TRY_BEGIN try {
#define PFEM_TRY_END                                   \
  }                                                    \
  catch (const pfem::Error& e) {                       \
    pfem::set_error(e.msg);                            \
    return e.code;                                     \
  }                                                    \
  catch (const std::bad_alloc&) {                      \
    pfem::set_error("host out of memory");             \
    return PFEM_E_OOM;                                 \
  }                                                    \
  catch (const std::exception& e) {                    \
    pfem::set_error(e.what());                         \
    return PFEM_E_INVALID_ARG;                         \
  }                                                    \
  catch (...) {                                        \
    pfem::set_error("unknown error");                  \
    return PFEM_E_INVALID_ARG;                         \
  }                                                    \
  pfem::set_error("");                                 \
  return PFEM_OK;

extern "C" {

const char* pfem_last_error(void) { return pfem::last_error_cstr(); }
const char* pfem_version(void) { return "pfem-mi355x 0.1 (gfx950)"; }

pfem_status pfem_ctx_create(int device, void* hip_stream, pfem_ctx** out) {
  PFEM_TRY_BEGIN
  require(out != nullptr, PFEM_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  PFEM_HIP(hipGetDeviceCount(&n));
  require(device >= 0 && device < n, PFEM_E_INVALID_ARG, "device index out of range");
  PFEM_HIP(hipSetDevice(device));
  noalloc_init(device);   // this device's address of the allocation-free scratch
  Ctx* c = new Ctx();
  c->device = device;
  try {
    if (hip_stream != nullptr) {
      c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      PFEM_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    c->ring.init(16u << 20, c->stream);
  } catch (...) {
    ctx_unref(c);
    throw;
  }
  pfem_ctx* h = new pfem_ctx();
  h->c = c;
  *out = h;
  PFEM_TRY_END
}

void pfem_ctx_destroy(pfem_ctx* ctx) {
  if (ctx == nullptr) return;
  ctx_unref(ctx->c);   // freed once the last mesh / batch on it is gone
  delete ctx;
}

pfem_status pfem_ctx_set_timing(pfem_ctx* ctx, int family_mask) {
  PFEM_TRY_BEGIN
  require(ctx != nullptr, PFEM_E_INVALID_ARG, "ctx is NULL");
  ctx->c->drain_timing();
  ctx->c->timing = family_mask;
  PFEM_TRY_END
}

pfem_status pfem_ctx_set_timing_sample(pfem_ctx* ctx, int every) {
  PFEM_TRY_BEGIN
  require(ctx != nullptr, PFEM_E_INVALID_ARG, "ctx is NULL");
  require(every >= 1, PFEM_E_INVALID_ARG, "sampling interval must be >= 1");
  ctx->c->drain_timing();
  ctx->c->sample_every = every;
  for (int i = 0; i < FAM_COUNT; ++i) ctx->c->fam_seen[i] = 0;
  PFEM_TRY_END
}

pfem_status pfem_ctx_kernel_time(pfem_ctx* ctx, int family, int64_t* launches,
                                 double* total_ms) {
  PFEM_TRY_BEGIN
  require(ctx != nullptr, PFEM_E_INVALID_ARG, "ctx is NULL");
  require(family >= 0 && family < FAM_COUNT, PFEM_E_INVALID_ARG, "bad kernel family");
  ctx->c->drain_timing();
  if (launches) *launches = ctx->c->fam_launches[family];
  if (total_ms) *total_ms = ctx->c->fam_ms[family];
  PFEM_TRY_END
}

pfem_status pfem_ctx_kernel_stats(pfem_ctx* ctx, int family, pfem_kernel_stats* out) {
  PFEM_TRY_BEGIN
  require(ctx != nullptr && out != nullptr, PFEM_E_INVALID_ARG, "NULL argument");
  require(family >= 0 && family < FAM_COUNT, PFEM_E_INVALID_ARG, "bad kernel family");
  ctx->c->drain_timing();
  out->launches_timed = ctx->c->fam_launches[family];
  out->total_ms = ctx->c->fam_ms[family];
  out->launches_run = ctx->c->fam_run[family];
  out->alg_bytes = ctx->c->fam_alg_bytes[family];
  PFEM_TRY_END
}

pfem_status pfem_ctx_reset_timing(pfem_ctx* ctx) {
  PFEM_TRY_BEGIN
  require(ctx != nullptr, PFEM_E_INVALID_ARG, "ctx is NULL");
  ctx->c->drain_timing();
  for (int i = 0; i < FAM_COUNT; ++i) {
    ctx->c->fam_launches[i] = 0;
    ctx->c->fam_ms[i] = 0.0;
    ctx->c->fam_run[i] = 0;
    ctx->c->fam_alg_bytes[i] = 0.0;
  }
  PFEM_TRY_END
}

pfem_status pfem_ctx_synchronize(pfem_ctx* ctx) {
  PFEM_TRY_BEGIN
  require(ctx != nullptr, PFEM_E_INVALID_ARG, "ctx is NULL");
  PFEM_HIP(hipStreamSynchronize(ctx->c->stream));
  PFEM_TRY_END
}

// ------------------------------------------------------------------- mesh
pfem_status pfem_mesh_create(pfem_ctx* ctx, int dim, int64_t n_nodes, const double* coords,
                             int64_t n_elems, const int32_t* conn, pfem_mesh** out) {
  PFEM_TRY_BEGIN
  require(out != nullptr, PFEM_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  require(dim == 2 || dim == 3, PFEM_E_INVALID_ARG, "dim must be 2 or 3");
  require(n_nodes > 0 && n_elems > 0, PFEM_E_INVALID_MESH, "empty mesh");
  require(n_nodes < INT32_MAX / 3 && n_elems < INT32_MAX / 4, PFEM_E_INVALID_ARG,
          "mesh too large for int32 indexing");
  require(coords != nullptr && conn != nullptr, PFEM_E_INVALID_ARG, "NULL array");
  pfem_mesh* m = new pfem_mesh();
  m->ctx = ctx != nullptr ? ctx->c : nullptr;
  m->dim = dim;
  m->n_nodes = n_nodes;
  m->n_elems = n_elems;
  m->coords.assign(coords, coords + n_nodes * dim);
  m->nv = dim + 1;
  m->conn.assign(conn, conn + n_elems * m->nv);
  *out = m;
  PFEM_TRY_END
}

pfem_status pfem_mesh_create_quad(pfem_ctx* ctx, int elem, int64_t n_nodes, const double* coords,
                                  int64_t n_elems, const int32_t* conn, pfem_mesh** out) {
  PFEM_TRY_BEGIN
  require(out != nullptr, PFEM_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  require(elem == PFEM_ELEM_Q4 || elem == PFEM_ELEM_Q8, PFEM_E_INVALID_ARG,
          "elem must be PFEM_ELEM_Q4 or PFEM_ELEM_Q8");
  require(n_nodes > 0 && n_elems > 0, PFEM_E_INVALID_MESH, "empty mesh");
  require(n_nodes < INT32_MAX / 3 && n_elems < INT32_MAX / 8, PFEM_E_INVALID_ARG,
          "mesh too large for int32 indexing");
  require(coords != nullptr && conn != nullptr, PFEM_E_INVALID_ARG, "NULL array");
  pfem_mesh* m = new pfem_mesh();
  m->ctx = ctx != nullptr ? ctx->c : nullptr;
  m->dim = 2;
  m->elem = elem;
  m->nv = elem == PFEM_ELEM_Q4 ? 4 : 8;
  m->n_nodes = n_nodes;
  m->n_elems = n_elems;
  m->coords.assign(coords, coords + n_nodes * 2);
  m->conn.assign(conn, conn + n_elems * m->nv);
  *out = m;
  PFEM_TRY_END
}

pfem_status pfem_mesh_set_material(pfem_mesh* m, int model, int param_kind, const double* p0,
                                   const double* p1) {
  PFEM_TRY_BEGIN
  require(m != nullptr && p0 != nullptr && p1 != nullptr, PFEM_E_INVALID_ARG, "NULL argument");
  require(!m->finalized, PFEM_E_STATE, "mesh already finalized");
  require(model >= PFEM_LIN_PLANE_STRESS && model <= PFEM_NH_3D, PFEM_E_INVALID_ARG, "bad model");
  require(param_kind == PFEM_PARAM_E_NU || param_kind == PFEM_PARAM_LAME, PFEM_E_INVALID_ARG,
          "bad param_kind");
  const bool three = model == PFEM_LIN_3D || model == PFEM_NH_3D;
  require(three == (m->dim == 3), PFEM_E_INVALID_ARG, "model does not match mesh dimension");
  std::vector<double> mu(m->n_elems), lam(m->n_elems);
  for (int64_t e = 0; e < m->n_elems; ++e) {
    lame_from_params(model, param_kind, p0[e], p1[e], &mu[e], &lam[e]);
    // the isotropic law (and the Neo-Hookean one at J = 1) is positive
    // definite iff mu > 0 and the bulk modulus lambda + 2 mu / dim is
    // positive (lambda* in plane stress); otherwise K is not SPD and the
    // solves break down.  Non-finite values are caught at finalize.
    if (std::isfinite(mu[e]) && std::isfinite(lam[e]) &&
        !(mu[e] > 0.0 && m->dim * lam[e] + 2.0 * mu[e] > 0.0))
      throw Error{PFEM_E_INVALID_ARG, "element " + std::to_string(e) +
                                          ": material not positive definite (needs mu > 0 "
                                          "and dim * lambda + 2 mu > 0)"};
  }
  m->model = model;
  m->nonlinear = model == PFEM_NH_PLANE_STRAIN || model == PFEM_NH_3D;
  m->mu.swap(mu);
  m->lam.swap(lam);
  PFEM_TRY_END
}

pfem_status pfem_mesh_set_dirichlet(pfem_mesh* m, int64_t n, const int32_t* node,
                                    const int8_t* comp, const double* value) {
  PFEM_TRY_BEGIN
  require(m != nullptr, PFEM_E_INVALID_ARG, "mesh is NULL");
  require(!m->finalized, PFEM_E_STATE, "mesh already finalized");
  require(n >= 0 && (n == 0 || (node && comp && value)), PFEM_E_INVALID_ARG, "bad Dirichlet arrays");
  std::vector<double> seen(m->n_nodes * m->dim, std::nan(""));
  m->dnode.clear();
  m->dcomp.clear();
  m->dval.clear();
  for (int64_t i = 0; i < n; ++i) {
    require(node[i] >= 0 && node[i] < m->n_nodes && comp[i] >= 0 && comp[i] < m->dim,
            PFEM_E_INVALID_ARG, "Dirichlet entry out of range");
    require(std::isfinite(value[i]), PFEM_E_INVALID_ARG, "non-finite Dirichlet value");
    const int64_t g = (int64_t)node[i] * m->dim + comp[i];
    if (!std::isnan(seen[g])) {
      require(seen[g] == value[i], PFEM_E_INVALID_ARG, "conflicting Dirichlet values");
      continue;
    }
    seen[g] = value[i];
    m->dnode.push_back(node[i]);
    m->dcomp.push_back(comp[i]);
    m->dval.push_back(value[i]);
  }
  PFEM_TRY_END
}

pfem_status pfem_mesh_set_neumann(pfem_mesh* m, int64_t n_facets, const int32_t* facet_nodes,
                                  const double* traction) {
  PFEM_TRY_BEGIN
  require(m != nullptr, PFEM_E_INVALID_ARG, "mesh is NULL");
  require(!m->finalized, PFEM_E_STATE, "mesh already finalized");
  require(n_facets >= 0 && (n_facets == 0 || (facet_nodes && traction)), PFEM_E_INVALID_ARG,
          "bad Neumann arrays");
  const int nfn = m->facet_nodes();
  for (int64_t i = 0; i < n_facets * nfn; ++i)
    require(facet_nodes[i] >= 0 && facet_nodes[i] < m->n_nodes, PFEM_E_INVALID_ARG,
            "Neumann facet node out of range");
  for (int64_t i = 0; i < n_facets * m->dim; ++i)
    require(std::isfinite(traction[i]), PFEM_E_INVALID_ARG, "non-finite traction");
  m->n_facets = n_facets;
  m->facets.assign(facet_nodes, facet_nodes + n_facets * nfn);
  m->traction.assign(traction, traction + n_facets * m->dim);
  PFEM_TRY_END
}

pfem_status pfem_mesh_set_periodic(pfem_mesh* m, int64_t n_pairs, const int32_t* pairs,
                                   double stiffness) {
  PFEM_TRY_BEGIN
  require(m != nullptr, PFEM_E_INVALID_ARG, "mesh is NULL");
  require(!m->finalized, PFEM_E_STATE, "mesh already finalized");
  require(n_pairs >= 0 && (n_pairs == 0 || pairs != nullptr), PFEM_E_INVALID_ARG,
          "bad pair array");
  require(n_pairs == 0 || (std::isfinite(stiffness) && stiffness > 0), PFEM_E_INVALID_ARG,
          "spring stiffness must be finite and > 0");
  for (int64_t q = 0; q < n_pairs; ++q) {
    const int32_t a = pairs[2 * q], b = pairs[2 * q + 1];
    require(a >= 0 && a < m->n_nodes && b >= 0 && b < m->n_nodes, PFEM_E_INVALID_ARG,
            "periodic pair node out of range");
    require(a != b, PFEM_E_INVALID_ARG, "periodic pair joins a node to itself");
  }
  m->pairs.assign(pairs, pairs + 2 * n_pairs);
  m->pair_k = n_pairs > 0 ? stiffness : 0.0;
  PFEM_TRY_END
}

pfem_status pfem_mesh_set_node_order(pfem_mesh* m, int order) {
  PFEM_TRY_BEGIN
  require(m != nullptr, PFEM_E_INVALID_ARG, "mesh is NULL");
  require(!m->finalized, PFEM_E_STATE, "mesh already finalized");
  require(order == PFEM_ORDER_BLOCKS || order == PFEM_ORDER_RCM, PFEM_E_INVALID_ARG,
          "unknown node order");
  m->node_order = order;
  PFEM_TRY_END
}

pfem_status pfem_mesh_finalize(pfem_mesh* m, int block_nodes) {
  PFEM_TRY_BEGIN
  require(m != nullptr, PFEM_E_INVALID_ARG, "mesh is NULL");
  require(!m->finalized, PFEM_E_STATE, "mesh already finalized");
  require(block_nodes >= 0, PFEM_E_INVALID_ARG, "block_nodes < 0");
  require(m->pairs.empty() || (m->model >= 0 && !m->nonlinear), PFEM_E_INVALID_ARG,
          "periodic springs need a linear model");
  mesh_finalize_host(m, block_nodes);
  if (m->ctx != nullptr) mesh_upload(m, m->ctx);
  PFEM_TRY_END
}

pfem_status pfem_mesh_get_info(const pfem_mesh* m, pfem_mesh_info* o) {
  PFEM_TRY_BEGIN
  require(m != nullptr && o != nullptr, PFEM_E_INVALID_ARG, "NULL argument");
  *o = pfem_mesh_info{};
  o->dim = m->dim;
  o->model = m->model;
  o->n_nodes = m->n_nodes;
  o->n_elems = m->n_elems;
  o->n_dof = m->n_dof();
  o->n_free = m->n_free;
  o->n_colors = m->n_colors;
  o->n_blocks = m->n_blocks;
  o->block_nodes = m->bn;
  o->bandwidth_in = m->bw_in;
  o->bandwidth_internal = m->bw_int;
  o->owner_elem_visits = m->owner_visits;
  o->device_bytes = m->finalized ? mesh_device_bytes(m) : 0;
  pfem_solve_opts d32;
  pfem_solve_opts_default(&d32);   // FP32 mode, AUTO formulation
  o->solve_bytes_fp32 = m->finalized ? solve_bytes(m, PFEM_FP32, krylov_fused(d32, m), false) : 0;
  o->solve_bytes_fp64 = m->finalized ? solve_bytes(m, PFEM_FP64, false, false) : 0;
  o->f_ext_norm = m->fext_norm;
  o->band_blocks = m->band_blocks;
  o->elem = m->elem;
  o->nodes_per_elem = m->nv;
  PFEM_TRY_END
}

pfem_status pfem_mesh_query_int(const pfem_mesh* m, int which, int32_t* out, int64_t cap,
                                int64_t* n) {
  PFEM_TRY_BEGIN
  require(m != nullptr, PFEM_E_INVALID_ARG, "mesh is NULL");
  require(m->finalized, PFEM_E_STATE, "mesh not finalized");
  std::vector<int32_t> tmp;
  const std::vector<int32_t>* src = nullptr;
  switch (which) {
    case PFEM_Q_PERM: src = &m->perm; break;
    case PFEM_Q_ELEM_ORDER: src = &m->elem_order; break;
    case PFEM_Q_COLOR: src = &m->color; break;
    case PFEM_Q_FREE_INDEX: src = &m->free_index; break;
    case PFEM_Q_BLOCKS:
      for (const int4& b : m->blocks) {
        const int first = b.w > b.z ? std::min(b.x, m->halo[b.z]) : b.x;
        tmp.push_back(first);
        tmp.push_back(b.x);
        tmp.push_back(b.y);
      }
      src = &tmp;
      break;
    case PFEM_Q_AGGREGATE: {
      const int G = coarse_group(m);
      tmp.resize(m->n_nodes);
      for (int64_t n = 0; n < m->n_nodes; ++n) tmp[n] = (m->perm[n] / m->bn) / G;
      src = &tmp;
      break;
    }
    default: throw Error{PFEM_E_INVALID_ARG, "bad query"};
  }
  if (n) *n = (int64_t)src->size();
  if (out != nullptr) {
    require(cap >= 0, PFEM_E_INVALID_ARG, "cap < 0");
    std::copy(src->begin(), src->begin() + std::min<int64_t>(cap, src->size()), out);
  }
  PFEM_TRY_END
}

pfem_status pfem_mesh_footprint(const pfem_mesh* m, int prec, int64_t* bytes) {
  PFEM_TRY_BEGIN
  require(m != nullptr && bytes != nullptr, PFEM_E_INVALID_ARG, "NULL argument");
  require(prec == PFEM_FP64 || prec == PFEM_FP32, PFEM_E_INVALID_ARG, "bad precision");
  require(m->finalized, PFEM_E_STATE, "mesh not finalized");
  pfem_solve_opts o;
  pfem_solve_opts_default(&o);   // AUTO formulation
  o.prec = prec;
  *bytes = mesh_device_bytes(m) + solve_bytes(m, prec, krylov_fused(o, m), false);
  PFEM_TRY_END
}

pfem_status pfem_mesh_prepare_coarse(pfem_mesh* m, int32_t* n_coarse) {
  PFEM_TRY_BEGIN
  require(m != nullptr, PFEM_E_INVALID_ARG, "mesh is NULL");
  require(m->finalized, PFEM_E_STATE, "mesh not finalized");
  require(m->elem == PFEM_ELEM_P1, PFEM_E_INVALID_ARG,
          "the two-level preconditioner is built for P1 meshes");
  coarse_build(m);
  if (n_coarse) *n_coarse = m->coarse->n_c;
  PFEM_TRY_END
}

pfem_status pfem_mesh_upload(pfem_mesh* m, pfem_ctx* ctx) {
  PFEM_TRY_BEGIN
  require(m != nullptr && ctx != nullptr, PFEM_E_INVALID_ARG, "NULL argument");
  require(m->finalized, PFEM_E_STATE, "mesh not finalized");
  if (m->uploaded) {
    require(m->ctx == ctx->c, PFEM_E_STATE, "mesh is resident on another context");
  } else {
    mesh_upload(m, ctx->c);
  }
  PFEM_TRY_END
}

pfem_status pfem_mesh_release_device(pfem_mesh* m) {
  PFEM_TRY_BEGIN
  require(m != nullptr, PFEM_E_INVALID_ARG, "mesh is NULL");
  if (m->uploaded) {
    PFEM_HIP(hipSetDevice(m->ctx->device));
    mesh_release_device(m);
  }
  PFEM_TRY_END
}

void pfem_mesh_destroy(pfem_mesh* m) {
  if (m == nullptr) return;
  try {
    if (m->uploaded) {
      (void)hipSetDevice(m->ctx->device);
      mesh_release_device(m);
    }
  } catch (...) {
  }
  delete m;
}

// ----------------------------------------------------- kernel-level calls
static void need_device(pfem_mesh* m) {
  require(m != nullptr, PFEM_E_INVALID_ARG, "mesh is NULL");
  require(m->finalized, PFEM_E_STATE, "mesh not finalized");
  require(m->uploaded && m->ctx != nullptr, PFEM_E_STATE, "mesh has no device context");
  PFEM_HIP(hipSetDevice(m->ctx->device));
}

static void check_prec(int prec) {
  require(prec == PFEM_FP64 || prec == PFEM_FP32, PFEM_E_INVALID_ARG, "bad precision");
}

pfem_status pfem_permute(pfem_mesh* m, int prec, int to_internal, const void* in, void* out) {
  PFEM_TRY_BEGIN
  need_device(m);
  check_prec(prec);
  require(in != nullptr && out != nullptr && in != out, PFEM_E_INVALID_ARG, "bad vectors");
  launch_permute(m->ctx, prec, m->dim, m->dev.perm, m->n_nodes, to_internal != 0, in, out);
  PFEM_TRY_END
}

static void elem_call(pfem_mesh* m, int prec, int layout, int scatter, int mask, int op,
                      const void* u, const void* v, void* y, double inv_diag) {
  need_device(m);
  check_prec(prec);
  require(layout == PFEM_LAYOUT_USER || layout == PFEM_LAYOUT_INTERNAL, PFEM_E_INVALID_ARG,
          "bad layout");
  require(scatter >= PFEM_SCATTER_OWNER && scatter <= PFEM_SCATTER_ATOMIC, PFEM_E_INVALID_ARG,
          "bad scatter mode");
  require(scatter == PFEM_SCATTER_OWNER || m->pairs.empty(), PFEM_E_INVALID_ARG,
          "periodic springs are applied by the owner scatter only");
  require(scatter == PFEM_SCATTER_OWNER || m->elem == PFEM_ELEM_P1, PFEM_E_INVALID_ARG,
          "quadrilateral meshes run the owner scatter only");
  require(y != nullptr, PFEM_E_INVALID_ARG, "output is NULL");
  Ctx* ctx = m->ctx;
  m->scratch.ensure(m->n_dof(), m->n_blocks);
  const bool need_u = (op != OP_APPLY && !(op == OP_DIAG && !m->nonlinear)) ||
                      (op == OP_APPLY && m->nonlinear);
  if (need_u) require(u != nullptr, PFEM_E_INVALID_ARG, "state u is NULL");
  if (op == OP_APPLY) require(v != nullptr, PFEM_E_INVALID_ARG, "direction is NULL");
  const void* ui = u;
  const void* vi = v;
  void* yi = y;
  if (layout == PFEM_LAYOUT_USER) {
    if (need_u) {
      launch_permute(ctx, prec, m->dim, m->dev.perm, m->n_nodes, true, u, m->scratch.in64);
      ui = m->scratch.in64;
    }
    if (v != nullptr) {
      launch_permute(ctx, prec, m->dim, m->dev.perm, m->n_nodes, true, v, m->scratch.v64);
      vi = m->scratch.v64;
    }
    yi = m->scratch.out64;
  }
  Task t{};
  t.m = m->md;
  t.u = ui;
  t.v = vi;
  t.y = yi;
  t.mask = mask;
  t.active = 1;
  t.s = inv_diag;
  t.fscale = 1.0;
  if (scatter == PFEM_SCATTER_OWNER) {
    const Task* td = static_cast<const Task*>(ctx->ring.put(&t, sizeof(Task)));
    launch_elem(ctx, m->kind(), prec, op, m->nonlinear, PFEM_SCATTER_OWNER, td, m->dev.work,
                m->n_blocks, m->bn, nullptr, nullptr);
  } else {
    launch_elem(ctx, m->dim, prec, op, m->nonlinear, scatter, nullptr, nullptr, 0, m->bn, &t,
                &m->color_ptr);
  }
  if (layout == PFEM_LAYOUT_USER)
    launch_permute(ctx, prec, m->dim, m->dev.perm, m->n_nodes, false, yi, y);
}

pfem_status pfem_hvp(pfem_mesh* m, int prec, int layout, int scatter, int mask, const void* u,
                     const void* v, void* y) {
  PFEM_TRY_BEGIN
  elem_call(m, prec, layout, scatter, mask, OP_APPLY, u, v, y, 0.0);
  PFEM_TRY_END
}

pfem_status pfem_apply_K(pfem_mesh* m, int prec, int layout, int scatter, int mask,
                         const void* v, void* y) {
  PFEM_TRY_BEGIN
  need_device(m);
  const void* u = nullptr;
  if (m->nonlinear) {   // K = K_T(0)
    m->scratch.ensure(m->n_dof(), m->n_blocks);
    u = m->scratch.zero64;
  }
  elem_call(m, prec, layout, scatter, mask, OP_APPLY, u, v, y, 0.0);
  PFEM_TRY_END
}

pfem_status pfem_force(pfem_mesh* m, int prec, int layout, int mask, const void* u, void* g) {
  PFEM_TRY_BEGIN
  elem_call(m, prec, layout, PFEM_SCATTER_OWNER, mask, OP_FORCE, u, nullptr, g, 0.0);
  PFEM_TRY_END
}

pfem_status pfem_diag(pfem_mesh* m, int prec, int layout, const void* u, void* d) {
  PFEM_TRY_BEGIN
  elem_call(m, prec, layout, PFEM_SCATTER_OWNER, PFEM_MASK_NONE, OP_DIAG, u, nullptr, d, 0.0);
  PFEM_TRY_END
}

pfem_status pfem_energy(pfem_mesh* m, int prec, int layout, const void* u, double* energy_dev) {
  PFEM_TRY_BEGIN
  need_device(m);
  check_prec(prec);
  require(u != nullptr && energy_dev != nullptr, PFEM_E_INVALID_ARG, "NULL argument");
  Ctx* ctx = m->ctx;
  m->scratch.ensure(m->n_dof(), m->n_blocks);
  const void* ui = u;
  if (layout == PFEM_LAYOUT_USER) {
    launch_permute(ctx, prec, m->dim, m->dev.perm, m->n_nodes, true, u, m->scratch.in64);
    ui = m->scratch.in64;
  }
  Task t{};
  t.m = m->md;
  t.u = ui;
  t.active = 1;
  t.fscale = 1.0;
  t.red.part = m->scratch.part;
  t.red.out = m->scratch.out;
  const Task* td = static_cast<const Task*>(ctx->ring.put(&t, sizeof(Task)));
  launch_energy(ctx, m->kind(), prec, false, td, m->dev.work, m->n_blocks);
  launch_reduce_store(ctx, td, 1);
  launch_energy_out(ctx, m->scratch.out, energy_dev, 1, kRedSlots);
  PFEM_TRY_END
}

// -------------------------------------------------------------- batches
pfem_status pfem_batch_create(pfem_ctx* ctx, int32_t n, pfem_mesh* const* meshes,
                              pfem_batch** out) {
  PFEM_TRY_BEGIN
  require(ctx != nullptr && out != nullptr && meshes != nullptr && n > 0, PFEM_E_INVALID_ARG,
          "bad batch arguments");
  *out = nullptr;
  pfem_batch* b = new pfem_batch();
  b->ctx = ctx->c;
  try {
    PFEM_HIP(hipSetDevice(ctx->c->device));
    b->offsets.push_back(0);
    int total = 0;
    int64_t poff = 0;
    for (int i = 0; i < n; ++i) {
      pfem_mesh* m = meshes[i];
      need_device(m);
      require(m->ctx == ctx->c, PFEM_E_INVALID_ARG, "mesh belongs to another context");
      if (i == 0) {
        b->dim = m->dim;
        b->kind = m->kind();
      }
      require(m->dim == b->dim, PFEM_E_INVALID_ARG, "all meshes of a batch share one dimension");
      require(m->kind() == b->kind, PFEM_E_INVALID_ARG,
              "all meshes of a batch share one element family");
      b->meshes.push_back(m);
      b->offsets.push_back(b->offsets.back() + m->n_dof());
      b->bn_max = std::max(b->bn_max, m->bn);
      b->part_off.push_back(poff);
      poff += (int64_t)m->n_blocks * kRedSlots;
      total += m->n_blocks;
    }
    auto remap = [](const std::vector<int2>& nat) {
      const int total = (int)nat.size();
      std::vector<int2> w(total);
      int cnt[8], pre[8];
      for (int k = 0; k < 8; ++k) cnt[k] = std::max((total - k + 7) / 8, 0);
      pre[0] = 0;
      for (int k = 1; k < 8; ++k) pre[k] = pre[k - 1] + cnt[k - 1];
      for (int i = 0; i < total; ++i) w[i] = nat[pre[i % 8] + i / 8];
      return w;
    };
    std::vector<int2> all_nat, kind_nat[2];
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < meshes[i]->n_blocks; ++k) {
        all_nat.push_back(make_int2(i, k));
        kind_nat[meshes[i]->nonlinear ? 1 : 0].push_back(make_int2(i, k));
      }
    std::vector<int2> w = remap(all_nat);
    b->n_work = total;
    PFEM_HIP(hipMalloc((void**)&b->work, w.size() * sizeof(int2)));
    PFEM_HIP(hipMemcpy(b->work, w.data(), w.size() * sizeof(int2), hipMemcpyHostToDevice));
    for (int kd = 0; kd < 2; ++kd) {
      if (kind_nat[kd].empty()) continue;
      std::vector<int2> wk = remap(kind_nat[kd]);
      b->n_work_kind[kd] = (int)wk.size();
      PFEM_HIP(hipMalloc((void**)&b->work_kind[kd], wk.size() * sizeof(int2)));
      PFEM_HIP(hipMemcpy(b->work_kind[kd], wk.data(), wk.size() * sizeof(int2),
                         hipMemcpyHostToDevice));
    }
    PFEM_HIP(hipMalloc((void**)&b->part, std::max<int64_t>(poff, 1) * 8));
    PFEM_HIP(hipMalloc((void**)&b->outs, (size_t)n * kRedSlots * 8));
    std::vector<Task> ts;
    for (int i = 0; i < n; ++i) {
      Task t{};
      t.m = b->meshes[i]->md;
      const uintptr_t off = (uintptr_t)b->offsets[i];
      t.u = reinterpret_cast<const void*>(off);
      t.v = reinterpret_cast<const void*>(off);
      t.y = reinterpret_cast<void*>(off);
      t.active = 1;
      t.fscale = 1.0;
      t.red.part = b->part + b->part_off[i];
      t.red.out = b->outs + kRedSlots * i;
      ts.push_back(t);
    }
    PFEM_HIP(hipMalloc((void**)&b->tasks_red, ts.size() * sizeof(Task)));
    PFEM_HIP(hipMemcpy(b->tasks_red, ts.data(), ts.size() * sizeof(Task), hipMemcpyHostToDevice));
    for (Task& t : ts) t.red.part = nullptr;
    PFEM_HIP(hipMalloc((void**)&b->tasks_plain, ts.size() * sizeof(Task)));
    PFEM_HIP(hipMemcpy(b->tasks_plain, ts.data(), ts.size() * sizeof(Task),
                       hipMemcpyHostToDevice));
  } catch (...) {
    if (b->work) (void)hipFree(b->work);
    for (int kd = 0; kd < 2; ++kd)
      if (b->work_kind[kd]) (void)hipFree(b->work_kind[kd]);
    if (b->part) (void)hipFree(b->part);
    if (b->outs) (void)hipFree(b->outs);
    if (b->tasks_red) (void)hipFree(b->tasks_red);
    if (b->tasks_plain) (void)hipFree(b->tasks_plain);
    delete b;
    throw;
  }
  ctx_ref(b->ctx);
  *out = b;
  PFEM_TRY_END
}

void pfem_batch_destroy(pfem_batch* b) {
  if (b == nullptr) return;
  (void)hipSetDevice(b->ctx->device);
  (void)hipStreamSynchronize(b->ctx->stream);
  if (b->work) (void)hipFree(b->work);
  for (int kd = 0; kd < 2; ++kd)
    if (b->work_kind[kd]) (void)hipFree(b->work_kind[kd]);
  if (b->part) (void)hipFree(b->part);
  if (b->outs) (void)hipFree(b->outs);
  if (b->tasks_red) (void)hipFree(b->tasks_red);
  if (b->tasks_plain) (void)hipFree(b->tasks_plain);
  ctx_unref(b->ctx);
  delete b;
}

pfem_status pfem_batch_offsets(const pfem_batch* b, int64_t* offsets) {
  PFEM_TRY_BEGIN
  require(b != nullptr && offsets != nullptr, PFEM_E_INVALID_ARG, "NULL argument");
  std::copy(b->offsets.begin(), b->offsets.end(), offsets);
  PFEM_TRY_END
}

pfem_status pfem_batch_energy(pfem_batch* b, int prec, const void* u, double* energies_dev) {
  PFEM_TRY_BEGIN
  require(b != nullptr && u != nullptr && energies_dev != nullptr, PFEM_E_INVALID_ARG,
          "NULL argument");
  check_prec(prec);
  Ctx* ctx = b->ctx;
  PFEM_HIP(hipSetDevice(ctx->device));
  const BaseArgs ba{u, nullptr, nullptr, 1, 0};
  launch_energy(ctx, b->kind, prec, false, b->tasks_red, b->work, b->n_work, &ba);
  launch_reduce_store(ctx, b->tasks_red, (int)b->meshes.size());
  launch_energy_out(ctx, b->outs, energies_dev, (int)b->meshes.size(), kRedSlots);
  PFEM_TRY_END
}

// One launch per model kind (the kinds compile to different kernels); the
// task table is persistent, so a call uploads nothing.
static pfem_status batch_elem(pfem_batch* b, int prec, int mask, int op, const void* u,
                              const void* v, void* y) {
  require(b != nullptr && y != nullptr, PFEM_E_INVALID_ARG, "NULL argument");
  check_prec(prec);
  Ctx* ctx = b->ctx;
  PFEM_HIP(hipSetDevice(ctx->device));
  const BaseArgs ba{u, v, y, 1, mask};
  for (int kd = 0; kd < 2; ++kd)
    if (b->n_work_kind[kd] > 0)
      launch_elem(ctx, b->kind, prec, op, kd == 1, PFEM_SCATTER_OWNER, b->tasks_plain,
                  b->work_kind[kd], b->n_work_kind[kd], b->bn_max, nullptr, nullptr, &ba);
  return PFEM_OK;
}

pfem_status pfem_batch_force(pfem_batch* b, int prec, int mask, const void* u, void* g) {
  PFEM_TRY_BEGIN
  require(u != nullptr, PFEM_E_INVALID_ARG, "u is NULL");
  batch_elem(b, prec, mask, OP_FORCE, u, nullptr, g);
  PFEM_TRY_END
}

pfem_status pfem_batch_hvp(pfem_batch* b, int prec, int mask, const void* u, const void* v,
                           void* y) {
  PFEM_TRY_BEGIN
  require(b != nullptr && v != nullptr, PFEM_E_INVALID_ARG, "NULL argument");
  for (pfem_mesh* m : b->meshes)
    if (m->nonlinear) require(u != nullptr, PFEM_E_INVALID_ARG, "u is NULL");
  batch_elem(b, prec, mask, OP_APPLY, u, v, y);
  PFEM_TRY_END
}

// ----------------------------------------------------------------- solve
void pfem_solve_opts_default(pfem_solve_opts* o) {
  if (o == nullptr) return;
  *o = pfem_solve_opts{};
  o->tol = 1e-8;
  o->tol_fine = 0.0;
  o->max_iter = 0;
  o->n_load_steps = 10;
  o->max_newton = 50;
  o->prec = PFEM_FP32;
  o->record_history = 1;
  o->inner_rtol = 0.0;   // automatic (by PCG formulation)
  o->krylov = PFEM_KRYLOV_AUTO;
  o->precond = PFEM_PRECOND_JACOBI;
}

pfem_status pfem_solve(pfem_mesh* m, const double* u0, const pfem_solve_opts* o, double* u_out,
                       int ptr_is_device, double* history, int64_t history_cap,
                       pfem_solve_report* rep) {
  PFEM_TRY_BEGIN
  require(m != nullptr && o != nullptr && u_out != nullptr, PFEM_E_INVALID_ARG,
          "NULL argument");
  check_solve_opts(*o);
  require(history_cap >= 0, PFEM_E_INVALID_ARG, "history_cap < 0");
  need_device(m);
  Ctx* ctx = m->ctx;
  const int64_t nd = m->n_dof();
  const int64_t hcap = (o->record_history && history) ? history_cap : 0;
  m->scratch.ensure(nd, m->n_blocks);
  // (re)use the mesh's cached solver state
  std::unique_ptr<SolveState>& cached = m->solve_state;
  const int prec = o->prec;
  check_solve_mesh(*o, m);
  const bool fused = krylov_fused(*o, m);
  const bool two_level = o->precond == PFEM_PRECOND_TWO_LEVEL;
  if (!cached || cached->prec != prec || cached->hist_cap < hcap || cached->fused != fused ||
      (two_level && cached->tl_dev == nullptr)) {
    cached.reset();
    cached.reset(new SolveState());
    cached->alloc(prec, nd, m->n_blocks, std::max<int64_t>(hcap, 1024), m->nonlinear, fused,
                  nh_cache_values(m));
    if (two_level) {
      coarse_upload(m, ctx);
      cached->alloc_two_level(m);
    }
  }
  SlotRun s;
  s.m = m;
  s.o = *o;
  s.prec = prec;
  s.nl = m->nonlinear;
  s.st = cached.get();
  PFEM_HIP(hipHostMalloc((void**)&s.sc_host, sizeof(Scalars), hipHostMallocDefault));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  pfem_status status = PFEM_OK;
  try {
    PFEM_HIP(hipEventCreate(&e0));
    PFEM_HIP(hipEventCreate(&e1));
    const double* u0_int = nullptr;
    if (u0 != nullptr) {
      const void* src = u0;
      if (!ptr_is_device) {
        PFEM_HIP(hipMemcpyAsync(m->scratch.v64, u0, nd * 8, hipMemcpyHostToDevice, ctx->stream));
        src = m->scratch.v64;
      }
      launch_permute(ctx, PFEM_FP64, m->dim, m->dev.perm, m->n_nodes, true, src, m->scratch.in64);
      u0_int = static_cast<const double*>(m->scratch.in64);
    }
    PFEM_HIP(hipEventRecord(e0, ctx->stream));
    slot_begin(ctx, &s, u0_int);
    std::vector<SlotRun*> live{&s};
    int64_t launches = 0;
    while (engine_tick(ctx, live, &launches) > 0) {
    }
    PFEM_HIP(hipEventRecord(e1, ctx->stream));
    // outputs
    if (ptr_is_device) {
      launch_permute(ctx, PFEM_FP64, m->dim, m->dev.perm, m->n_nodes, false, s.st->x64, u_out);
    } else {
      launch_permute(ctx, PFEM_FP64, m->dim, m->dev.perm, m->n_nodes, false, s.st->x64,
                     m->scratch.out64);
      PFEM_HIP(hipMemcpyAsync(u_out, m->scratch.out64, nd * 8, hipMemcpyDeviceToHost, ctx->stream));
    }
    PFEM_HIP(hipMemcpyAsync(s.sc_host, s.st->sc, sizeof(Scalars), hipMemcpyDeviceToHost,
                            ctx->stream));
    PFEM_HIP(hipStreamSynchronize(ctx->stream));
    const int64_t hl = std::min<int64_t>(s.sc_host->hist_len, hcap);
    if (hl > 0)
      PFEM_HIP(hipMemcpy(history, s.st->hist, hl * 8, hipMemcpyDeviceToHost));
    float ms = 0.f;
    PFEM_HIP(hipEventElapsedTime(&ms, e0, e1));
    s.rep.history_len = hl;
    s.rep.t_device_ms = ms;
    s.rep.status = s.status;
    if (rep) *rep = s.rep;
    status = s.status;
  } catch (...) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipHostFree(s.sc_host);
    s.st = nullptr;
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipHostFree(s.sc_host);
  s.sc_host = nullptr;
  s.st = nullptr;
  if (status < 0) {
    set_error(std::string("solve failed with status ") + std::to_string(status));
    return status;
  }
  set_error("");
  return status;
  PFEM_TRY_END
}

}  // extern "C"
