// Batched solve engine (see solver.h).
#include "solver.h"

#include "coarse.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>

namespace pfem {

// ------------------------------------------------------------ state memory
void SolveState::alloc(int pr, int64_t nd, int nb, int64_t hcap, bool nonlinear,
                       bool fused_pcg, int64_t nh_cache_vals) {
  prec = pr;
  fused = fused_pcg;
  n_dof = nd;
  n_blocks = nb;
  const size_t s = pr == PFEM_FP64 ? 8 : 4;
  bytes = 0;
  auto A = [&](void** p, size_t n) {
    PFEM_HIP(hipMalloc(p, std::max<size_t>(n, 8)));
    bytes += (int64_t)std::max<size_t>(n, 8);
  };
  A((void**)&x64, nd * 8);
  A((void**)&g64, nd * 8);
  A((void**)&aux64, nd * 8);
  A(&d, nd * s);
  A(&r, nd * s);
  A(&p, nd * s);
  A(&q, nd * s);
  A(&minv, nd * s);
  if (nonlinear && pr == PFEM_FP32) A(&u32, nd * 4);
  if (nh_cache_vals > 0) A(&nhc, (size_t)nh_cache_vals * s);
  if (fused_pcg) {
    A(&rec[0], 4 * nd * s);
    A(&rec[1], 4 * nd * s);
    A(&tmp, nd * s);
  }
  A((void**)&part, (size_t)std::max(nb, 1) * 2 * kRedSlots * 8);
  A((void**)&sc, sizeof(Scalars));
  PFEM_HIP(hipMemset(sc, 0, sizeof(Scalars)));
  hist_cap = std::max<int64_t>(hcap, 0);
  A((void**)&hist, (size_t)std::max<int64_t>(hist_cap, 1) * 8);
  Scalars init{};
  init.hist_cap = (int32_t)std::min<int64_t>(hist_cap, INT32_MAX);
  PFEM_HIP(hipMemcpy(sc, &init, sizeof(Scalars), hipMemcpyHostToDevice));
}

void SolveState::alloc_two_level(const pfem_mesh* m) {
  const CoarseHost& c = *m->coarse;
  auto A = [&](void** p, size_t n) {
    PFEM_HIP(hipMalloc(p, std::max<size_t>(n, 8)));
    bytes += (int64_t)std::max<size_t>(n, 8);
  };
  const int n_chunks = (c.n_c + kCoarseRows - 1) / kCoarseRows;
  A((void**)&rc_part, (size_t)std::max(m->n_blocks, 1) * 6 * 8);
  A((void**)&tl_y, (size_t)c.n_agg * 6 * 8);
  A((void**)&gc_part, (size_t)n_chunks * 8);
  A((void**)&tl_dev, sizeof(TwoLevelDev));
  TwoLevelDev t{};
  t.rel = prec == PFEM_FP64 ? (const void*)m->dev.coarse_rel64 : (const void*)m->dev.coarse_rel32;
  t.B = prec == PFEM_FP64 ? (const void*)m->dev.coarse_B64 : (const void*)m->dev.coarse_B32;
  t.rc_part = rc_part;
  t.y = tl_y;
  t.gc_part = gc_part;
  t.nrb = c.n_rb;
  t.G = c.G;
  t.n_agg = c.n_agg;
  t.n_c = c.n_c;
  t.n_chunks = n_chunks;
  PFEM_HIP(hipMemcpy(tl_dev, &t, sizeof(t), hipMemcpyHostToDevice));
}

void SolveState::release() {
  void* ptrs[] = {x64, g64, aux64, d, r, p, q, minv, u32, nhc, rec[0], rec[1], tmp, part, sc,
                  hist, rc_part, tl_y, gc_part, tl_dev};
  for (void* ptr : ptrs)
    if (ptr != nullptr) (void)hipFree(ptr);
  x64 = g64 = aux64 = nullptr;
  d = r = p = q = minv = u32 = nhc = nullptr;
  rec[0] = rec[1] = tmp = nullptr;
  part = nullptr;
  sc = nullptr;
  hist = nullptr;
  rc_part = tl_y = gc_part = nullptr;
  tl_dev = nullptr;
  bytes = 0;
}

void check_solve_opts(const pfem_solve_opts& o) {
  require(o.tol > 0 && std::isfinite(o.tol), PFEM_E_INVALID_ARG, "tol must be finite and > 0");
  require(o.prec == PFEM_FP64 || o.prec == PFEM_FP32, PFEM_E_INVALID_ARG, "bad precision");
  require(o.krylov >= PFEM_KRYLOV_AUTO && o.krylov <= PFEM_KRYLOV_FUSED, PFEM_E_INVALID_ARG,
          "bad krylov formulation");
  require(o.inner_rtol >= 0.0 && o.inner_rtol <= 0.5, PFEM_E_INVALID_ARG,
          "inner_rtol must be 0 (automatic) or in (0, 0.5]");
  require(o.precond == PFEM_PRECOND_JACOBI || o.precond == PFEM_PRECOND_TWO_LEVEL,
          PFEM_E_INVALID_ARG, "bad preconditioner");
  require(!(o.precond == PFEM_PRECOND_TWO_LEVEL && o.krylov == PFEM_KRYLOV_FUSED),
          PFEM_E_INVALID_ARG, "the two-level preconditioner runs with the classic PCG loop");
}

void check_solve_mesh(const pfem_solve_opts& o, const pfem_mesh* m) {
  require(!(krylov_fused(o, m) && !m->pairs.empty()), PFEM_E_INVALID_ARG,
          "the fused PCG does not apply periodic springs: use the classic formulation");
  if (m->elem != PFEM_ELEM_P1) {
    require(o.krylov != PFEM_KRYLOV_FUSED, PFEM_E_INVALID_ARG,
            "quadrilateral meshes run the classic PCG loop");
    require(o.precond != PFEM_PRECOND_TWO_LEVEL, PFEM_E_INVALID_ARG,
            "the two-level preconditioner is built for P1 meshes");
  }
}

void slot_alloc(SlotRun* s, pfem_mesh* m, const pfem_solve_opts& o, int64_t hist_cap) {
  check_solve_mesh(o, m);
  s->m = m;
  s->o = o;
  s->prec = o.prec == PFEM_FP64 ? PFEM_FP64 : PFEM_FP32;
  s->nl = m->nonlinear;
  s->st = new SolveState();
  try {
    s->st->alloc(s->prec, m->n_dof(), m->n_blocks, hist_cap, m->nonlinear, krylov_fused(o, m),
                 nh_cache_values(m));
    if (o.precond == PFEM_PRECOND_TWO_LEVEL) {
      require(m->uploaded && m->ctx != nullptr, PFEM_E_STATE, "mesh has no device context");
      coarse_upload(m, m->ctx);
      s->st->alloc_two_level(m);
    }
    PFEM_HIP(hipHostMalloc((void**)&s->sc_host, sizeof(Scalars), hipHostMallocDefault));
  } catch (...) {
    delete s->st;
    s->st = nullptr;
    throw;
  }
}

void slot_free(SlotRun* s) {
  delete s->st;
  s->st = nullptr;
  if (s->sc_host != nullptr) (void)hipHostFree(s->sc_host);
  s->sc_host = nullptr;
}

// ---------------------------------------------------------------- helpers
// Algorithmic bytes of one apply (K.v / HVP) or one fused PCG iteration of a
// slot: connectivity, one material value per element and the coordinates
// once, then the apply's input and output, or the fused iteration's node
// records ({r, w, s, M^-1} read, {r, w, s} written) and p and d (read and
// written); Neo-Hookean meshes also read the state u -- counted as the
// nodal state also where the kernels read the per-element cache of it
// instead (more bytes, less arithmetic: the difference is traffic above
// the algorithmic count, not part of it).
static double alg_bytes(const SlotRun* s, bool fused) {
  const double d = s->m->dim, ne = (double)s->m->n_elems, nn = (double)s->m->n_nodes;
  const double sz = s->prec == PFEM_FP64 ? 8.0 : 4.0;
  // a right-hand side after the first of a multi-right-hand-side apply
  // shares the element data read for the first
  double b = s->shares_elements ? 0.0 : 4.0 * s->m->nv * ne + sz * ne + d * sz * nn;
  b += (fused ? 11.0 : 2.0) * d * sz * nn;
  if (s->nl) b += d * sz * nn;
  return b;
}

// A cached solver state may carry two-level buffers from an earlier solve;
// the options of this solve decide whether they are used.
static bool uses_two_level(const SlotRun* s) {
  return s->o.precond == PFEM_PRECOND_TWO_LEVEL && s->st->tl_dev != nullptr;
}

static Task base_task(SlotRun* s) {
  Task t{};
  t.m = s->m->md;
  t.active = 1;
  t.sc = s->st->sc;
  t.hist = s->st->hist;
  t.minv = s->st->minv;
  t.r = s->st->r;
  t.p = s->st->p;
  t.d = s->st->d;
  t.red.part = s->st->part;
  t.red.out = &s->st->sc->red[0];
  t.rec[0] = s->st->rec[0];
  t.rec[1] = s->st->rec[1];
  t.tmp = s->st->tmp;
  t.mask = PFEM_MASK_OUT;
  t.k_base = s->k_before;
  t.hist_base = s->hist_base;
  t.fscale = (double)s->step / s->n_steps;   // load step n applies n / N_f of the load
  t.fext = s->fext;
  t.tl = uses_two_level(s) ? s->st->tl_dev : nullptr;
  return t;
}

struct Group {
  int dim, kind, prec;   // kind: element kernel family (pfem::elem_kind)
  bool nl;
  bool fused;
  bool tl;   // two-level preconditioner
  std::vector<SlotRun*> slots;
};

// Groups slots by (dim, precision, model kind, PCG formulation) so one
// templated launch covers a group.
static std::vector<Group> group_by(const std::vector<SlotRun*>& v, bool force_fp64) {
  std::map<std::tuple<int, int, int, int, int>, Group> g;
  for (SlotRun* s : v) {
    const int pr = force_fp64 ? PFEM_FP64 : s->prec;
    const bool fused = !force_fp64 && s->st->fused;
    const bool tl = !force_fp64 && uses_two_level(s);
    const int kind = s->m->kind();
    auto key = std::make_tuple(kind, pr, s->nl ? 1 : 0, fused ? 1 : 0, tl ? 1 : 0);
    auto it = g.find(key);
    if (it == g.end())
      it = g.emplace(key, Group{s->m->dim, kind, pr, s->nl, fused, tl, {}}).first;
    it->second.slots.push_back(s);
  }
  std::vector<Group> out;
  for (auto& kv : g) out.push_back(kv.second);
  return out;
}

struct Uploaded {
  const Task* tasks = nullptr;
  const int2* work = nullptr;
  int n_work = 0;
  int bn_max = 0;
};

// Work table for a group: all (task, block) pairs, remapped so that
// consecutive blocks of a mesh land on the same XCD.
static Uploaded upload_group(Ctx* ctx, const Group& g, const std::vector<Task>& tasks) {
  Uploaded u;
  u.tasks = static_cast<const Task*>(ctx->ring.put(tasks.data(), tasks.size() * sizeof(Task)));
  int total = 0;
  for (SlotRun* s : g.slots) {
    total += s->m->n_blocks;
    u.bn_max = std::max(u.bn_max, s->m->bn);
  }
  u.n_work = total;
  if (g.slots.size() == 1) {
    u.work = g.slots[0]->m->dev.work;   // persistent single-mesh table (task 0)
    return u;
  }
  std::vector<int2> nat;
  nat.reserve(total);
  for (size_t i = 0; i < g.slots.size(); ++i)
    for (int b = 0; b < g.slots[i]->m->n_blocks; ++b) nat.push_back(make_int2((int)i, b));
  std::vector<int2> w(total);
  int cnt[8], pre[8];
  for (int k = 0; k < 8; ++k) cnt[k] = std::max((total - k + 7) / 8, 0);
  pre[0] = 0;
  for (int k = 1; k < 8; ++k) pre[k] = pre[k - 1] + cnt[k - 1];
  for (int i = 0; i < total; ++i) w[i] = nat[pre[i % 8] + i / 8];
  u.work = static_cast<const int2*>(ctx->ring.put(w.data(), w.size() * sizeof(int2)));
  return u;
}

// Work items (task, chunk of aggregates) of the coarse solve of a group.
static const int2* coarse_work(Ctx* ctx, const Group& g, int* n_items) {
  std::vector<int2> w;
  for (size_t i = 0; i < g.slots.size(); ++i) {
    const CoarseHost& c = *g.slots[i]->m->coarse;
    const int nch = (c.n_c + kCoarseRows - 1) / kCoarseRows;
    for (int k = 0; k < nch; ++k) w.push_back(make_int2((int)i, k));
  }
  *n_items = (int)w.size();
  return static_cast<const int2*>(ctx->ring.put(w.data(), w.size() * sizeof(int2)));
}

// Sweeps in a row without halving the true residual that end a linear solve.
constexpr int kStalledSweeps = 3;

// Input of a slot's Hessian-vector products: the per-element cache of the
// Newton state where the solve keeps one (P1), else the nodal state.
static void* hvp_state(const SlotRun* s) {
  if (!s->nl) return nullptr;
  if (s->st->nhc != nullptr) return s->st->nhc;
  return s->prec == PFEM_FP32 ? s->st->u32 : (void*)s->st->x64;
}

// Element op of a group's Krylov products.
static int apply_op(const Group& g) {
  return g.nl && !is_quad_kind(g.kind) ? OP_HVPC : OP_APPLY;
}

static double inner_target(const SlotRun* s) {
  const double floor_abs = 0.5 * s->o.tol * s->den;
  if (!s->nl) {
    if (s->prec == PFEM_FP64) return s->o.tol * s->den;
    // automatic: the reduction per sweep that minimised the work of a warm
    // 200k-triangle solve for each formulation (fused 1e-4, classic 1e-3)
    const double rt = s->o.inner_rtol > 0 ? s->o.inner_rtol : (s->st->fused ? 1e-4 : 1e-3);
    return std::max(rt * s->gnorm, floor_abs);
  }
  double eta = std::min(0.1, s->rho);
  if (s->prec == PFEM_FP32) eta = std::max(eta, 1e-5);
  return std::max(eta * s->gnorm, floor_abs);
}

static void finish(SlotRun* s, pfem_status st) {
  s->status = st;
  s->finished = true;
  s->action = A_DONE;
  s->rep.status = st;
  s->rep.rel_residual_final = s->rho;
}

// ----------------------------------------------------------------- begin
void slot_begin(Ctx* ctx, SlotRun* s, const double* u0_dev) {
  pfem_mesh* m = s->m;
  s->warm = u0_dev != nullptr;
  s->n_steps = s->nl ? std::max(1, s->o.n_load_steps) : 1;
  s->step = (s->warm || !s->nl) ? s->n_steps : 1;
  // automatic cap on K.v products over the whole solve: 10 per free DOF plus
  // 1000 per load step (a Newton solve runs one Krylov loop per iteration of
  // every load step; on a mesh with a handful of free DOFs 10 per DOF alone
  // stopped it after the first steps)
  s->max_iter = s->o.max_iter > 0
                    ? s->o.max_iter
                    : (int)std::min<int64_t>(10 * std::max<int64_t>(m->n_free, 1) +
                                                 1000 * (int64_t)s->n_steps,
                                             INT32_MAX / 2);
  s->rep = pfem_solve_report{};
  s->first_resid = true;
  s->minv_valid = false;
  s->newton_in_step = 0;
  s->rho_sweep = 0.0;
  s->stalled = 0;
  s->finished = false;
  s->status = PFEM_OK;
  const double scale = (double)s->step / s->n_steps;
  // x64: caller guess (Dirichlet DOFs forced to the load-step values) or lift
  if (s->warm)
    launch_axpy_state(ctx, PFEM_FP64, m->md, s->st->x64, u0_dev, nullptr, 0.0, true, scale);
  else
    launch_lift(ctx, m->md, s->st->x64, nullptr, scale);
  launch_lift(ctx, m->md, s->st->aux64, nullptr, scale);
  launch_set_scalars(ctx, s->st->sc, 1.0, 0.0, 0, true, true);
  s->hist_len_host = 0;
  s->action = A_DEN;
}

// ------------------------------------------------------------- launches
static void do_force(Ctx* ctx, const std::vector<SlotRun*>& v, bool at_lift, int64_t* nl) {
  for (const Group& g : group_by(v, true)) {
    std::vector<Task> ts;
    for (SlotRun* s : g.slots) {
      Task t = base_task(s);
      t.u = at_lift ? s->st->aux64 : s->st->x64;
      t.y = s->st->g64;
      t.w = nullptr;
      ts.push_back(t);
    }
    Uploaded u = upload_group(ctx, g, ts);
    launch_elem(ctx, g.kind, PFEM_FP64, OP_FORCE, g.nl, PFEM_SCATTER_OWNER, u.tasks, u.work,
                u.n_work, u.bn_max, nullptr, nullptr);
    launch_reduce_store(ctx, u.tasks, (int)ts.size());
    *nl += 2;
  }
}

static void do_krylov(Ctx* ctx, const std::vector<SlotRun*>& start,
                      const std::vector<SlotRun*>& all, int64_t* nl) {
  // chunk bookkeeping: iterations done so far and where history goes
  for (SlotRun* s : all) {
    if (s->action == A_KRYLOV_START) {
      s->k_before = 0;
      const int64_t h0 = s->hist_len_host;
      s->hist_base = (h0 == 0 && s->st->hist_cap > 0) ? 1 : (int)h0;
    } else {
      s->k_before = s->sc_host->k;
    }
  }
  // diagonal + init for the slots that start an inner solve
  if (!start.empty()) {
    std::vector<SlotRun*> need_diag;
    for (SlotRun* s : start) {
      if (s->nl && s->prec == PFEM_FP32)
        launch_cast(ctx, true, s->st->x64, s->st->u32, s->m->n_dof());
      if (s->nl || !s->minv_valid) need_diag.push_back(s);
      launch_set_scalars(ctx, s->st->sc, s->den, inner_target(s) * inner_target(s),
                         std::max(0, s->max_iter - s->rep.kv_count - (s->st->fused ? 1 : 0)),
                         false, false);
    }
    // Neo-Hookean: the element state of this Newton step, once for all of
    // its Krylov products
    std::vector<SlotRun*> need_cache;
    for (SlotRun* s : start)
      if (s->nl && s->st->nhc != nullptr) need_cache.push_back(s);
    for (const Group& g : group_by(need_cache, false)) {
      std::vector<Task> ts;
      for (SlotRun* s : g.slots) {
        Task t = base_task(s);
        t.u = s->prec == PFEM_FP32 ? s->st->u32 : (void*)s->st->x64;
        t.y = s->st->nhc;
        ts.push_back(t);
      }
      Uploaded u = upload_group(ctx, g, ts);
      launch_nh_cache(ctx, g.dim, g.prec, u.tasks, u.work, u.n_work);
      ++*nl;
    }
    for (const Group& g : group_by(need_diag, false)) {
      std::vector<Task> ts;
      for (SlotRun* s : g.slots) {
        Task t = base_task(s);
        t.u = s->nl ? (s->prec == PFEM_FP32 ? s->st->u32 : (void*)s->st->x64) : nullptr;
        t.y = s->st->minv;
        t.s = 1.0;  // write the inverse diagonal
        t.red.part = nullptr;
        ts.push_back(t);
        s->minv_valid = true;
      }
      Uploaded u = upload_group(ctx, g, ts);
      launch_elem(ctx, g.kind, g.prec, OP_DIAG, g.nl, PFEM_SCATTER_OWNER, u.tasks, u.work, u.n_work,
                  u.bn_max, nullptr, nullptr);
      ++*nl;
    }
    for (const Group& g : group_by(start, false)) {
      std::vector<Task> ts;
      for (SlotRun* s : g.slots) {
        Task t = base_task(s);
        t.u = s->st->g64;
        ts.push_back(t);
      }
      Uploaded u = upload_group(ctx, g, ts);
      if (g.tl) {   // r = -g, then p = M^-1 r through the coarse solve
        int ncw = 0;
        const int2* cw = coarse_work(ctx, g, &ncw);
        launch_tl_init(ctx, g.dim, g.prec, u.tasks, u.work, u.n_work);
        launch_tl_coarse(ctx, g.prec, u.tasks, cw, ncw, 1);
        launch_tl_prolong_init(ctx, g.dim, g.prec, u.tasks, u.work, u.n_work);
        launch_pcg_init_finish(ctx, u.tasks, (int)ts.size());
        *nl += 4;
        continue;
      }
      if (!g.fused) {
        launch_pcg_init(ctx, g.dim, g.prec, u.tasks, u.work, u.n_work, (int)ts.size());
        *nl += 2;
        continue;
      }
      // fused start: records {r, 0, 0, M^-1}, p = u = M^-1 r, d = 0;
      // tmp = A u (+ partial w.u); w of the records = tmp
      launch_fcg_init(ctx, g.dim, g.prec, u.tasks, u.work, u.n_work);
      std::vector<Task> ta;
      for (SlotRun* s : g.slots) {
        Task t = base_task(s);
        t.u = hvp_state(s);
        t.v = s->st->p;
        t.y = s->st->tmp;
        t.w = s->st->p;
        ta.push_back(t);
      }
      Uploaded ua = upload_group(ctx, g, ta);
      launch_elem(ctx, g.kind, g.prec, apply_op(g), g.nl, PFEM_SCATTER_OWNER, ua.tasks, ua.work,
                  ua.n_work, ua.bn_max, nullptr, nullptr);
      if (ctx->timing & (1 << FAM_APPLY)) {
        ctx->fam_run[FAM_APPLY] += 1;
        for (SlotRun* s : g.slots) ctx->fam_alg_bytes[FAM_APPLY] += alg_bytes(s, false);
      }
      launch_fcg_init_w(ctx, g.dim, g.prec, u.tasks, u.work, u.n_work);
      launch_pcg_init_finish(ctx, u.tasks, (int)ts.size());
      *nl += 4;
    }
  }
  // chunk of iterations for every Krylov slot
  int k = 0;
  for (SlotRun* s : all) k = std::max(k, s->chunk);
  for (const Group& g : group_by(all, false)) {
    const int64_t key = ctx->next_key++;
    for (SlotRun* s : g.slots) {
      s->timing_key = key;
      s->chunk_launched = k;
    }
    std::vector<Task> apply, upd;
    for (SlotRun* s : g.slots) {
      Task t = base_task(s);
      t.u = hvp_state(s);
      t.v = s->st->p;
      t.y = s->st->q;
      t.w = s->st->p;
      t.pcg = 1;
      apply.push_back(t);
      Task t2 = base_task(s);
      t2.y = s->st->q;
      t2.pcg = 1;
      upd.push_back(t2);
    }
    Uploaded ua = upload_group(ctx, g, apply);
    ctx->cur_key = key;
    if (g.fused) {
      // the chunk is timed as one run of k launches
      hipEvent_t ev = nullptr;
      ctx->timing_begin_run(FAM_FUSED, &ev);
      bool packed = true;
      for (SlotRun* sr : g.slots) packed = packed && sr->m->md.conn_packed != 0;
      for (int it = 0; it < k; ++it) {
        launch_fcg_iter(ctx, g.dim, g.prec, g.nl, ua.tasks, ua.work, ua.n_work, ua.bn_max, it,
                        packed);
        *nl += 1;
      }
      ctx->timing_end_run(FAM_FUSED, ev, k);
      ctx->cur_key = -1;
      ctx->cur_it = 0;
      continue;
    }
    Uploaded uu = upload_group(ctx, g, upd);
    // several right-hand sides on one linear 3D mesh (a homogenisation's
    // cell problems): one element visit serves all of them
    bool one_mesh = g.dim == 3 && !g.nl && g.slots.size() >= 2;
    for (SlotRun* sr : g.slots) one_mesh = one_mesh && sr->m == g.slots[0]->m;
    const bool multi = one_mesh && owner_multi_fits(g.slots[0]->m->bn, (int)g.slots.size());
    for (size_t i = 0; i < g.slots.size(); ++i) g.slots[i]->shares_elements = multi && i > 0;
    int ncw = 0;
    const int2* cw = g.tl ? coarse_work(ctx, g, &ncw) : nullptr;
    for (int it = 0; it < k; ++it) {
      ctx->cur_it = it;
      if (multi)
        launch_owner_multi(ctx, g.prec, ua.tasks, (int)g.slots.size(), g.slots[0]->m->dev.work,
                           g.slots[0]->m->n_blocks, g.slots[0]->m->bn);
      else
        launch_elem(ctx, g.kind, g.prec, apply_op(g), g.nl, PFEM_SCATTER_OWNER, ua.tasks,
                    ua.work, ua.n_work, ua.bn_max, nullptr, nullptr);
      if (g.tl) {
        launch_tl_update(ctx, g.dim, g.prec, uu.tasks, uu.work, uu.n_work, it);
        launch_tl_coarse(ctx, g.prec, uu.tasks, cw, ncw, 0);
        launch_tl_direction(ctx, g.dim, g.prec, uu.tasks, uu.work, uu.n_work, it);
        *nl += 4;
      } else {
        launch_pcg_update(ctx, g.dim, g.prec, uu.tasks, uu.work, uu.n_work, it);
        launch_pcg_direction(ctx, g.dim, g.prec, uu.tasks, uu.work, uu.n_work, it);
        *nl += 3;
      }
    }
    ctx->cur_key = -1;
    ctx->cur_it = 0;
  }
}

static void do_linesearch(Ctx* ctx, const std::vector<SlotRun*>& v, int64_t* nl) {
  std::vector<SlotRun*> first;
  for (SlotRun* s : v)
    if (s->ls_tries == 0) first.push_back(s);
  for (const Group& g : group_by(first, false)) {   // slope g . d -> lsred[0]
    std::vector<Task> ts;
    for (SlotRun* s : g.slots) {
      Task t = base_task(s);
      t.u = s->st->g64;
      t.v = s->st->d;
      t.red.out = &s->st->sc->lsred[0];
      ts.push_back(t);
    }
    Uploaded u = upload_group(ctx, g, ts);
    launch_dot(ctx, g.dim, g.prec, u.tasks, u.work, u.n_work);
    launch_reduce_store(ctx, u.tasks, (int)ts.size());
    *nl += 2;
  }
  // Pi(x + s d) - Pi(x) -> red[0], #inverted -> red[1], sum of |terms| -> red[2]
  for (const Group& g : group_by(v, false)) {
    std::vector<Task> ts;
    for (SlotRun* s : g.slots) {
      Task t = base_task(s);
      t.u = s->st->x64;
      t.v = s->st->d;
      t.s = s->ls_s;
      ts.push_back(t);
    }
    Uploaded u = upload_group(ctx, g, ts);
    launch_energy(ctx, g.kind, g.prec, true, u.tasks, u.work, u.n_work);
    launch_reduce_store(ctx, u.tasks, (int)ts.size(), 3);
    *nl += 2;
  }
}

// -------------------------------------------------------- transitions
static void after_resid(Ctx* ctx, SlotRun* s) {
  const Scalars& h = *s->sc_host;
  s->gnorm = std::sqrt(h.red[1]);
  s->rho = s->gnorm / s->den;
  s->rep.residual_evals += 1;
  if (!std::isfinite(s->rho)) {
    finish(s, PFEM_E_BREAKDOWN);
    return;
  }
  if (s->first_resid) {
    s->first_resid = false;
    s->rep.rel_residual_initial = s->rho;
    if (s->o.tol_fine > 0 && s->rho < s->o.tol_fine) {
      finish(s, PFEM_SKIPPED_FINE);
      return;
    }
  }
  if (s->rho <= s->o.tol) {
    if (s->nl) s->rep.load_steps_done += 1;
    if (s->nl && s->step < s->n_steps) {
      s->step += 1;
      const double scale = (double)s->step / s->n_steps;
      // predictor: the converged state scaled to the new load fraction
      // (exact for a linear response; the Dirichlet DOFs land exactly on
      // the new values), instead of moving only the prescribed DOFs
      launch_axpy_state(ctx, PFEM_FP64, s->m->md, s->st->x64, nullptr, s->st->x64,
                        (double)s->step / (s->step - 1), true, scale);
      launch_lift(ctx, s->m->md, s->st->aux64, nullptr, scale);
      s->newton_in_step = 0;
      s->first_resid = false;
      s->action = A_DEN;
      return;
    }
    finish(s, PFEM_OK);
    return;
  }
  if (s->rep.kv_count >= s->max_iter) {
    finish(s, PFEM_NOT_CONVERGED);
    return;
  }
  if (!s->nl) {
    // Every sweep of a linear solve starts from the true residual.  When
    // tol lies below what the FP64 residual evaluation can resolve on this
    // mesh (its rounding grows with the mesh size), each sweep meets its
    // recurred target in a few iterations and the true residual stays at
    // that floor; three sweeps in a row that fail to halve it end the solve.
    if (s->rep.outer_sweeps > 0) s->stalled = s->rho > 0.5 * s->rho_sweep ? s->stalled + 1 : 0;
    if (s->stalled >= kStalledSweeps) {
      finish(s, PFEM_NOT_CONVERGED);
      return;
    }
    s->rho_sweep = s->rho;
  }
  if (s->nl && s->newton_in_step >= (s->o.max_newton > 0 ? s->o.max_newton : 50)) {
    finish(s, PFEM_NOT_CONVERGED);
    return;
  }
  s->chunk = 16;
  s->k_chunk = 0;
  s->rho_chunk = s->rho;
  s->action = A_KRYLOV_START;
}

static void after_krylov(Ctx* ctx, SlotRun* s) {
  const Scalars& h = *s->sc_host;
  if (h.state == 0) {
    // still running: size the next chunk from the observed convergence rate
    const int dk = h.k - s->k_chunk;
    int next = std::min(2 * s->chunk, 256);
    if (dk > 0 && h.rho > 0 && s->rho_chunk > 0 && h.rho < s->rho_chunk) {
      const double rate = std::log(s->rho_chunk / h.rho) / dk;
      const double target = std::sqrt(std::max(h.target2, 1e-300)) / s->den;
      const double rem = std::log(h.rho / std::max(target, 1e-300)) / rate;
      next = (int)std::min(256.0, std::max(8.0, rem + 2.0));
    }
    s->chunk = next;
    s->k_chunk = h.k;
    s->rho_chunk = h.rho;
    s->action = A_KRYLOV;
    return;
  }
  // the fused start applies A once more (w = A u) before iteration 0
  s->rep.kv_count += h.k + (s->st->fused ? 1 : 0);
  s->rep.pcg_iters += h.k;
  s->rep.outer_sweeps += 1;
  if (h.state == 3 && (!s->nl || h.k == 0)) {
    if (!s->nl) {
      finish(s, PFEM_E_BREAKDOWN);
      return;
    }
    // negative curvature on the first step: preconditioned steepest descent
    // (M^-1 r: the first direction of both formulations, held in p)
    PFEM_HIP(hipMemcpyAsync(s->st->d, s->st->p,
                            s->m->n_dof() * (s->prec == PFEM_FP64 ? 8 : 4),
                            hipMemcpyDeviceToDevice, ctx->stream));
  }
  if (!s->nl) {
    launch_axpy_state(ctx, s->prec, s->m->md, s->st->x64, s->st->x64, s->st->d, 1.0, false, 0.0);
    s->action = A_RESID;
    return;
  }
  s->ls_s = 1.0;
  s->ls_tries = 0;
  s->action = A_LS;
}

static void after_ls(Ctx* ctx, SlotRun* s) {
  const Scalars& h = *s->sc_host;
  if (s->ls_tries == 0) s->ls_slope = h.lsred[0];
  s->rep.line_search_evals += 1;
  const double de = h.red[0];
  const bool inverted = h.red[1] > 0.5;
  // Armijo on the energy; a change within the rounding level of the summed
  // terms is inconclusive (near convergence the decrease of a Newton step
  // falls below what float64 resolves) and the step is taken, leaving the
  // decision to the residual test.
  const double noise = 64.0 * 2.220446049250313e-16 * h.red[2];
  if (!inverted && std::isfinite(de) &&
      (de <= 1e-4 * s->ls_s * s->ls_slope || std::fabs(de) <= noise)) {
    launch_axpy_state(ctx, s->prec, s->m->md, s->st->x64, s->st->x64, s->st->d, s->ls_s,
                      false, 0.0);
    s->newton_in_step += 1;
    s->rep.newton_iters += 1;
    s->action = A_RESID;
    return;
  }
  s->ls_tries += 1;
  if (s->ls_tries > 20) {
    finish(s, inverted ? PFEM_E_INVERTED : PFEM_E_LINESEARCH);
    return;
  }
  s->ls_s *= 0.5;
  s->action = A_LS;
}

int engine_tick(Ctx* ctx, std::vector<SlotRun*>& live, int64_t* launches,
                const std::function<void()>* overlap) {
  std::vector<SlotRun*> den, resid, kstart, kall, ls;
  for (SlotRun* s : live) {
    if (s->finished) continue;
    switch (s->action) {
      case A_DEN: den.push_back(s); break;
      case A_RESID: resid.push_back(s); break;
      case A_KRYLOV_START: kstart.push_back(s); kall.push_back(s); break;
      case A_KRYLOV: kall.push_back(s); break;
      case A_LS: ls.push_back(s); break;
      default: break;
    }
  }
  int64_t nl = 0;
  if (!den.empty()) do_force(ctx, den, true, &nl);
  if (!resid.empty()) do_force(ctx, resid, false, &nl);
  if (!kall.empty()) do_krylov(ctx, kstart, kall, &nl);
  if (!ls.empty()) do_linesearch(ctx, ls, &nl);
  // read back the scalars of every slot that did something
  std::vector<SlotRun*> touched;
  touched.insert(touched.end(), den.begin(), den.end());
  touched.insert(touched.end(), resid.begin(), resid.end());
  touched.insert(touched.end(), kall.begin(), kall.end());
  touched.insert(touched.end(), ls.begin(), ls.end());
  for (SlotRun* s : touched)
    PFEM_HIP(hipMemcpyAsync(s->sc_host, s->st->sc, sizeof(Scalars), hipMemcpyDeviceToHost,
                            ctx->stream));
  if (overlap != nullptr && *overlap) (*overlap)();
  PFEM_HIP(hipStreamSynchronize(ctx->stream));
  if (launches) *launches += nl;
  for (SlotRun* s : touched) s->hist_len_host = s->sc_host->hist_len;
  for (SlotRun* s : den) {
    const double dn = std::sqrt(s->sc_host->red[1]);
    s->den = dn > 0 ? dn : 1.0;
    s->action = A_RESID;
  }
  for (SlotRun* s : resid) after_resid(ctx, s);
  if (ctx->timing != 0) {
    // launches after the last real iteration of a group returned at once
    // and are not timed: a classic chunk keeps its launches before that
    // point, a fused chunk (timed as one run) is kept only when all of its
    // launches did work.  The kept launches advanced each solve of the
    // group by its own iterations: those are the algorithmic bytes.
    std::map<int64_t, int> ran;
    std::map<int64_t, int> fam_of, launched;
    for (SlotRun* s : kall) {
      int& r = ran[s->timing_key];
      r = std::max(r, s->sc_host->k - s->k_before);
      fam_of[s->timing_key] = s->st->fused ? FAM_FUSED : FAM_APPLY;
      launched[s->timing_key] = s->chunk_launched;
    }
    for (SlotRun* s : kall) {
      const int fam = fam_of[s->timing_key];
      const bool kept = fam == FAM_APPLY || ran[s->timing_key] >= launched[s->timing_key];
      if ((ctx->timing & (1 << fam)) && kept)
        ctx->fam_alg_bytes[fam] += (s->sc_host->k - s->k_before) * alg_bytes(s, s->st->fused);
    }
    for (auto& kv : ran) {
      ctx->drop_noop(kv.first, kv.second);
      const int fam = fam_of[kv.first];
      const bool kept = fam == FAM_APPLY || kv.second >= launched[kv.first];
      if ((ctx->timing & (1 << fam)) && kept) ctx->fam_run[fam] += kv.second;
    }
  }
  for (SlotRun* s : kall) after_krylov(ctx, s);
  for (SlotRun* s : ls) after_ls(ctx, s);
  int running = 0;
  for (SlotRun* s : live)
    if (!s->finished) ++running;
  return running;
}

}  // namespace pfem
