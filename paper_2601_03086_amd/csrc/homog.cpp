// Numerical homogenisation of a periodic cell (App. D): the six cell
// problems of the unit macroscopic strains solved together, and the
// homogenised elasticity tensor from their fluctuation fields.
//
// For load case (IJ) the fluctuation X^v solves (K + P) X^v = F^(IJ): K the
// element stiffness, P the periodic springs between opposite-face nodes
// (the virtual elements of the cell, a penalty), F^(IJ) the element loads
// of the uniform stress E : eps0^(IJ).  P1 elements reproduce the affine
// field X^0 = eps0 . X exactly, so F^(IJ) = K X^0 (elements only).  The six
// solves are six slots of the batched engine on one mesh, so every launch
// of the element kernels covers all of them.  The tensor
// E^H_(IJ)(KL) = 1/|Omega| int (eps0 - eps^v)^(IJ) : E : (eps0 - eps^v)^(KL)
// is the element energy form of the total fields T = X^0 - X^v:
// E^H = T_(IJ) . K T_(KL) / |Omega|, one apply per case and a 6 x 6 Gram.
#include <algorithm>
#include <memory>
#include <vector>

#include "mesh.h"
#include "solver.h"

using namespace pfem;

namespace {

// Device buffers of one call, released on every exit path.
struct DevBufs {
  std::vector<void*> ptrs;
  double* get(size_t n) {
    void* p = nullptr;
    PFEM_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(double)));
    ptrs.push_back(p);
    return static_cast<double*>(p);
  }
  ~DevBufs() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

// y = K x over the elements alone (no periodic springs), float64, internal
// order, one launch.
void apply_elements(Ctx* ctx, pfem_mesh* m, const double* x, double* y) {
  Task t{};
  t.m = m->md;
  t.v = x;
  t.y = y;
  t.active = 1;
  t.fscale = 1.0;
  t.no_pairs = 1;
  const Task* td = static_cast<const Task*>(ctx->ring.put(&t, sizeof(Task)));
  launch_elem(ctx, 3, PFEM_FP64, OP_APPLY, false, PFEM_SCATTER_OWNER, td, m->dev.work,
              m->n_blocks, m->bn, nullptr, nullptr);
}

}  // namespace

extern "C" pfem_status pfem_homogenize(pfem_mesh* m, const double* u0, const pfem_solve_opts* o,
                                       double* x_out, int ptr_is_device, double* eh,
                                       pfem_solve_report* reps) {
  std::vector<SlotRun> s(6);
  try {
    require(m != nullptr && o != nullptr && x_out != nullptr && eh != nullptr,
            PFEM_E_INVALID_ARG, "NULL argument");
    check_solve_opts(*o);
    require(m->finalized, PFEM_E_STATE, "mesh not finalized");
    require(m->uploaded && m->ctx != nullptr, PFEM_E_STATE, "mesh has no device context");
    require(m->dim == 3 && m->model == PFEM_LIN_3D, PFEM_E_INVALID_ARG,
            "homogenisation needs a 3D linear-elastic mesh");
    require(!m->pairs.empty(), PFEM_E_INVALID_ARG,
            "homogenisation needs periodic node pairs (pfem_mesh_set_periodic)");
    require(m->cell_volume > 0, PFEM_E_INVALID_MESH, "cell has no volume");
    Ctx* ctx = m->ctx;
    PFEM_HIP(hipSetDevice(ctx->device));
    const int64_t nd = m->n_dof();
    DevBufs buf;
    double* X0 = buf.get(6 * nd);
    double* F = buf.get(6 * nd);
    double* T = buf.get(6 * nd);
    double* KT = buf.get(6 * nd);
    double* part = buf.get((size_t)36 * gram6_parts(nd));
    double* out = buf.get(36);
    double* stage = (u0 != nullptr || !ptr_is_device) ? buf.get(nd) : nullptr;
    double* u0i = u0 != nullptr ? buf.get(6 * nd) : nullptr;
    // affine fields and the loads of the uniform stresses
    launch_affine6(ctx, m->dev.X, m->n_nodes, X0);
    for (int k = 0; k < 6; ++k) apply_elements(ctx, m, X0 + k * nd, F + k * nd);
    // warm starts of the fluctuations, caller order -> internal
    if (u0 != nullptr) {
      for (int k = 0; k < 6; ++k) {
        const double* src = u0 + k * nd;
        if (!ptr_is_device) {
          PFEM_HIP(hipMemcpyAsync(stage, src, nd * 8, hipMemcpyHostToDevice, ctx->stream));
          src = stage;
        }
        launch_permute(ctx, PFEM_FP64, 3, m->dev.perm, m->n_nodes, true, src, u0i + k * nd);
        if (!ptr_is_device) PFEM_HIP(hipStreamSynchronize(ctx->stream));   // stage reused
      }
    }
    // the six cell problems as six slots of the engine
    std::vector<SlotRun*> live;
    for (int k = 0; k < 6; ++k) {
      slot_alloc(&s[k], m, *o, 1);
      s[k].id = k;
      s[k].fext = F + k * nd;
      slot_begin(ctx, &s[k], u0 != nullptr ? u0i + k * nd : nullptr);
      live.push_back(&s[k]);
    }
    int64_t launches = 0;
    while (engine_tick(ctx, live, &launches) > 0) {
    }
    // E^H from the total fields T = X^0 - X^v
    for (int k = 0; k < 6; ++k) {
      launch_axpy_state(ctx, PFEM_FP64, m->md, T + k * nd, X0 + k * nd, s[k].st->x64, -1.0,
                        false, 0.0);
      apply_elements(ctx, m, T + k * nd, KT + k * nd);
    }
    launch_gram6(ctx, T, KT, nd, part, out, 1.0 / m->cell_volume);
    PFEM_HIP(hipMemcpyAsync(eh, out, 36 * 8, hipMemcpyDeviceToHost, ctx->stream));
    // fluctuations in the caller's order
    for (int k = 0; k < 6; ++k) {
      double* dst = ptr_is_device ? x_out + k * nd : stage;
      launch_permute(ctx, PFEM_FP64, 3, m->dev.perm, m->n_nodes, false, s[k].st->x64, dst);
      if (!ptr_is_device) {
        PFEM_HIP(hipMemcpyAsync(x_out + k * nd, stage, nd * 8, hipMemcpyDeviceToHost,
                                ctx->stream));
        PFEM_HIP(hipStreamSynchronize(ctx->stream));
      }
    }
    PFEM_HIP(hipStreamSynchronize(ctx->stream));
    pfem_status st = PFEM_OK;
    for (int k = 0; k < 6; ++k) {
      s[k].rep.status = s[k].status;
      if (reps) reps[k] = s[k].rep;
      if (s[k].status < 0 && (st >= 0 || s[k].status < st)) st = s[k].status;
      else if (st >= 0 && s[k].status == PFEM_NOT_CONVERGED) st = PFEM_NOT_CONVERGED;
    }
    for (int k = 0; k < 6; ++k) slot_free(&s[k]);
    set_error(st < 0 ? "a cell problem failed (see the reports)" : "");
    return st;
  } catch (const pfem::Error& e) {
    for (auto& r : s) slot_free(&r);
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    for (auto& r : s) slot_free(&r);
    set_error("host out of memory");
    return PFEM_E_OOM;
  } catch (const std::exception& e) {
    for (auto& r : s) slot_free(&r);
    set_error(e.what());
    return PFEM_E_INVALID_ARG;
  }
}
