// Warm-started solves as device-resident state machines ("slots").
//
// Linear elasticity: Jacobi-PCG on the Dirichlet-reduced system.  In FP64
// mode the Krylov vectors are float64 and a converged recursive residual is
// confirmed by a float64 residual evaluation (restart if it fails).  In FP32
// mode the Krylov loop runs in float32 on the correction equation
// K d = r(x) and x (float64) is refined until the float64 residual meets
// the tolerance (mixed-precision iterative refinement).
//
// Neo-Hookean: Newton with load steps (App. B); each Newton step solves
// K_T(u) d = -g(u) inexactly with the same Jacobi-PCG (forcing term
// min(0.1, rho)), then an Armijo backtracking line search on the float64
// energy difference.  A warm start skips the first N_f - 1 load steps
// (App. B, warm-start bypass of the outer iteration).
//
// Every heavy step of every live slot is batched: one launch per kernel
// family per tick covers all slots that need it (continuous batching).
#pragma once

#include <functional>

#include <vector>

#include "mesh.h"

namespace pfem {

enum Action { A_NONE = 0, A_DEN, A_RESID, A_KRYLOV_START, A_KRYLOV, A_LS, A_DONE };

struct SlotRun {
  pfem_mesh* m = nullptr;
  SolveState* st = nullptr;
  Scalars* sc_host = nullptr;     // pinned mirror of st->sc
  pfem_solve_opts o{};
  pfem_solve_report rep{};
  int prec = PFEM_FP32;
  bool nl = false;
  bool warm = false;
  int n_steps = 1, step = 1;
  double den = 1.0, rho = 0.0, gnorm = 0.0, eta = 0.1;
  int newton_in_step = 0;
  bool minv_valid = false;
  bool first_resid = true;
  int action = A_NONE;
  int chunk = 16;
  double rho_chunk = 0.0;
  int k_chunk = 0;
  int k_before = 0;         // Krylov count when the current chunk started
  int hist_base = 0;        // history index of iteration 0 of the inner solve
  int64_t hist_len_host = 0;
  int64_t timing_key = -1;  // launch group of the current chunk
  int chunk_launched = 0;   // launches of that chunk
  double ls_s = 1.0, ls_slope = 0.0;
  int ls_tries = 0;
  int max_iter = 0;
  double rho_sweep = 0.0;   // linear: true residual at the start of the last sweep
  int stalled = 0;          // linear: sweeps in a row that did not halve it
  bool finished = false;
  pfem_status status = PFEM_OK;
  int64_t id = -1;
  const double* fext = nullptr;   // external force of this solve (nullptr: the mesh's)
  bool shares_elements = false;   // applied with earlier slots of one mesh in one visit
};

// Prepares slot state on the device: x64 <- initial guess (internal order,
// float64, already on the device) and the first action.  `u0_internal`
// may be null (zero start).
void slot_begin(Ctx* ctx, SlotRun* s, const double* u0_internal_dev);

// Runs one tick for every live slot.  Returns the number not finished.
// overlap (optional): host work to run after the tick's launches are
// enqueued and before the tick waits for them (work that may enqueue on
// the library stream only behind them).
int engine_tick(Ctx* ctx, std::vector<SlotRun*>& live, int64_t* launches,
                const std::function<void()>* overlap = nullptr);

// Allocates device and pinned state for a slot on mesh m.
// Argument checks of a solve's options (pfem_solve, pfem_server_submit):
// PFEM_E_INVALID_ARG for a tolerance that is not finite and positive, an
// unknown precision or Krylov formulation, or an inner reduction outside
// {0} U (0, 0.5].  A sweep whose inner target is not below its starting
// residual would end at iteration 0 and leave x unchanged, forever; 0.5
// keeps a factor 2 above the float32 rounding of that starting residual.
void check_solve_opts(const pfem_solve_opts& o);
// Refuses option / mesh combinations no solve path covers (PFEM_E_INVALID_ARG).
void check_solve_mesh(const pfem_solve_opts& o, const pfem_mesh* m);
void slot_alloc(SlotRun* s, pfem_mesh* m, const pfem_solve_opts& o, int64_t hist_cap);
void slot_free(SlotRun* s);

}  // namespace pfem
