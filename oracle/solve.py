"""Linear and nonlinear solves in float64 (oracle; test infrastructure only).

* Reduced linear system (App. B, K U = F with Dirichlet elimination):
  K_ff u_f = F_f with F_f = f_ext,f - K_fD u_D.
* Relative residual (App. B, L_rel = |K U - F| / |F|), measured on free DOFs.
* Jacobi-preconditioned CG (Saad, Iterative Methods for Sparse Linear
  Systems, Alg. 9.1).  The paper names CG and an unnamed preconditioner for
  its warm-start solves (Sec. 'Three-dimensional solid mechanics
  homogenization'); the diagonal (Jacobi) preconditioner is the reading.
* Newton-Raphson with load steps (App. B): for each load step the Dirichlet
  values are scaled to n / N_f, then Newton iterations
  u <- u + s Delta with K_T(u) Delta = -r_f(u) until the relative residual
  is below tol.  A warm start skips the first N_f - 1 load steps.
  Readings (paper silent): load step n applies the fraction n / N_f of the
  whole load, prescribed displacements and tractions alike; the relative
  residual divides by the residual of the lifted state (free DOFs zero,
  load-step Dirichlet values, load-step tractions); the step
  length s follows Armijo backtracking on the total potential (factor 1/2,
  sufficient-decrease constant 1e-4, at most 20 halvings), rejecting any
  trial state with J <= 0; an energy change within the float64 rounding
  level of its summed terms (64 eps times their magnitudes) counts as
  inconclusive and the step is taken, because near convergence a Newton
  step lowers the energy by O(|r|^2), below what the sum resolves; each
  load step after the first starts from the previous converged state
  scaled to the new load fraction (a linear predictor: moving only the
  prescribed DOFs would stretch the element layer next to the loaded
  boundary by the whole increment).
"""
import numpy as np
import scipy.sparse.linalg as spla

from .fe import Model


def reduced_system(m: Model, u_dirichlet=None):
    """K_ff, F_f and the lifted vector for a linear model."""
    K = m.assemble()
    uD = m.lifted() if u_dirichlet is None else u_dirichlet
    f = m.f_ext - K @ uD
    fr = m.free_dofs
    return K[fr][:, fr].tocsr(), f[fr], uD


def relative_residual(Kff, Ff, uf):
    nf = np.linalg.norm(Ff)
    r = np.linalg.norm(Kff @ uf - Ff)
    return r / nf if nf > 0 else r


def pcg(A, b, x0=None, tol=1e-10, max_iter=None, diag=None, precond=None):
    """Jacobi-PCG with the true-residual confirmation described in the module.

    Stops when |r_k| / |b| <= tol and the recomputed residual b - A x also
    satisfies it; otherwise restarts from the true residual.  Returns
    (x, history, kv_count, status) with status 0 converged, 1 max-iter,
    -5 breakdown (p.Ap <= 0).  kv_count counts the products A p only.
    precond: a function r -> M^-1 r replacing the Jacobi preconditioner.
    """
    n = b.shape[0]
    if max_iter is None:
        max_iter = 10 * n
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    if precond is None:
        dinv = 1.0 / (A.diagonal() if diag is None else diag)

        def precond(v):
            return dinv * v
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros(n), [0.0], 0, 0
    r = b - A @ x
    hist = [np.linalg.norm(r) / bn]
    if hist[0] <= tol:
        return x, hist, 0, 0
    z = precond(r)
    p = z.copy()
    rz = r @ z
    k = 0
    while k < max_iter:
        q = A @ p
        k += 1
        pq = p @ q
        if not pq > 0.0:
            return x, hist, k, -5
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        rho = np.linalg.norm(r) / bn
        hist.append(rho)
        if rho <= tol:
            rt = b - A @ x
            if np.linalg.norm(rt) / bn <= tol:
                return x, hist, k, 0
            r = rt
            z = precond(r)
            p = z.copy()
            rz = r @ z
            continue
        z = precond(r)
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, hist, k, 1


def solve_linear(prob, u0=None, tol=1e-10, method="pcg", max_iter=None):
    """Full-length displacement of a linear problem and a report dict."""
    m = Model(prob)
    Kff, Ff, uD = reduced_system(m)
    fr = m.free_dofs
    if method == "direct":
        uf = spla.spsolve(Kff.tocsc(), Ff)
        hist, kv, st = [relative_residual(Kff, Ff, uf)], 0, 0
    else:
        x0 = None if u0 is None else np.asarray(u0, np.float64)[fr]
        uf, hist, kv, st = pcg(Kff, Ff, x0, tol, max_iter)
    u = uD.copy()
    u[fr] = uf
    return u, {"history": hist, "kv_count": kv, "status": st,
               "rel_residual": relative_residual(Kff, Ff, uf)}


def _residual_free(m, u):
    return m.gradient(u)[m.free_dofs]


def _energy_change(m, psi0, u, ut):
    """Pi(ut) - Pi(u) summed element by element, and the sum of the
    magnitudes of its terms (the scale of its rounding error).  +inf if an
    element of ut has J <= 0."""
    psit = m.energy_density(ut)
    if not np.all(np.isfinite(psit)):
        return np.inf, 0.0
    w = m.f_ext * (ut - u)
    de = float(np.sum(m.vol * (psit - psi0)) - np.sum(w))
    size = float(np.sum(m.vol * (np.abs(psi0) + np.abs(psit))) + np.sum(np.abs(w)))
    return de, size


def newton(prob, u0=None, tol=1e-8, n_load_steps=None, max_newton=50,
           linear_solver="direct", lin_tol=1e-12, armijo_c=1e-4,
           max_halvings=20):
    """Newton with load steps on Pi(u) = sum vol Psi - f_ext . u.

    Returns (u, report) where report['steps'] lists, per load step, the
    converged displacement (copy), Newton count and residual history.
    """
    m = Model(prob)
    f_full = m.f_ext.copy()
    nls = prob.n_load_steps if n_load_steps is None else n_load_steps
    fr = m.free_dofs
    if u0 is None:
        u = m.lifted(0.0)
        steps = range(1, nls + 1)
    else:
        u = np.array(u0, dtype=np.float64)
        steps = [nls]
    out = []
    status = 0
    prev = None
    for n in steps:
        scale = n / nls
        m.f_ext = scale * f_full
        if prev is not None:       # predictor: previous state scaled to this load
            u = u * (n / prev)
        u[m.dir_dofs] = scale * m.dir_vals
        prev = n
        den = np.linalg.norm(_residual_free(m, m.lifted(scale)))
        hist = []
        it = 0
        while True:
            r = _residual_free(m, u)
            rn = np.linalg.norm(r)
            rho = rn / den if den > 0 else rn
            hist.append(rho)
            if rho <= tol:
                break
            if it >= max_newton:
                status = 1
                break
            KT = m.assemble(u)[fr][:, fr].tocsc()
            if linear_solver == "direct":
                delta = spla.spsolve(KT, -r)
            else:
                delta, _, _, _ = pcg(KT.tocsr(), -r, None, lin_tol)
            psi0 = m.energy_density(u)
            slope = r @ delta
            s = 1.0
            ok = False
            for _ in range(max_halvings + 1):
                ut = u.copy()
                ut[fr] += s * delta
                de, size = _energy_change(m, psi0, u, ut)
                # Armijo; a change within the rounding level of the summed
                # terms is inconclusive and the step is taken (the residual
                # test then decides convergence)
                if np.isfinite(de) and (de <= armijo_c * s * slope
                                        or abs(de) <= 64 * np.finfo(float).eps * size):
                    ok = True
                    break
                s *= 0.5
            if not ok:
                status = -7
                break
            u = ut
            it += 1
        out.append({"load_step": n, "u": u.copy(), "newton_iters": it,
                    "history": hist})
        if status < 0:
            break
    m.f_ext = f_full
    return u, {"steps": out, "status": status}
