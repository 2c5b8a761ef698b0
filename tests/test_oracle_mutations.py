"""The oracle's pins catch plausible mistakes (CPU).

Each case plants one mistake in the oracle (in memory, through monkeypatch)
and calls the pins that should expose it; at least one of them must fail.
A pin suite that still passed with a dropped factor, a transposed operand
or a flipped sign would not fix the oracle.
"""
import numpy as np
import pytest

from oracle import fe, prep, solve
from tests import test_oracle_pins as pins

_orig_grad = fe.shape_gradients
_orig_inv = fe.nh_invariants
_orig_lame = fe.lame_parameters
_orig_bisect = prep.bisect_blocks
_orig_energy_change = solve._energy_change


def _vol_without_factorial(coords, conn):
    G, vol = _orig_grad(coords, conn)
    return G, vol * (2.0 if G.shape[2] == 2 else 6.0)


def _grad_n0_sign(coords, conn):
    G, vol = _orig_grad(coords, conn)
    G = G.copy()
    G[:, 0, :] = -G[:, 0, :]
    return G, vol


def _piola_with_finv(H, mu, lam):
    d = H.shape[1]
    Fi = np.linalg.inv(np.eye(d) + H)            # F^-1 where F^-T belongs
    j, _, _ = fe.nh_invariants(H)
    return (mu[:, None, None] * (H + np.einsum("eik,ejk->eij", Fi, H))
            + (lam * np.log1p(j))[:, None, None] * Fi)


def _tangent(H, mu, lam, lam_term, sign):
    d = H.shape[1]
    Fi = np.linalg.inv(np.eye(d) + H)
    j, _, _ = fe.nh_invariants(H)
    lnJ = np.log1p(j)
    I = np.eye(d)
    return (mu[:, None, None, None, None] * np.einsum("ik,JL->iJkL", I, I)[None]
            + lam[:, None, None, None, None] * np.einsum(lam_term, Fi, Fi)
            + (mu + sign * lam * lnJ)[:, None, None, None, None]
            * np.einsum("eLi,eJk->eiJkL", Fi, Fi))


def _tangent_sign(H, mu, lam):
    return _tangent(H, mu, lam, "eJi,eLk->eiJkL", +1.0)


def _tangent_transposed(H, mu, lam):
    return _tangent(H, mu, lam, "eiJ,ekL->eiJkL", -1.0)


def _j_without_det(H):
    j, tr, detH = _orig_inv(H)
    return (j - detH if H.shape[1] == 3 else j), tr, detH


def _lame_swapped(model, kind, p0, p1):
    mu, lam = _orig_lame(model, kind, p0, p1)
    return lam, mu


def _stress_mu_not_2mu(H, mu, lam):
    eps = 0.5 * (H + np.transpose(H, (0, 2, 1)))
    tr = np.trace(eps, axis1=1, axis2=2)
    return mu[:, None, None] * eps + (lam * tr)[:, None, None] * np.eye(H.shape[1])


def _rcm_not_reversed(conn, n):
    order, _ = prep.cuthill_mckee(conn, n)
    new_id = np.empty(n, dtype=np.int32)
    new_id[np.array(order)] = np.arange(n, dtype=np.int32)
    return new_id


def _element_order_by_largest(conn, new_id):
    nc = np.asarray(new_id, dtype=np.int64)[np.asarray(conn, dtype=np.int64)]
    srt = -np.sort(-nc, axis=1)
    keys = [np.arange(conn.shape[0])] + [srt[:, c] for c in range(srt.shape[1] - 1, -1, -1)]
    return np.lexsort(keys).astype(np.int32)


def _colour_increasing_priority(sorted_conn, n_nodes):
    sc = np.asarray(sorted_conn, dtype=np.int64)
    k = np.arange(sc.shape[0], dtype=np.int64)
    order = np.lexsort((k, prep.fmix32(k ^ 0x9E3779B9).astype(np.int64)))
    n2e = [[] for _ in range(n_nodes)]
    for e, row in enumerate(sc.tolist()):
        for n in row:
            n2e[n].append(e)
    col = [-1] * sc.shape[0]
    for e in order.tolist():
        used = {col[f] for n in sc[e] for f in n2e[n] if col[f] >= 0}
        c = 0
        while c in used:
            c += 1
        col[e] = c
    return np.array(col, dtype=np.int32)


def _bisect_blocks_reversed(nodes, coords, pos, bn):
    return _orig_bisect(nodes, coords, pos, bn)[::-1]


def _pcg_beta_inverted(A, b, x0=None, tol=1e-10, max_iter=None, diag=None):
    n = b.shape[0]
    max_iter = max_iter or 10 * n
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    Minv = 1.0 / A.diagonal()
    bn = np.linalg.norm(b)
    r = b - A @ x
    z = Minv * r
    p = z.copy()
    rz = r @ z
    hist = [np.linalg.norm(r) / bn]
    for k in range(1, max_iter + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        hist.append(np.linalg.norm(r) / bn)
        if hist[-1] <= tol:
            return x, hist, k, 0
        z = Minv * r
        rz_new = r @ z
        p = z + (rz / rz_new) * p          # beta inverted
        rz = rz_new
    return x, hist, max_iter, 1


def _energy_change_flipped(m, psi0, u, ut):
    de, size = _orig_energy_change(m, psi0, u, ut)
    return -de, size


CASES = {
    "element measure without 1/d!": (
        fe, "shape_gradients", _vol_without_factorial,
        [(pins.test_closed_form_bar_2d, ("lin_plane_strain",)),
         (pins.test_closed_form_bar_3d, ())]),
    "sign of grad N_0": (
        fe, "shape_gradients", _grad_n0_sign,
        [(pins.test_patch_dirichlet_2d, ("lin_plane_stress",)),
         (pins.test_patch_dirichlet_3d, ())]),
    "Piola stress with F^-1 for F^-T": (
        fe, "nh_piola", _piola_with_finv,
        [(pins.test_nh_finite_rotation, ("nh_plane_strain",)),
         (pins.test_gradient_and_hvp_finite_differences, ("nh_3d",))]),
    "sign of the (mu - lambda ln J) tangent term": (
        fe, "nh_tangent_moduli", _tangent_sign,
        [(pins.test_gradient_and_hvp_finite_differences, ("nh_plane_strain",)),
         (pins.test_gradient_and_hvp_finite_differences, ("nh_3d",))]),
    "transposed lambda tangent term": (
        fe, "nh_tangent_moduli", _tangent_transposed,
        [(pins.test_gradient_and_hvp_finite_differences, ("nh_plane_strain",)),
         (pins.test_gradient_and_hvp_finite_differences, ("nh_3d",))]),
    "3D J - 1 without det H": (
        fe, "nh_invariants", _j_without_det,
        [(pins.test_nh_rearranged_energy_matches_literal, ()),
         (pins.test_nh_homogeneous_uniaxial_stretch, ())]),
    "mu and lambda swapped": (
        fe, "lame_parameters", _lame_swapped,
        [(pins.test_closed_form_bar_2d, ("lin_plane_strain",)),
         (pins.test_nh_homogeneous_uniaxial_stretch, ())]),
    "mu eps for 2 mu eps": (
        fe, "linear_stress", _stress_mu_not_2mu,
        [(pins.test_nh_reduces_to_linear, ("nh_3d", "lin_3d")),
         (pins.test_energy_quadratic_form_and_minimum, ())]),
    "Cuthill-McKee order not reversed": (
        prep, "rcm", _rcm_not_reversed,
        [(pins.test_rcm_hand_example, ()), (pins.test_rcm_two_components_and_ties, ())]),
    "elements sorted by their largest node": (
        prep, "element_order", _element_order_by_largest,
        [(pins.test_preprocessing_invariants, ())]),
    "colouring in increasing priority": (
        prep, "colour_elements", _colour_increasing_priority,
        [(pins.test_preprocessing_invariants, ())]),
    "bisection blocks in reverse order": (
        prep, "bisect_blocks", _bisect_blocks_reversed,
        [(pins.test_bisect_blocks_hand_example, ()),
         (pins.test_block_numbering_hand_example, ())]),
    "CG beta inverted": (
        solve, "pcg", _pcg_beta_inverted,
        [(pins.test_pcg_matches_direct_c1, ()), (pins.test_pcg_warm_start_saves_iterations, ())]),
    "line search with the energy change negated": (
        solve, "_energy_change", _energy_change_flipped,
        [(pins.test_nh_homogeneous_uniaxial_stretch, ()),
         (pins.test_newton_load_steps_and_warm_start, ())]),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_pins_catch_planted_mistake(monkeypatch, case):
    module, attr, wrong, checks = CASES[case]
    monkeypatch.setattr(module, attr, wrong)
    failed = []
    for pin, args in checks:
        try:
            pin(*args)
        except AssertionError:          # only a failed check counts, not a broken call
            failed.append(pin.__name__)
    assert failed, f"no pin failed with the planted mistake: {case}"
