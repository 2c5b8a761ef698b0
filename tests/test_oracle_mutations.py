"""The oracle's pins catch plausible mistakes (CPU).

Each case plants one mistake in the oracle (in memory, through monkeypatch)
and calls the pins that should expose it; at least one of them must fail.
A pin suite that still passed with a dropped factor, a transposed operand
or a flipped sign would not fix the oracle.
"""
import numpy as np
import pytest

from oracle import fe
from tests import test_oracle_pins as pins

_orig_grad = fe.shape_gradients
_orig_inv = fe.nh_invariants
_orig_lame = fe.lame_parameters


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


CASES = {
    "element measure without 1/d!": (
        "shape_gradients", _vol_without_factorial,
        [(pins.test_closed_form_bar_2d, ("lin_plane_strain",)),
         (pins.test_closed_form_bar_3d, ())]),
    "sign of grad N_0": (
        "shape_gradients", _grad_n0_sign,
        [(pins.test_patch_dirichlet_2d, ("lin_plane_stress",)),
         (pins.test_patch_dirichlet_3d, ())]),
    "Piola stress with F^-1 for F^-T": (
        "nh_piola", _piola_with_finv,
        [(pins.test_nh_finite_rotation, ("nh_plane_strain",)),
         (pins.test_gradient_and_hvp_finite_differences, ("nh_3d",))]),
    "sign of the (mu - lambda ln J) tangent term": (
        "nh_tangent_moduli", _tangent_sign,
        [(pins.test_gradient_and_hvp_finite_differences, ("nh_plane_strain",)),
         (pins.test_gradient_and_hvp_finite_differences, ("nh_3d",))]),
    "transposed lambda tangent term": (
        "nh_tangent_moduli", _tangent_transposed,
        [(pins.test_gradient_and_hvp_finite_differences, ("nh_plane_strain",)),
         (pins.test_gradient_and_hvp_finite_differences, ("nh_3d",))]),
    "3D J - 1 without det H": (
        "nh_invariants", _j_without_det,
        [(pins.test_nh_rearranged_energy_matches_literal, ()),
         (pins.test_nh_homogeneous_uniaxial_stretch, ())]),
    "mu and lambda swapped": (
        "lame_parameters", _lame_swapped,
        [(pins.test_closed_form_bar_2d, ("lin_plane_strain",)),
         (pins.test_nh_homogeneous_uniaxial_stretch, ())]),
    "mu eps for 2 mu eps": (
        "linear_stress", _stress_mu_not_2mu,
        [(pins.test_nh_reduces_to_linear, ("nh_3d", "lin_3d")),
         (pins.test_energy_quadratic_form_and_minimum, ())]),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_pins_catch_planted_mistake(monkeypatch, case):
    attr, wrong, checks = CASES[case]
    monkeypatch.setattr(fe, attr, wrong)
    failed = []
    for pin, args in checks:
        try:
            pin(*args)
        except AssertionError:          # only a failed check counts, not a broken call
            failed.append(pin.__name__)
    assert failed, f"no pin failed with the planted mistake: {case}"
