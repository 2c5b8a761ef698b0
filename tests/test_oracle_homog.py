"""Pins of the homogenisation oracle (CPU).

The oracle (App. D) is fixed by results it does not compute itself:
* a fully solid isotropic cell: the fluctuation vanishes in the limit of
  stiff periodic springs, so E^H tends to eps0 : C : eps0 (the tensor
  contractions of the unit strains), with an error that falls in
  proportion to 1 / k, from below (springs relax the periodic constraint,
  so no load case can store more energy than in the limit);
* a laminate of layers normal to z: piecewise-uniform layer strains with
  continuous tractions solve the cell problem exactly (P1 represents them
  when the layers follow the element faces), so E^H equals the laminate
  formula, computed here from the layer equations alone;
* TPMS cells: E^H is symmetric positive definite and below the Voigt
  bound phi C (volume fraction times the solid's tensor) as a quadratic
  form, and the six fluctuations vanish at the pinned node and are
  periodic up to the spring stretch;
* the element formula of E^H equals the quadratic form (X^0 - X^v).K.(X^0 -
  X^v) / |Omega| of the assembled stiffness.
Each planted mistake (a shear unit strain with one entry, springs of the
wrong sign, the cell volume of the solid only, the load of a transposed
stress) fails at least one pin.
"""
import numpy as np
import pytest

from oracle import homog
from synth import tpms


def _iso_C(E, nu):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    I = np.eye(3)
    return (lam * np.einsum("ij,kl->ijkl", I, I)
            + mu * (np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I)))


# the six unit strain tensors as printed in App. D (unit-strain equation),
# typed in independently of the oracle
PRINTED_E0 = np.array([
    [[1, 0, 0], [0, 0, 0], [0, 0, 0]],
    [[0, 0, 0], [0, 1, 0], [0, 0, 0]],
    [[0, 0, 0], [0, 0, 0], [0, 0, 1]],
    [[0, 1, 0], [1, 0, 0], [0, 0, 0]],
    [[0, 0, 1], [0, 0, 0], [1, 0, 0]],
    [[0, 0, 0], [0, 0, 1], [0, 1, 0]]], dtype=float)


def _contract(C):
    return np.einsum("aij,ijkl,bkl->ab", PRINTED_E0, C, PRINTED_E0)


def laminate_EH(f, E, nu):
    """E^H of a laminate normal to e3 from the layer equations: layer strain
    eps_i = eps0 + sym(c_i x n), tractions C_i:eps_i n equal in every layer,
    sum f_i c_i = 0; E^H = sum f_i eps_i^(IJ) : C_i : eps_i^(KL)."""
    n = np.array([0.0, 0.0, 1.0])
    Cs = [_iso_C(e, v) for e, v in zip(E, nu)]
    Ainv = [np.linalg.inv(np.einsum("j,ijkl,l->ik", n, C, n)) for C in Cs]
    S = np.linalg.inv(sum(fi * Ai for fi, Ai in zip(f, Ainv)))
    E0 = PRINTED_E0
    eps = np.zeros((len(f), 6, 3, 3))
    for k in range(6):
        tc = [np.einsum("ijkl,kl,j->i", C, E0[k], n) for C in Cs]   # C_i eps0 n
        t = S @ sum(fi * Ai @ ti for fi, Ai, ti in zip(f, Ainv, tc))
        for i in range(len(f)):
            c = Ainv[i] @ (t - tc[i])
            eps[i, k] = E0[k] + 0.5 * (np.outer(c, n) + np.outer(n, c))
    return sum(fi * np.einsum("aij,ijkl,bkl->ab", eps[i], Cs[i], eps[i])
               for i, fi in enumerate(f))


def pin_solid_cube():
    E, nu = 1.0, 0.3
    exact = _contract(_iso_C(E, nu))
    errs = []
    for keh in (1e3, 1e5):
        cell = tpms.cell_from_mask(np.ones((4, 4, 4), bool), E, nu, penalty_eh=keh)
        EH = homog.homogenized_tensor(cell, homog.fluctuations(cell))
        errs.append(np.abs(EH - exact).max() / np.abs(exact).max())
        # springs relax the periodic constraint: the energy of every load
        # case can only fall, so exact - E^H is positive semidefinite
        assert np.linalg.eigvalsh(exact - EH).min() >= -1e-12 * np.abs(exact).max()
    assert errs[0] < 1e-2 and errs[1] < 1e-4, errs
    assert 50 < errs[0] / errs[1] < 200, errs   # the penalty error scales as 1 / k


def pin_laminate():
    n = 6
    layers = [0, 0, 1, 1, 1, 0]
    E, nu = [1.0, 0.1], [0.3, 0.2]
    cell = tpms.laminate_cell(n, layers, E, nu, penalty_eh=1e7)
    EH = homog.homogenized_tensor(cell, homog.fluctuations(cell))
    f = [layers.count(0) / n, layers.count(1) / n]
    ref = laminate_EH(f, E, nu)
    assert np.abs(EH - ref).max() <= 1e-5 * np.abs(ref).max(), (EH, ref)


def pin_tpms_bounds():
    cell = tpms.tpms_cell(7, n=12, kind="gyroid", network="solid", vf=0.45, nu=0.3)
    X = homog.fluctuations(cell)
    EH = homog.homogenized_tensor(cell, X)
    assert np.allclose(EH, EH.T, rtol=1e-10, atol=1e-14)
    assert np.linalg.eigvalsh(EH).min() > 0
    phi = cell.meta["vf"]
    voigt = phi * _contract(_iso_C(1.0, 0.3))
    assert np.linalg.eigvalsh(voigt - EH).min() > 0     # E^H < phi C
    assert np.abs(X[:, 3 * cell.pin:3 * cell.pin + 3]).max() == 0.0
    # periodic up to the stretch of the springs, which carry the traction
    a, b = cell.pairs[:, 0], cell.pairs[:, 1]
    jump = np.abs(X.reshape(6, -1, 3)[:, a] - X.reshape(6, -1, 3)[:, b]).max()
    assert jump < 1e-2 * np.abs(X).max()


def pin_quadratic_form():
    cell = tpms.tpms_cell(8, n=8, kind="diamond", network="sheet", vf=0.5, nu=0.25)
    X = homog.fluctuations(cell)
    EH = homog.homogenized_tensor(cell, X)
    K = homog.cell_model(cell).assemble()
    T = homog.affine_fields(cell) - X
    Q = T @ (K @ T.T) / homog.cell_volume(cell)
    assert np.abs(Q - EH).max() <= 1e-10 * np.abs(EH).max()


def pin_unit_strains_as_printed():
    assert np.array_equal(homog.unit_strains(), PRINTED_E0)


PINS = [pin_unit_strains_as_printed, pin_solid_cube, pin_laminate, pin_tpms_bounds,
        pin_quadratic_form]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


def test_tpms_generator():
    """Volume fraction met to within a voxel layer, one periodic component,
    pairs on opposite faces with the same in-face lattice position."""
    for seed in range(4):
        c = tpms.tpms_cell(seed, n=16)
        assert abs(c.meta["vf"] - c.meta["vf_target"]) < 0.05
        P = c.coords[c.pairs[:, 0]]
        Q = c.coords[c.pairs[:, 1]]
        d = np.abs(Q - P)
        assert np.all(np.isclose(d, 1.0).sum(axis=1) == 1)
        assert np.all((np.isclose(d, 1.0) | np.isclose(d, 0.0)).all(axis=1))


# ------------------------------------------------------------ planted mistakes
def _one_entry_shear():
    E0 = np.zeros((6, 3, 3))
    for k, (p, q) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        E0[k, p, q] = 1.0
    return E0


def _negative_springs(cell):
    return -_orig_penalty(cell)


def _solid_volume(cell):
    m = homog.cell_model(cell)
    return float(m.vol.sum())


def _transposed_load(m):
    out = _orig_load(m)
    return out[[0, 1, 2, 3, 5, 4]]


_orig_penalty = homog.penalty_matrix
_orig_load = homog.load_vectors

MUTANTS = {
    "one_entry_shear": ("unit_strains", _one_entry_shear),
    "negative_springs": ("penalty_matrix", _negative_springs),
    "solid_volume": ("cell_volume", _solid_volume),
    "swapped_shear_loads": ("load_vectors", _transposed_load),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(monkeypatch, name):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(homog, attr, fn)
    failed = 0
    for pin in PINS:
        try:
            pin()
        except (AssertionError, RuntimeError, ValueError, np.linalg.LinAlgError):
            failed += 1
    assert failed > 0, name
