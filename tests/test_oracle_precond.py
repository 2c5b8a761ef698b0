"""Pins of the two-level preconditioner oracle (CPU).

* The coarse space of an unconstrained mesh lies in the kernel of K (its
  modes are rigid motions: zero strain), in 2D and 3D.
* The coarse correction reproduces piecewise-rigid fields: for u = P c,
  P (P^T K P)^-1 P^T K u = u (it is the K-orthogonal projector onto P).
* M^-1 is symmetric positive definite.
* It does not depend on the basis that spans the coarse space (rotations
  about another point give the same M^-1).
* Preconditioned CG reaches the direct solution and needs far fewer
  iterations than Jacobi on a plate.
Planted mistakes (a rotation mode of the wrong sign, the Jacobi part left
out) each fail a pin.
"""
import functools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import fe, precond, solve
from tests import meshkit as mk


def _blocks(coords, size):
    """Aggregates of about `size` nodes: lexicographic cells of the box."""
    X = np.asarray(coords)
    lo, hi = X.min(axis=0), X.max(axis=0)
    n_per = max(1, int(round((len(X) / size) ** (1.0 / X.shape[1]))))
    cell = np.minimum(((X - lo) / (hi - lo + 1e-30) * n_per).astype(int), n_per - 1)
    key = np.zeros(len(X), dtype=np.int64)
    for i in range(X.shape[1]):
        key = key * n_per + cell[:, i]
    return np.unique(key, return_inverse=True)[1]


def _free_problem(dim):
    if dim == 2:
        p = synth.plate_problem(31, 32, 33, n_holes=2, target_tris=1500)
    else:
        p = synth.box_problem(34, 35, n_per_unit=3, n_voids=1, n_load_steps=1,
                              model="lin_3d")
    q = mk.make_problem("lin_3d" if dim == 3 else "lin_plane_strain", p.coords, p.conn,
                        E=1.0, nu=0.3)
    return q


def pin_rigid_kernel():
    for dim in (2, 3):
        q = _free_problem(dim)
        m = fe.Model(q)
        K = m.assemble()
        agg = np.zeros(q.n_nodes, dtype=np.int64)          # one aggregate: the body
        P = precond.coarse_basis(q.coords, agg, dim, np.ones(q.n_dof, bool))
        assert P.shape[1] == 3 * (dim - 1)
        assert np.abs(K @ P).max() <= 1e-10 * abs(K).max()


@functools.lru_cache(maxsize=1)
def _plate_base():
    p = synth.plate_problem(41, 42, 43, n_holes=3, target_tris=3000)
    m = fe.Model(p)
    Kff, Ff, uD = solve.reduced_system(m)
    agg = _blocks(p.coords, 50)
    return p, m, Kff, Ff, agg


def _plate():
    p, m, Kff, Ff, agg = _plate_base()
    M = precond.two_level(Kff, m.free_dofs, p.coords, agg, 2)
    return p, m, Kff, Ff, agg, M


def pin_projector():
    p, m, Kff, Ff, agg, M = _plate()
    c = np.random.default_rng(0).normal(size=M.P.shape[1])
    u = M.P @ c
    r = Kff @ u
    uc = M.P @ np.linalg.solve(M.Ac, M.P.T @ r)
    assert np.abs(uc - u).max() <= 1e-8 * np.abs(u).max()


def pin_spd():
    p, m, Kff, Ff, agg, M = _plate()
    rng = np.random.default_rng(1)
    x, y = rng.normal(size=(2, Kff.shape[0]))
    assert abs(x @ M(y) - y @ M(x)) <= 1e-10 * abs(x @ M(y))
    for _ in range(5):
        v = rng.normal(size=Kff.shape[0])
        assert v @ M(v) > 0
    # every direction gets at least the Jacobi part
    e = np.zeros(Kff.shape[0])
    e[17] = 1.0
    assert M(e)[17] >= 1.0 / Kff.diagonal()[17] * (1 - 1e-12)


def pin_basis_free():
    p, m, Kff, Ff, agg, M = _plate()
    free_mask = np.zeros(p.n_dof, bool)
    free_mask[m.free_dofs] = True
    # rotations about each aggregate's first node instead of its centroid
    shifted = np.asarray(p.coords, dtype=np.float64).copy()
    P2 = []
    for a in np.unique(agg):
        nodes = np.nonzero(agg == a)[0]
        R = precond.rigid_modes(shifted, nodes, 2)
        Y = shifted[nodes] - shifted[nodes[0]]
        R[:, 2] = np.stack([-Y[:, 1], Y[:, 0]], axis=1).reshape(-1)
        dofs = (nodes[:, None] * 2 + np.arange(2)).reshape(-1)
        R[~free_mask[dofs]] = 0.0
        for k in range(3):
            col = np.zeros(p.n_dof)
            col[dofs] = R[:, k]
            if np.any(col):
                P2.append(col)
    P2 = np.array(P2).T[m.free_dofs]
    r = np.random.default_rng(2).normal(size=Kff.shape[0])
    Ac2 = P2.T @ (Kff @ P2)
    z2 = r / Kff.diagonal() + P2 @ np.linalg.lstsq(Ac2, P2.T @ r, rcond=1e-12)[0]
    z = M(r)
    assert np.abs(z - z2).max() <= 1e-8 * np.abs(z).max()


def pin_pcg():
    p, m, Kff, Ff, agg, M = _plate()
    ud = spla.spsolve(Kff.tocsc(), Ff)
    x2, h2, k2, s2 = solve.pcg(Kff, Ff, None, 1e-10, precond=M)
    xj, hj, kj, sj = solve.pcg(Kff, Ff, None, 1e-10)
    assert s2 == 0 and sj == 0
    assert np.linalg.norm(x2 - ud) <= 1e-7 * np.linalg.norm(ud)
    assert k2 * 3 <= kj, (k2, kj)


PINS = [pin_rigid_kernel, pin_projector, pin_spd, pin_basis_free, pin_pcg]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


_orig_modes = precond.rigid_modes
_orig_two_level = precond.two_level


def _rotation_sign(coords, nodes, dim):
    R = _orig_modes(coords, nodes, dim).copy()
    if dim == 2:
        R[0::2, 2] = -R[0::2, 2]            # (y, x) instead of (-y, x)
    else:
        R[1::3, 3] = -R[1::3, 3]
    return R


def _no_jacobi(Kff, free_dofs, coords, aggregates, dim):
    M = _orig_two_level(Kff, free_dofs, coords, aggregates, dim)
    P, Ac = M.P, M.Ac

    def apply(r):
        return P @ np.linalg.solve(Ac, P.T @ r)

    apply.P, apply.Ac = P, Ac
    return apply


@pytest.mark.parametrize("name,attr,fn", [("rotation_sign", "rigid_modes", _rotation_sign),
                                          ("no_jacobi", "two_level", _no_jacobi)])
def test_planted_mistake_fails_a_pin(monkeypatch, name, attr, fn):
    monkeypatch.setattr(precond, attr, fn)
    failed = 0
    for pin in PINS:
        try:
            pin()
        except (AssertionError, np.linalg.LinAlgError, ValueError):
            failed += 1
    assert failed > 0, name
