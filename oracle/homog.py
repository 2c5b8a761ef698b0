"""Numerical homogenisation of a periodic cell in float64 (oracle; test
infrastructure only: only tests/, the smoke check and the benchmark's CPU
leg use it).

App. D, in the paper's notation and order:
* six macroscopic unit strains eps0^(IJ), (IJ) = 11, 22, 33, 12, 13, 23
  (unit-strain equation): a one on the diagonal for the normal cases, ones
  at (p, q) and (q, p) for the shear cases;
* the fluctuation X^v(IJ) satisfies the weak form (weak-form equation)
  int eps(X*) : E : eps(X^v) = int eps(X*) : E : eps0 for every virtual
  fluctuation X*, i.e. K X^v = F^(IJ) with F^(IJ)_a = sum_e vol_e
  B_a^T (E : eps0^(IJ)) -- the element loads of a uniform stress;
* periodicity (PBC equation) is imposed as in PFEM by virtual elements:
  springs of stiffness k between paired nodes on opposite faces, whose
  strain energy 1/2 k |X_a - X_b|^2 joins the potential -- a penalty
  (reading: the paper gives no value for k; the cell carries it);
* the homogenised tensor (homogenised-elastic-matrix equation)
  E^H_(IJ)(KL) = 1/|Omega| int (eps0^(IJ) - eps^v(IJ)) : E : (eps0^(KL) -
  eps^v(KL)) dOmega over the solid elements, |Omega| the volume of the
  whole cell, voids included.
Readings: one node (the cell's pin) is held at zero fluctuation, which
removes the rigid translations that periodicity leaves free; the loss of
the homogenisation-loss equation is read as 1/2 X^v.(K + P) X^v -
F^(IJ).X^v (its printed second term lacks the fluctuation strain).
"""
import types

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fe import Model, linear_moduli

CASES = ("11", "22", "33", "12", "13", "23")


def unit_strains():
    """The six unit strain tensors eps0^(IJ) (App. D, unit-strain equation)."""
    out = np.zeros((6, 3, 3))
    for k, (p, q) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        out[k, p, q] = 1.0
        out[k, q, p] = 1.0
    return out


def cell_model(cell):
    """The oracle's element model of a cell (linear 3D elasticity, (E, nu)
    per element), with the pin as its only Dirichlet node."""
    prob = types.SimpleNamespace(
        model="lin_3d", param_kind="E_nu", dim=3, coords=cell.coords, conn=cell.conn,
        p0=cell.p0, p1=cell.p1, n_dof=3 * len(cell.coords),
        dir_nodes=np.full(3, cell.pin, np.int32), dir_comps=np.arange(3, dtype=np.int8),
        dir_values=np.zeros(3), neu_facets=np.zeros((0, 3), np.int32),
        neu_traction=np.zeros((0, 3)))
    return Model(prob)


def penalty_matrix(cell):
    """P with 1/2 x.P x = sum over pairs of 1/2 k |x_a - x_b|^2."""
    n = 3 * len(cell.coords)
    a = np.asarray(cell.pairs[:, 0], np.int64)
    b = np.asarray(cell.pairs[:, 1], np.int64)
    rows, cols, vals = [], [], []
    for i in range(3):
        ai, bi = 3 * a + i, 3 * b + i
        rows += [ai, bi, ai, bi]
        cols += [ai, bi, bi, ai]
        k = np.full(len(a), cell.penalty)
        vals += [k, k, -k, -k]
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def affine_fields(cell):
    """X^0(IJ) = eps0^(IJ) . X at every node (node-major), shape (6, n_dof)."""
    E0 = unit_strains()
    return np.einsum("kij,nj->kni", E0, cell.coords).reshape(6, -1)


def load_vectors(m):
    """F^(IJ) = sum_e vol_e B^T (E : eps0^(IJ)), shape (6, n_dof)."""
    C = linear_moduli(m.mu, m.lam, 3)
    out = np.zeros((6, m.n_dof))
    for k, e0 in enumerate(unit_strains()):
        sig = np.einsum("eijkl,kl->eij", C, e0)
        fe = m.vol[:, None, None] * np.einsum("eij,eaj->eai", sig, m.G)
        np.add.at(out[k], m.dofs.reshape(-1), fe.reshape(-1))
    return out


def fluctuations(cell):
    """X^v(IJ) for the six cases, shape (6, n_dof): (K + P) X^v = F^(IJ) on
    the DOFs other than the pin's, solved directly."""
    m = cell_model(cell)
    A = (m.assemble() + penalty_matrix(cell)).tocsr()
    fr = m.free_dofs
    lu = spla.splu(A[fr][:, fr].tocsc())
    F = load_vectors(m)
    X = np.zeros((6, m.n_dof))
    for k in range(6):
        X[k, fr] = lu.solve(F[k, fr])
    return X


def cell_volume(cell):
    lo = cell.coords.min(axis=0)
    hi = cell.coords.max(axis=0)
    return float(np.prod(hi - lo))


def homogenized_tensor(cell, Xv):
    """E^H (6 x 6) from the fluctuations by the element formula of App. D."""
    m = cell_model(cell)
    C = linear_moduli(m.mu, m.lam, 3)
    E0 = unit_strains()
    eps = []
    for k in range(6):
        H = m.H(Xv[k])
        ev = 0.5 * (H + np.swapaxes(H, 1, 2))
        eps.append(E0[k][None] - ev)
    EH = np.zeros((6, 6))
    for i in range(6):
        s = np.einsum("eijkl,ekl->eij", C, eps[i])
        for j in range(6):
            EH[i, j] = np.sum(m.vol * np.einsum("eij,eij->e", s, eps[j]))
    return EH / cell_volume(cell)


def operator(cell):
    """K + P (the cell's periodic stiffness) as CSR, all DOFs."""
    m = cell_model(cell)
    return (m.assemble() + penalty_matrix(cell)).tocsr()
