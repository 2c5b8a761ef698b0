"""Shared helpers for the GPU parity tests (oracle side + device side)."""
import numpy as np
import pytest

from oracle import fe


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel(a, b):
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - b) / (nb if nb > 0 else 1.0)


def bound_rel(y, y_ref, Kabs_vabs, label=None):
    """|y - y_ref| / | |K| |v| |: the cancellation-aware kernel error.

    With a label, the measured error is printed together with its worst row,
    max_i |y_i - y_ref,i| / (|K| |v|)_i over rows with a non-zero bound."""
    d = np.abs(np.asarray(y) - y_ref)
    b = np.abs(np.asarray(Kabs_vabs))
    e = np.linalg.norm(d) / np.linalg.norm(b)
    if label is not None:
        nz = b > 0
        row = float((d[nz] / b[nz]).max()) if nz.any() else 0.0
        print(f"[err] {label}: norm {e:.2e} worst row {row:.2e}", flush=True)
    return e


def assert_bound(y, y_ref, Kabs_vabs, tol, label):
    """The cancellation-aware bound both norm-wise and row by row:
    |y - y_ref| <= tol | |K| |v| | and |y_i - y_ref,i| <= tol (|K| |v|)_i."""
    e = bound_rel(y, y_ref, Kabs_vabs, label)
    r = row_rel(y, y_ref, Kabs_vabs)
    assert e <= tol and r <= tol, (label, e, r, tol)


def row_rel(y, y_ref, Kabs_vabs):
    """Worst row of the bound: max_i |y_i - y_ref,i| / (|K| |v|)_i."""
    d = np.abs(np.asarray(y) - y_ref)
    b = np.abs(np.asarray(Kabs_vabs))
    nz = b > 0
    return float((d[nz] / b[nz]).max()) if nz.any() else 0.0


def compressed_field(prob, j_min, seed=0, noise_strain=0.01):
    """A displacement whose deformation compresses a Gaussian patch
    (width 0.25) around the domain centre to J = j_min at its centre, plus a
    smooth 1% strain field: u = -a w(X) (X - c) with (1 - a)^d = j_min and
    w the Gaussian.  F = (1 - a w) I + a w (X - c)(X - c)^T / 0.25^2 has
    positive eigenvalues for a < 1, so every element stays admissible and
    J ranges from 1 down to about j_min."""
    X = np.asarray(prob.coords, dtype=np.float64)
    c = 0.5 * (X.min(axis=0) + X.max(axis=0))
    a = 1.0 - j_min ** (1.0 / prob.dim)
    r = X - c
    w = np.exp(-np.einsum("ni,ni->n", r, r) / (2 * 0.25 ** 2))
    u = (-a * w[:, None] * r).reshape(-1)
    return u + smooth_field(prob, seed, noise_strain)


def smooth_field(prob, seed, strain):
    """A smooth displacement (RFF, length 0.2) scaled to max element strain."""
    from synth.fields import rff_field
    m = fe.Model(prob)
    g = rff_field(prob.coords, seed, 0.2, 64, n_comp=prob.dim).reshape(-1)
    g *= strain / np.abs(m.H(g)).max()
    return g


def sample_rows(prob, nodes):
    """Sub-problem holding only the elements incident to `nodes`: its
    assembled rows at those nodes equal the full problem's rows."""
    import copy
    conn = np.asarray(prob.conn)
    sel = np.nonzero(np.isin(conn, nodes).any(axis=1))[0]
    sub = copy.copy(prob)
    sub.conn = conn[sel]
    sub.p0 = np.asarray(prob.p0)[sel]
    sub.p1 = np.asarray(prob.p1)[sel]
    sub.neu_facets = np.zeros((0, prob.dim), np.int32)
    sub.neu_traction = np.zeros((0, prob.dim))
    return sub
