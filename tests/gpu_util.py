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


def bound_rel(y, y_ref, Kabs_vabs):
    """|y - y_ref| / | |K| |v| |: the cancellation-aware kernel error."""
    return np.linalg.norm(np.asarray(y) - y_ref) / np.linalg.norm(Kabs_vabs)


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
