"""Periodic cells and homogenisation on the GPU against the oracle.

The periodic springs (virtual elements) inside K.v, force, energy and the
Jacobi diagonal, element-wise against the oracle's K + P; the six cell
problems and E^H of pfem_homogenize against the oracle's direct solves and
element formula (App. D), from zero and from warm starts, in both
precisions.
"""
import numpy as np
import pytest

from oracle import homog
from synth import tpms
from tests.gpu_util import assert_bound, rel, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    from paper_2601_03086_amd import core
    c = core.Context(0)
    yield c
    c.close()


def _cell(n=10, seed=21, **kw):
    kw.setdefault("kind", "gyroid")
    kw.setdefault("network", "sheet")
    kw.setdefault("vf", 0.5)
    return tpms.tpms_cell(seed, n=n, **kw)


def _masked(A, free):
    D = np.zeros(A.shape[0])
    D[free] = 1.0
    import scipy.sparse as sp
    Dm = sp.diags(D)
    return (Dm @ A @ Dm).tocsr()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("mask", [0, 3])
def test_periodic_apply_matches_oracle(ctx, prec, mask):
    from paper_2601_03086_amd import core
    cell = _cell()
    m = core.Mesh.from_cell(ctx, cell)
    assert m.info["n_blocks"] > 1
    A = homog.operator(cell)
    if mask:
        A = _masked(A, homog.cell_model(cell).free_dofs)
    v = np.random.default_rng(3).normal(size=cell.n_dof)
    y = m.apply_K(v, prec=prec, mask=mask).double().cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert_bound(y, A @ v, abs(A) @ abs(v), tol, f"periodic K.v {prec} mask {mask}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_periodic_force_energy_diag(ctx, prec):
    from paper_2601_03086_amd import core
    cell = _cell(seed=22, kind="diamond", network="solid", vf=0.4)
    m = core.Mesh.from_cell(ctx, cell)
    A = homog.operator(cell)
    u = np.random.default_rng(4).normal(size=cell.n_dof) * 1e-2
    g = m.force(u, prec=prec).double().cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert_bound(g, A @ u, abs(A) @ abs(u), tol, f"periodic force {prec}")
    e = m.energy(u, prec=prec).item()
    e_ref = 0.5 * u @ (A @ u)
    assert abs(e - e_ref) <= (1e-12 if prec == "fp64" else 1e-5) * abs(e_ref)
    d = m.diag(prec=prec).double().cpu().numpy()
    dref = A.diagonal().copy()
    om = homog.cell_model(cell)
    dref[om.dir_dofs] = 1.0
    assert rel(d, dref) <= (1e-13 if prec == "fp64" else 1e-6)


def test_homogenize_fp64_matches_oracle(ctx):
    from paper_2601_03086_amd import core
    cell = _cell(n=12, seed=23)
    m = core.Mesh.from_cell(ctx, cell)
    X, EH, reps = core.homogenize(m, tol=1e-12, prec="fp64")
    Xo = homog.fluctuations(cell)
    EHo = homog.homogenized_tensor(cell, Xo)
    ex = max(rel(X[k], Xo[k]) for k in range(6))
    ee = np.abs(EH - EHo).max() / np.abs(EHo).max()
    print(f"[err] homogenize fp64: fluctuations {ex:.2e} E^H {ee:.2e}; K.v "
          f"{[r['kv_count'] for r in reps]}", flush=True)
    assert all(r["status"] == 0 for r in reps)
    assert ex <= 1e-7 and ee <= 1e-10
    assert np.all(X[:, 3 * cell.pin:3 * cell.pin + 3] == 0.0)


def test_homogenize_fp32_mode_and_warm_start(ctx):
    """FP32 mode (FP32 element kernels and Krylov vectors, FP64 refinement)
    to 1e-9, from zero and from the oracle's fluctuations plus 1% smooth
    noise (the network's prediction stand-in): the same tensor, fewer
    products from the warm start."""
    from paper_2601_03086_amd import core
    from synth.fields import rff_field
    cell = _cell(n=12, seed=24, kind="fks", network="solid", vf=0.45)
    m = core.Mesh.from_cell(ctx, cell)
    Xo = homog.fluctuations(cell)
    EHo = homog.homogenized_tensor(cell, Xo)
    X0, EH0, r0 = core.homogenize(m, tol=1e-9, prec="fp32")
    noise = np.stack([rff_field(cell.coords, 900 + k, 0.2, 64, n_comp=3).reshape(-1)
                      for k in range(6)])
    noise[:, 3 * cell.pin:3 * cell.pin + 3] = 0.0
    scale = 0.01 * np.linalg.norm(Xo, axis=1) / np.linalg.norm(noise, axis=1)
    u0 = Xo + scale[:, None] * noise
    X1, EH1, r1 = core.homogenize(m, u0=u0, tol=1e-9, prec="fp32")
    for X, EH, reps in ((X0, EH0, r0), (X1, EH1, r1)):
        assert all(r["status"] == 0 and r["rel_residual_final"] <= 1e-9 for r in reps)
        assert max(rel(X[k], Xo[k]) for k in range(6)) <= 1e-5
        assert np.abs(EH - EHo).max() <= 1e-7 * np.abs(EHo).max()
    kz = sum(r["kv_count"] for r in r0)
    kw = sum(r["kv_count"] for r in r1)
    print(f"[homog] K.v zero start {kz}, warm start {kw}", flush=True)
    assert kw < kz


def test_homogenize_device_io_and_refusals(ctx):
    from paper_2601_03086_amd import _lib as L
    from paper_2601_03086_amd import core
    cell = _cell(n=8, seed=25)
    m = core.Mesh.from_cell(ctx, cell)
    Xh, EHh, _ = core.homogenize(m, tol=1e-11, prec="fp64")
    Xd, EHd, _ = core.homogenize(m, tol=1e-11, prec="fp64", device_io=True)
    # two solves to 1e-11 whose LDS sums may differ in the last bits: the
    # same fields up to the condition number times the tolerance
    assert np.abs(Xd.cpu().numpy() - Xh).max() <= 1e-8 * np.abs(Xh).max()
    assert np.abs(EHd - EHh).max() <= 1e-10 * np.abs(EHh).max()
    with pytest.raises(L.PfemError) as ei:    # the fused PCG has no springs
        core.homogenize(m, tol=1e-8, prec="fp32", krylov="fused")
    assert ei.value.status == L.PFEM_E_INVALID_ARG
    with pytest.raises(L.PfemError) as ei:    # nor the coloured scatter
        m.apply_K(np.zeros(cell.n_dof), prec="fp64", scatter="colored")
    assert ei.value.status == L.PFEM_E_INVALID_ARG


def test_homogenize_one_visit_and_per_task_paths(ctx):
    """Small owner blocks run the six right-hand sides in one element visit,
    blocks too large for its LDS accumulators run them as six tasks of one
    launch; both give the oracle's tensor."""
    from paper_2601_03086_amd import core
    cell = _cell(n=12, seed=26, kind="diamond", network="solid", vf=0.5)
    Xo = homog.fluctuations(cell)
    EHo = homog.homogenized_tensor(cell, Xo)
    for bn in (64, 1024):
        m = core.Mesh.from_cell(ctx, cell, block_nodes=bn)
        X, EH, reps = core.homogenize(m, tol=1e-12, prec="fp64")
        ee = np.abs(EH - EHo).max() / np.abs(EHo).max()
        print(f"[err] homogenize block {m.info['block_nodes']}: E^H {ee:.2e}", flush=True)
        assert all(r["status"] == 0 for r in reps) and ee <= 1e-10
        assert max(rel(X[k], Xo[k]) for k in range(6)) <= 1e-7
