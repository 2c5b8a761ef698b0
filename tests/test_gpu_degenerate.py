"""Degenerate inputs of the method through the C ABI: one-element meshes,
every DOF prescribed, a zero load, each against the FP64 oracle."""
import numpy as np
import pytest

from oracle import fe, solve as osolve
from tests import meshkit as mk
from tests.gpu_util import assert_bound, bound_rel, rel, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    from paper_2601_03086_amd import core
    c = core.Context(0)
    yield c
    c.close()


def _one_element(dim, model):
    if dim == 2:
        coords = np.array([[0.0, 0.0], [1.0, 0.1], [0.2, 0.9]])
        conn = np.array([[0, 1, 2]])
    else:
        coords = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1],
                           [0.1, 0.2, 1.1]])
        conn = np.array([[0, 1, 2, 3]])
    # node 0 clamped, node 1 pulled along x with its other components held,
    # in 3D node 2's z held too: no rigid rotation is left, not even a
    # finite one (holding only node 1's x lets a Neo-Hookean element reach
    # the pulled position by rotating, a zero-energy mechanism)
    if dim == 2:
        dn, dc, dv = [0, 0, 1, 1], [0, 1, 0, 1], [0.0, 0.0, 0.05, 0.0]
    else:
        dn, dc, dv = [0, 0, 0, 1, 1, 1, 2], [0, 1, 2, 0, 1, 2, 2], [0, 0, 0, 0.05, 0, 0, 0]
    return mk.make_problem(model, coords, conn, E=2.0, nu=0.25, dir_nodes=dn,
                           dir_comps=dc, dir_values=dv)


@pytest.mark.parametrize("dim,model", [(2, "lin_plane_strain"), (3, "lin_3d"),
                                       (2, "nh_plane_strain"), (3, "nh_3d")])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_one_element(ctx, dim, model, prec):
    """A mesh of one element: one owner block with one visit (every other
    thread idle), K.v / HVP and a solve against the oracle."""
    from paper_2601_03086_amd import core
    torch = torch_cuda()
    p = _one_element(dim, model)
    m = core.Mesh.from_problem(ctx, p)
    assert m.info["n_blocks"] == 1
    om = fe.Model(p)
    v = np.random.default_rng(0).normal(size=p.n_dof)
    dt = torch.float64 if prec == "fp64" else torch.float32
    tv = torch.tensor(v, dtype=dt)
    vv = tv.double().numpy()
    if model.startswith("nh"):
        u = 0.01 * np.random.default_rng(1).normal(size=p.n_dof)
        tu = torch.tensor(u, dtype=dt)
        K = om.assemble(tu.double().numpy())
        y = m.hvp(tu, tv, prec=prec).double().cpu().numpy()
    else:
        K = om.assemble()
        y = m.apply_K(tv, prec=prec).double().cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert_bound(y, K @ vv, abs(K) @ abs(vv), tol, f"one element {dim}D {model} {prec}")
    if model.startswith("nh"):
        uo, _ = osolve.newton(p, tol=1e-10)
        u, rep, _ = m.solve(tol=1e-9 if prec == "fp32" else 1e-10, prec=prec)
    else:
        uo, _ = osolve.solve_linear(p, method="direct")
        u, rep, _ = m.solve(tol=1e-8 if prec == "fp32" else 1e-10, prec=prec)
    print(f"[one element] {dim}D {model} {prec}: {rep['status_name']} kv={rep['kv_count']}",
          flush=True)
    assert rep["status"] == 0
    assert rel(u, uo) <= (1e-6 if prec == "fp32" else 1e-9)


@pytest.mark.parametrize("krylov", ["classic", "fused"])
def test_every_dof_prescribed(ctx, krylov):
    """No free DOF: the solve returns the prescribed field at once."""
    from paper_2601_03086_amd import core
    p0 = mk.fan_problem(m=12)
    n = p0.coords.shape[0]
    rng = np.random.default_rng(2)
    vals = rng.normal(size=(n, 2)) * 1e-3
    p = mk.make_problem("lin_plane_strain", p0.coords, p0.conn,
                        dir_nodes=np.repeat(np.arange(n), 2),
                        dir_comps=np.tile([0, 1], n), dir_values=vals.reshape(-1))
    m = core.Mesh.from_problem(ctx, p)
    assert m.info["n_free"] == 0
    for prec in ("fp64", "fp32"):
        u, rep, _ = m.solve(tol=1e-10, prec=prec, krylov=krylov)
        assert rep["status"] == 0 and rep["kv_count"] == 0
        assert np.array_equal(u, vals.reshape(-1))


@pytest.mark.parametrize("krylov", ["classic", "fused"])
def test_zero_load(ctx, krylov):
    """Clamped plate without load: zero is the solution and the zero start
    stops at once; a nonzero start is driven back to zero."""
    import synth
    from paper_2601_03086_amd import core
    q = synth.plate_problem(31, 32, 33, n_holes=4, target_tris=4000)
    p = mk.make_problem("lin_plane_strain", q.coords, q.conn, dir_nodes=q.dir_nodes,
                        dir_comps=q.dir_comps, dir_values=np.zeros(len(q.dir_nodes)))
    m = core.Mesh.from_problem(ctx, p)
    for prec in ("fp64", "fp32"):
        u, rep, _ = m.solve(tol=1e-10, prec=prec, krylov=krylov)
        assert rep["status"] == 0 and rep["kv_count"] == 0
        assert not np.any(u)
    u0 = 1e-3 * np.random.default_rng(3).normal(size=p.n_dof)
    u0.reshape(-1, 2)[q.dir_nodes, q.dir_comps] = 0.0
    u, rep, _ = m.solve(u0=u0, tol=1e-10, prec="fp64", krylov=krylov)
    print(f"[zero load] {krylov}: {rep['status_name']} kv={rep['kv_count']} "
          f"max|u|={np.abs(u).max():.2e}", flush=True)
    assert rep["status"] == 0
    om = fe.Model(p)
    Kff, _, _ = osolve.reduced_system(om)
    # zero right-hand side: the tolerance is absolute on |K_ff u_f|
    assert np.linalg.norm(Kff @ u[om.free_dofs]) <= 1.1e-10


def _two_plates():
    import synth
    q = synth.plate_problem(31, 32, 33, n_holes=2, target_tris=1500)
    n = q.coords.shape[0]
    coords = np.vstack([q.coords, q.coords + np.array([1.5, 0.2])])
    conn = np.vstack([q.conn, q.conn + n])
    dn = np.concatenate([q.dir_nodes, q.dir_nodes + n])
    dc = np.concatenate([q.dir_comps, q.dir_comps])
    dv = np.concatenate([q.dir_values, q.dir_values])
    facets = np.vstack([q.neu_facets, q.neu_facets + n])
    trac = np.vstack([q.neu_traction, 2.0 * q.neu_traction])
    return mk.make_problem("lin_plane_strain", coords, conn, E=np.tile(q.p0, 2),
                           nu=np.tile(q.p1, 2), dir_nodes=dn, dir_comps=dc, dir_values=dv,
                           facets=facets, traction=trac)


@pytest.mark.parametrize("order,bn", [("blocks", 0), ("blocks", 1), ("rcm", 1), ("blocks", 7)])
def test_two_components_and_tiny_blocks(ctx, order, bn):
    """Two disconnected plates in one mesh (numbering, bands and halo lists
    across components) and owner blocks of one or seven nodes: K.v in both
    precisions and fused / classic solves against the oracle."""
    from paper_2601_03086_amd import core
    torch = torch_cuda()
    p = _two_plates()
    m = core.Mesh.from_problem(ctx, p, bn, order)
    om = fe.Model(p)
    K = om.assemble()
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        dt = torch.float64 if prec == "fp64" else torch.float32
        tv = torch.tensor(np.random.default_rng(7).normal(size=p.n_dof), dtype=dt)
        vv = tv.double().numpy()
        y = m.apply_K(tv, prec=prec).double().cpu().numpy()
        assert bound_rel(y, K @ vv, abs(K) @ abs(vv)) <= tol
    uo, _ = osolve.solve_linear(p, method="direct")
    for krylov in ("classic", "fused"):
        u, rep, _ = m.solve(tol=1e-10, prec="fp64", krylov=krylov)
        print(f"[two plates] {order} bn={bn} {krylov}: {rep['status_name']} "
              f"kv={rep['kv_count']} blocks={m.info['n_blocks']}", flush=True)
        assert rep["status"] == 0
        assert rel(u, uo) <= 1e-8
