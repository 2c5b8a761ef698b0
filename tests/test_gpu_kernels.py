"""Element-kernel parity: device K.v, Hessian-vector product, internal force,
energy and Jacobi diagonal against the FP64 oracle (assembled K, K_T)."""
import numpy as np
import pytest

import synth
from oracle import fe
from tests import meshkit as mk
from tests.gpu_util import (assert_bound, bound_rel, compressed_field, rel, sample_rows,
                            smooth_field, torch_cuda)

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    from paper_2601_03086_amd import core
    c = core.Context(0)
    yield c
    c.close()


def _varied_ratio(p, seed):
    """Same mesh with a Poisson ratio (or lambda / mu) that varies per
    element, so the kernels read both material arrays."""
    rng = np.random.default_rng(seed)
    if p.param_kind == "E_nu":
        p.p1 = rng.uniform(0.15, 0.45, size=p.n_elems)
    else:
        p.p1 = p.p0 * rng.uniform(1.0, 6.0, size=p.n_elems)
    p.name = p.name + "_varied"
    return p


def _problems():
    return {
        "plate_nu": _varied_ratio(synth.plate_problem(71, 72, 73, n_holes=4, target_tris=5000,
                                                      model="lin_plane_strain"), 1),
        "box_nh_lam": _varied_ratio(synth.box_problem(74, 75, n_per_unit=5, n_voids=3,
                                                      n_load_steps=2), 2),
        "c1": synth.unit_square_c1(),
        "plate_lin": synth.plate_problem(61, 62, 63, n_holes=5, target_tris=6000,
                                         model="lin_plane_strain"),
        "plate_nh": synth.plate_problem(64, 65, 66, n_holes=3, target_tris=3000,
                                        model="nh_plane_strain"),
        "box_lin": synth.box_problem(67, 68, n_per_unit=6, n_voids=4, model="lin_3d",
                                     n_load_steps=1),
        "box_nh": synth.box_problem(69, 70, n_per_unit=5, n_voids=3, n_load_steps=2),
    }


PROBS = _problems()


def _mesh(ctx, name, bn=0, order="blocks"):
    from paper_2601_03086_amd import core
    return core.Mesh.from_problem(ctx, PROBS[name], bn, order)


@pytest.mark.parametrize("name", ["c1", "plate_lin", "box_lin", "plate_nu"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("scatter", ["owner", "colored", "atomic"])
@pytest.mark.parametrize("bn", [0, 32])
def test_apply_K_parity(ctx, name, prec, scatter, bn):
    torch = torch_cuda()
    p = PROBS[name]
    print(f"[apply_K] {name} {prec} {scatter} bn={bn}", flush=True)
    m = _mesh(ctx, name, bn)
    om = fe.Model(p)
    K = om.assemble()
    v = np.random.default_rng(1).normal(size=p.n_dof)
    y = m.apply_K(torch.tensor(v), prec=prec, scatter=scatter).double().cpu().numpy()
    yref = K @ v
    vv = v.astype(np.float32).astype(np.float64) if prec == "fp32" else v
    assert_bound(y, K @ vv, abs(K) @ abs(vv), TOL[prec], f"K.v {name} {prec} {scatter}")
    assert rel(y, yref) <= (1e-12 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("name", ["plate_lin", "box_lin", "plate_nh", "box_nh"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("bn", [0, 32])
def test_rcm_numbering_parity(ctx, name, prec, bn):
    """The element kernels do not depend on the node numbering: K.v (or the
    Neo-Hookean HVP at a smooth state) with plain RCM blocks."""
    torch = torch_cuda()
    p = PROBS[name]
    print(f"[rcm order] {name} {prec} bn={bn}", flush=True)
    m = _mesh(ctx, name, bn, "rcm")
    om = fe.Model(p)
    dt = torch.float64 if prec == "fp64" else torch.float32
    tv = torch.tensor(np.random.default_rng(3).normal(size=p.n_dof), dtype=dt)
    vv = tv.double().numpy()
    if p.model.startswith("nh"):
        tu = torch.tensor(smooth_field(p, 3, 0.08), dtype=dt)
        K = om.assemble(tu.double().numpy())
        y = m.hvp(tu, tv, prec=prec).double().cpu().numpy()
    else:
        K = om.assemble()
        y = m.apply_K(tv, prec=prec).double().cpu().numpy()
    assert_bound(y, K @ vv, abs(K) @ abs(vv), TOL[prec], f"rcm {name} {prec}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_unpacked_connectivity_apply_K(ctx, prec):
    """A 70k-triangle fan under plain RCM has element node offsets beyond
    16 bits, so the kernels read plain int32 rows (the run-time format test)
    instead of packed ones."""
    from paper_2601_03086_amd import core
    torch = torch_cuda()
    p = mk.fan_problem()
    m = core.Mesh.from_problem(ctx, p, 0, "rcm")
    assert m.info["bandwidth_internal"] > 65535
    K = fe.Model(p).assemble()
    dt = torch.float64 if prec == "fp64" else torch.float32
    tv = torch.tensor(np.random.default_rng(5).normal(size=p.n_dof), dtype=dt)
    vv = tv.double().numpy()
    y = m.apply_K(tv, prec=prec).double().cpu().numpy()
    # the fan's sliver elements (aspect ratio ~1e4) amplify FP32 geometry
    # rounding about 10x beyond the usual bound (measured 8.5e-5); an indexing
    # error in the unpacked path would show at O(1)
    tol = TOL[prec] if prec == "fp64" else 5e-4
    # norm-wise only: single sliver rows reach 1.5e-2 of their own bound
    assert bound_rel(y, K @ vv, abs(K) @ abs(vv), f"fan {prec}") <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_K_masks_and_internal_layout(ctx, prec):
    torch = torch_cuda()
    from paper_2601_03086_amd import _lib as L
    p = PROBS["plate_lin"]
    m = _mesh(ctx, "plate_lin", 48)
    K = fe.Model(p).assemble().toarray()
    con = np.zeros(p.n_dof, dtype=bool)
    con[np.asarray(p.dir_nodes) * 2 + np.asarray(p.dir_comps)] = True
    v = np.random.default_rng(2).normal(size=p.n_dof)
    tv = torch.tensor(v)
    for mask in (L.PFEM_MASK_OUT, L.PFEM_MASK_IN, L.PFEM_MASK_OUT | L.PFEM_MASK_IN):
        Km = K.copy()
        if mask & L.PFEM_MASK_OUT:
            Km[con, :] = 0
        if mask & L.PFEM_MASK_IN:
            Km[:, con] = 0
        y = m.apply_K(tv, prec=prec, mask=mask).double().cpu().numpy()
        assert bound_rel(y, Km @ v, abs(Km) @ abs(v)) <= TOL[prec]
    # internal layout: permute in, apply, permute out
    vi = m.permute(tv, True, prec)
    yi = m.apply_K(vi, prec=prec, layout="internal")
    y = m.permute(yi, False, prec).double().cpu().numpy()
    assert bound_rel(y, K @ v, abs(K) @ abs(v)) <= TOL[prec]


@pytest.mark.parametrize("name", ["plate_nh", "box_nh", "box_nh_lam"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("bn", [0, 40])
def test_hvp_force_energy_diag_nh(ctx, name, prec, bn):
    torch = torch_cuda()
    p = PROBS[name]
    print(f"[nh] {name} {prec} bn={bn}", flush=True)
    m = _mesh(ctx, name, bn)
    om = fe.Model(p)
    u = smooth_field(p, 3, 0.08)
    v = np.random.default_rng(4).normal(size=p.n_dof)
    dt = torch.float64 if prec == "fp64" else torch.float32
    tu = torch.tensor(u, dtype=dt)
    y = m.hvp(tu, torch.tensor(v, dtype=dt), prec=prec).double().cpu().numpy()
    vv = torch.tensor(v, dtype=dt).double().numpy()
    _check_nh_state(m, om, p, tu, vv, y, prec, f"{name} bn={bn}")


def _check_nh_state(m, om, p, tu, vv, y, prec, label):
    """HVP y = K_T(u) v, force, energy and Jacobi diagonal of the device at
    the state tu against the oracle at the same (rounded) state."""
    uu = tu.double().numpy()
    KTu = om.assemble(uu)
    assert_bound(y, KTu @ vv, abs(KTu) @ abs(vv), TOL[prec], f"hvp {label} {prec}")
    g = m.force(tu, prec=prec).double().cpu().numpy()
    gref = om.gradient(uu)
    # |K_T| |u| (+ |f_ext|) bounds the rounding of the element stresses
    scale = np.linalg.norm(abs(KTu) @ abs(uu)) + np.linalg.norm(om.f_ext)
    eg = np.linalg.norm(g - gref) / scale
    print(f"[err] force {label} {prec}: {eg:.2e}", flush=True)
    assert eg <= TOL[prec]
    e = m.energy(tu, prec=prec).item()
    eref = om.energy(uu)
    print(f"[err] energy {label} {prec}: {abs(e - eref) / abs(eref):.2e}", flush=True)
    assert abs(e - eref) <= TOL[prec] * abs(eref)
    d = m.diag(tu, prec=prec).double().cpu().numpy()
    dref = KTu.diagonal().copy()
    con = np.asarray(p.dir_nodes) * p.dim + np.asarray(p.dir_comps)
    dref[con] = 1.0
    print(f"[err] diag {label} {prec}: {rel(d, dref):.2e}", flush=True)
    assert rel(d, dref) <= TOL[prec]


@pytest.mark.parametrize("name", ["plate_nh", "box_nh"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nh_compressed_state(ctx, name, prec):
    """Neo-Hookean kernels near compression: a Gaussian patch squeezed to
    J = 0.2 at its centre (plus a smooth 1% strain field), where ln J and 1/J
    amplify the rounding of J - 1 (float32 kernels evaluate det F in float64
    there).  HVP, force, energy and diagonal against the oracle."""
    torch = torch_cuda()
    p = PROBS[name]
    m = _mesh(ctx, name)
    om = fe.Model(p)
    # the coarse box (h = 0.2) resolves the patch centre less sharply: aim
    # lower so that its most compressed element reaches J of about 0.2 too
    u = compressed_field(p, 0.2 if p.dim == 2 else 0.12, seed=11)
    Jm = 1.0 + fe.nh_invariants(om.H(u))[0]
    print(f"[compressed] {name}: J in [{Jm.min():.3f}, {Jm.max():.3f}], "
          f"{(Jm < 0.7).sum()} of {Jm.size} elements below 0.7", flush=True)
    assert Jm.min() < 0.25 and Jm.min() > 0.1
    dt = torch.float64 if prec == "fp64" else torch.float32
    tu = torch.tensor(u, dtype=dt)
    tv = torch.tensor(np.random.default_rng(12).normal(size=p.n_dof), dtype=dt)
    y = m.hvp(tu, tv, prec=prec).double().cpu().numpy()
    _check_nh_state(m, om, p, tu, tv.double().numpy(), y, prec, f"{name} compressed")


@pytest.mark.parametrize("name", ["c1", "plate_lin", "box_lin"])
def test_linear_force_energy_diag(ctx, name):
    torch = torch_cuda()
    p = PROBS[name]
    m = _mesh(ctx, name)
    om = fe.Model(p)
    K = om.assemble()
    u = smooth_field(p, 5, 0.01)
    tu = torch.tensor(u)
    g = m.force(tu, prec="fp64").cpu().numpy()
    assert rel(g, K @ u - om.f_ext) <= 1e-12
    e = m.energy(tu, prec="fp64").item()
    assert abs(e - om.energy(u)) <= 1e-12 * abs(om.energy(u))
    d = m.diag(None, prec="fp64").cpu().numpy()
    dref = K.diagonal().copy()
    con = np.asarray(p.dir_nodes) * p.dim + np.asarray(p.dir_comps)
    dref[con] = 1.0
    assert rel(d, dref) <= 1e-13


def test_energy_inverted_element_is_inf(ctx):
    torch = torch_cuda()
    p = PROBS["plate_nh"]
    m = _mesh(ctx, "plate_nh")
    u = np.zeros(p.n_dof)
    a, b, c = p.conn[0]
    u[2 * a:2 * a + 2] = (p.coords[b] - p.coords[a]) * 3.0   # fold element 0
    e = m.energy(torch.tensor(u), prec="fp64").item()
    assert e == float("inf")
    assert fe.Model(p).energy(u) == float("inf")


def test_full_size_c2_apply_K(ctx):
    """C2-size plate (~2e5 triangles): every output of K.v against the
    oracle's assembled K, FP64 and FP32, owner scatter as the solver runs it."""
    torch = torch_cuda()
    from paper_2601_03086_amd import core
    p = synth.plate_problem(2, 1002, 2002)
    print(f"[c2] {p.n_elems} triangles", flush=True)
    m = core.Mesh.from_problem(ctx, p)
    K = fe.Model(p).assemble()
    v = np.random.default_rng(6).normal(size=p.n_dof)
    Kav = abs(K) @ abs(v)
    for prec in ("fp64", "fp32"):
        y = m.apply_K(torch.tensor(v), prec=prec).double().cpu().numpy()
        vv = v.astype(np.float32).astype(np.float64) if prec == "fp32" else v
        assert_bound(y, K @ vv, Kav, TOL[prec], f"c2 K.v {prec}")


def test_full_size_c3_hvp_sampled_rows(ctx):
    """C3-size box (~1e6 tets, Neo-Hookean): sampled rows of K_T(u) v and of
    f_int(u) against the oracle evaluated on the incident elements only."""
    torch = torch_cuda()
    from paper_2601_03086_amd import core
    p = synth.box_problem(3, 1003)
    print(f"[c3] {p.n_elems} tets", flush=True)
    m = core.Mesh.from_problem(ctx, p)
    rng = np.random.default_rng(7)
    u = np.zeros(p.n_dof)
    u.reshape(-1, 3)[:, 2] = 0.02 * p.coords[:, 2] * (1 + 0.1 * np.sin(3 * p.coords[:, 0]))
    v = rng.normal(size=p.n_dof)
    nodes = rng.choice(p.n_nodes, 256, replace=False)
    sub = sample_rows(p, nodes)
    om = fe.Model(sub)
    KT = om.assemble(u)
    rows = (nodes[:, None] * 3 + np.arange(3)).reshape(-1)
    for prec in ("fp64", "fp32"):
        dt = torch.float64 if prec == "fp64" else torch.float32
        tu = torch.tensor(u, dtype=dt)
        y = m.hvp(tu, torch.tensor(v, dtype=dt), prec=prec).double().cpu().numpy()
        uu = tu.double().numpy()
        vv = torch.tensor(v, dtype=dt).double().numpy()
        KTu = om.assemble(uu)
        ref = (KTu @ vv)[rows]
        assert_bound(y[rows], ref, (abs(KTu) @ abs(vv))[rows], TOL[prec], f"c3 hvp {prec}")
        g = m.force(tu, prec=prec).double().cpu().numpy()
        gref = om.internal_force(uu)[rows]   # no tractions in C3
        assert_bound(g[rows], gref, (abs(KTu) @ abs(uu))[rows], TOL[prec], f"c3 force {prec}")
    del KT
