"""The differentiable energy: torch.autograd over the device kernels.

energy -> backward is the internal-force kernel, double backward the
Hessian-vector kernel.  Checked against the FP64 oracle, central finite
differences (h = 1e-3, FP64) and torch.autograd.gradcheck on a tiny mesh;
the batched form (many meshes per launch) against per-mesh oracle values.
"""
import numpy as np
import pytest

import synth
from oracle import fe
from tests import meshkit as mk
from tests.gpu_util import assert_bound, bound_rel, rel, smooth_field, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    from paper_2601_03086_amd import core
    c = core.Context(0)
    yield c
    c.close()


def _mesh(ctx, p, bn=0):
    from paper_2601_03086_amd import core
    return core.Mesh.from_problem(ctx, p, bn)


@pytest.mark.parametrize("model", ["lin_plane_strain", "nh_plane_strain", "nh_3d"])
def test_energy_grad_hvp_fp64(ctx, model):
    torch = torch_cuda()
    from paper_2601_03086_amd import autograd
    if model == "nh_3d":
        p = synth.box_problem(101, 102, n_per_unit=4, n_voids=2, n_load_steps=1)
    else:
        p = synth.plate_problem(103, 104, 105, n_holes=3, target_tris=2500, model=model)
    m = _mesh(ctx, p)
    om = fe.Model(p)
    u = smooth_field(p, 6, 0.05)
    w = np.random.default_rng(7).normal(size=p.n_dof)
    ut = torch.tensor(u, device="cuda", requires_grad=True)
    e = autograd.energy(m, ut, prec="fp64")
    assert abs(e.item() - om.energy(u)) <= 1e-12 * abs(om.energy(u))
    (g,) = torch.autograd.grad(e, ut, create_graph=True)
    assert rel(g.detach().cpu().numpy(), om.gradient(u)) <= 1e-12
    (hv,) = torch.autograd.grad(g, ut, grad_outputs=torch.tensor(w, device="cuda"))
    KT = om.assemble(u)
    assert bound_rel(hv.cpu().numpy(), KT @ w, abs(KT) @ abs(w)) <= 1e-12


@pytest.mark.parametrize("model", ["lin_plane_strain", "nh_plane_strain"])
def test_central_finite_differences(ctx, model):
    """Directional derivatives of the device energy and force by central
    differences in FP64, h = 1e-3, unit direction on the free DOFs."""
    torch = torch_cuda()
    from paper_2601_03086_amd import autograd
    p = synth.plate_problem(106, 107, 108, n_holes=2, target_tris=1500, model=model)
    m = _mesh(ctx, p)
    om = fe.Model(p)
    u = smooth_field(p, 8, 0.05)
    w = np.zeros(p.n_dof)
    w[om.free_dofs] = np.random.default_rng(9).normal(size=om.free_dofs.size)
    w /= np.linalg.norm(w)
    h = 1e-3
    dev = lambda a: torch.tensor(a, device="cuda", dtype=torch.float64)
    E = lambda a: m.energy(dev(a), prec="fp64").item()
    G = lambda a: m.force(dev(a), prec="fp64").cpu().numpy()
    ut = dev(u).requires_grad_(True)
    e = autograd.energy(m, ut, prec="fp64")
    (g,) = torch.autograd.grad(e, ut, create_graph=True)
    (hv,) = torch.autograd.grad(g, ut, grad_outputs=dev(w))
    fd_e = (E(u + h * w) - E(u - h * w)) / (2 * h)
    gw = float(g.detach().cpu().numpy() @ w)
    assert abs(fd_e - gw) <= 1e-6 * max(1.0, abs(gw))
    fd_g = (G(u + h * w) - G(u - h * w)) / (2 * h)
    hvn = hv.cpu().numpy()
    assert np.linalg.norm(fd_g - hvn) <= 1e-5 * np.linalg.norm(hvn)


def test_gradcheck_tiny_mesh(ctx):
    torch = torch_cuda()
    from paper_2601_03086_amd import autograd
    coords, conn = mk.patch_2d(3, seed=2)
    p = mk.make_problem("nh_plane_strain", coords, conn, E=2.0, nu=0.3)
    m = _mesh(ctx, p)
    u = torch.tensor(smooth_field(p, 3, 0.05), device="cuda", requires_grad=True)
    f = lambda x: autograd.energy(m, x, prec="fp64")
    assert torch.autograd.gradcheck(f, (u,), eps=1e-6, atol=1e-7, rtol=1e-6)
    assert torch.autograd.gradgradcheck(f, (u,), eps=1e-6, atol=1e-7, rtol=1e-6)


@pytest.mark.parametrize("model", ["lin_plane_strain", "nh_plane_strain"])
def test_fp32_energy_force_hvp(ctx, model):
    torch = torch_cuda()
    from paper_2601_03086_amd import autograd
    p = synth.plate_problem(110, 111, 112, n_holes=3, target_tris=4000, model=model)
    m = _mesh(ctx, p)
    om = fe.Model(p)
    u32 = torch.tensor(smooth_field(p, 10, 0.05), device="cuda", dtype=torch.float32)
    u = u32.double().cpu().numpy()
    w = torch.randn(p.n_dof, device="cuda", dtype=torch.float32)
    ut = u32.clone().requires_grad_(True)
    e = autograd.energy(m, ut, prec="fp32")
    (g,) = torch.autograd.grad(e, ut, create_graph=True)
    (hv,) = torch.autograd.grad(g, ut, grad_outputs=w)
    assert abs(e.item() - om.energy(u)) <= 1e-5 * abs(om.energy(u))
    KT = om.assemble(u)
    ww = w.double().cpu().numpy()
    scale = np.linalg.norm(abs(KT) @ abs(u)) + np.linalg.norm(om.f_ext)
    eg = np.linalg.norm(g.detach().double().cpu().numpy() - om.gradient(u)) / scale
    print(f"[err] autograd force {model} fp32: {eg:.2e}", flush=True)
    assert eg <= 1e-5
    assert_bound(hv.double().cpu().numpy(), KT @ ww, abs(KT) @ abs(ww), 1e-5,
                 f"autograd hvp {model} fp32")


def _internal(vec_user, perm, d):
    out = np.empty_like(vec_user)
    out.reshape(-1, d)[perm] = vec_user.reshape(-1, d)
    return out


@pytest.mark.parametrize("n", [6, 64])
def test_batched_energy_matches_per_mesh_oracle(ctx, n):
    """The differentiable-energy batch: n plates (alternating linear and
    Neo-Hookean, 5k-20k triangles when n = 64), one launch per kernel."""
    torch = torch_cuda()
    from paper_2601_03086_amd import _lib as L
    from paper_2601_03086_amd import autograd, core
    if n == 64:
        members = synth.batch_c4(64)
    else:
        members = [synth.problems.c4_member(i, target=2500 + 500 * i) for i in range(n)]
    meshes = [_mesh(ctx, p) for p, _ in members]
    b = core.Batch(ctx, meshes)
    perms = [m.query(L.PFEM_Q_PERM) for m in meshes]
    u_cat = np.concatenate([_internal(u.astype(np.float64), pr, 2)
                            for (p, u), pr in zip(members, perms)])
    ut = torch.tensor(u_cat, device="cuda", dtype=torch.float32, requires_grad=True)
    e = autograd.batch_energy(b, ut, prec="fp32")
    (g,) = torch.autograd.grad(e.sum(), ut, create_graph=True)
    w = torch.randn_like(ut)
    (hv,) = torch.autograd.grad(g, ut, grad_outputs=w)
    e = e.detach().cpu().numpy()
    g = g.detach().double().cpu().numpy()
    hv = hv.double().cpu().numpy()
    wn = w.double().cpu().numpy()
    off = b.offsets
    check = range(n) if n <= 8 else [0, 1, 17, 32, 63]
    for i, ((p, u), pr) in enumerate(zip(members, perms)):
        om = fe.Model(p)
        uu = u.astype(np.float64)
        assert abs(e[i] - om.energy(uu)) <= 1e-5 * abs(om.energy(uu)), i
        if i not in check:
            continue
        KT = om.assemble(uu)
        gi = _internal(om.gradient(uu), pr, 2)
        scale = np.linalg.norm(abs(KT) @ abs(uu)) + np.linalg.norm(om.f_ext)
        eg = np.linalg.norm(g[off[i]:off[i + 1]] - gi) / scale
        print(f"[err] batch force mesh {i}: {eg:.2e}", flush=True)
        assert eg <= 1e-5, i
        # HVP: K_T in internal order applied to the internal-order direction
        wi = wn[off[i]:off[i + 1]]
        wu = wi.reshape(-1, 2)[pr].reshape(-1)        # back to user order
        ref = _internal(KT @ wu, pr, 2)
        bound = _internal(abs(KT) @ abs(wu), pr, 2)
        assert_bound(hv[off[i]:off[i + 1]], ref, bound, 1e-5, f"batch hvp mesh {i}")
