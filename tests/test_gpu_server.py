"""Serving: continuous batching of solve requests on one GPU.

Each request's result is the same alone and in the mix (within the solve
tolerance), admission never exceeds the memory budget or the slot count,
and cancellation / oversize requests are reported.
"""
import time

import numpy as np
import pytest

import synth
from oracle import solve as osolve
from tests.gpu_util import rel, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    from paper_2601_03086_amd import core
    c = core.Context(0)
    yield c
    c.close()


def _requests():
    reqs = []
    for k in range(4):
        p = synth.plate_problem(200 + k, 300 + k, 400 + k, n_holes=3,
                                target_tris=2000 + 1500 * k)
        ud, _ = osolve.solve_linear(p, method="direct")
        u0 = synth.warm_start_guess(ud, p.coords, p.dir_nodes, seed=500 + k)
        reqs.append((p, u0 if k % 2 == 0 else None, ud))
    for k in range(2):
        p = synth.box_problem(600 + k, 700 + k, n_per_unit=4, n_voids=2, uz=0.2,
                              n_load_steps=2)
        reqs.append((p, None, None))
    return reqs


def _wait(srv, ids, timeout=120.0):
    done = set()
    t0 = time.time()
    while len(done) < len(ids):
        done.update(srv.poll())
        if time.time() - t0 > timeout:
            raise TimeoutError(f"server finished {len(done)} of {len(ids)}")
        time.sleep(0.002)
    return done


def test_alone_equals_in_the_mix(ctx):
    from paper_2601_03086_amd import core
    reqs = _requests()
    host_meshes = [core.Mesh.from_problem(None, p) for p, _, _ in reqs]
    dev_meshes = [core.Mesh.from_problem(ctx, p) for p, _, _ in reqs]
    opts = dict(tol=1e-9, prec="fp32", n_load_steps=2)
    alone = [m.solve(u0=u0, **opts) for m, (_, u0, _) in zip(dev_meshes, reqs)]
    budget = 64 << 20
    srv = core.Server(ctx, budget, max_slots=3)
    for i, (m, (_, u0, _)) in enumerate(zip(host_meshes, reqs)):
        srv.submit(i, m, u0=u0, **opts)
    _wait(srv, list(range(len(reqs))))
    st = srv.stats()
    assert 2 <= st["peak_live"] <= 3 and st["peak_bytes"] <= budget
    assert st["completed"] == len(reqs) and st["bytes_in_use"] == 0
    spans = []
    for i, (p, u0, ud) in enumerate(reqs):
        u, r = srv.result(i)
        ua, ra, _ = alone[i]
        print(i, r["status_name"], r["kv_count"], ra["kv_count"], flush=True)
        assert r["status"] == 0 and ra["status"] == 0
        assert r["rel_residual_final"] <= 1e-9
        assert rel(u, ua) <= 1e-6
        if ud is not None:
            assert rel(u, ud) <= 1e-6
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        spans.append((r["t_admit"], r["t_done"]))
    # the requests overlapped on the device: one was admitted while another
    # was live (admitted earlier, not yet done)
    assert any(a0 < a1 < d0 for i, (a0, d0) in enumerate(spans)
               for j, (a1, _) in enumerate(spans) if i != j)
    srv.close()


def test_mesh_charged_once(ctx):
    """Two requests on one host mesh: the mesh arrays are charged once while
    the server holds them, each request its solve state; a budget for the
    mesh and two solves runs both at once, a budget for the mesh and one
    solve runs them one after the other, and the memory in use returns to 0.
    A request whose mesh and solve can never fit ends with E_OOM when it
    reaches the head of the queue, without blocking the one behind it."""
    from paper_2601_03086_amd import _lib as L
    from paper_2601_03086_amd import core
    p = synth.plate_problem(811, 812, 813, n_holes=3, target_tris=20000)
    m = core.Mesh.from_problem(None, p)
    mesh_b = m.info["device_bytes"]
    solve_b = m.info["solve_bytes_fp32"]
    assert m.footprint("fp32") == mesh_b + solve_b
    opts = dict(tol=1e-8, prec="fp32")
    for budget, live in ((mesh_b + 2 * solve_b, 2), (mesh_b + solve_b, 1)):
        srv = core.Server(ctx, budget, max_slots=4)
        srv.submit(0, m, **opts)
        srv.submit(1, m, tol=1e-9, prec="fp32")
        _wait(srv, [0, 1])
        st = srv.stats()
        print(budget, st, flush=True)
        assert st["peak_live"] == live and st["bytes_in_use"] == 0
        assert st["peak_bytes"] == mesh_b + live * solve_b
        for i in (0, 1):
            _, r = srv.result(i)
            assert r["status"] == 0
        srv.close()
    # mesh + solve beyond the budget, solve alone within it
    small = synth.plate_problem(821, 822, 823, n_holes=2, target_tris=3000)
    ms = core.Mesh.from_problem(None, small)
    srv = core.Server(ctx, mesh_b + solve_b - 1, max_slots=4)
    srv.submit(0, m, **opts)
    srv.submit(1, ms, **opts)
    _wait(srv, [0, 1])
    _, r0 = srv.result(0)
    _, r1 = srv.result(1)
    assert r0["status"] == L.PFEM_E_OOM and r1["status"] == 0
    assert srv.stats()["bytes_in_use"] == 0
    srv.close()


def test_admission_waits_for_memory(ctx):
    """A budget that fits one request at a time serialises the stream."""
    from paper_2601_03086_amd import core
    reqs = _requests()[:3]
    host = [core.Mesh.from_problem(None, p) for p, _, _ in reqs]
    need = max(m.info["device_bytes"] + m.info["solve_bytes_fp32"] for m in host)
    srv = core.Server(ctx, need + 1024, max_slots=8)
    for i, m in enumerate(host):
        srv.submit(i, m, u0=reqs[i][1], tol=1e-8, prec="fp32")
    _wait(srv, [0, 1, 2])
    st = srv.stats()
    assert st["peak_live"] == 1 and st["peak_bytes"] <= need + 1024
    times = [srv.result(i)[1] for i in range(3)]
    for a, b in zip(times, times[1:]):
        assert b["t_admit"] >= a["t_done"] - 1e-3
    srv.close()


def test_oversize_and_cancel(ctx):
    from paper_2601_03086_amd import _lib as L
    from paper_2601_03086_amd import core
    p = synth.plate_problem(801, 802, 803, n_holes=4, target_tris=30000)
    m = core.Mesh.from_problem(None, p)
    srv = core.Server(ctx, 1 << 20, max_slots=2)       # 1 MiB: too small
    with pytest.raises(L.PfemError) as ei:
        srv.submit(0, m, tol=1e-8)
    assert ei.value.status == L.PFEM_E_OOM
    srv.close()
    # a long request (FP64 from zero to the residual floor of a 100k-triangle
    # plate: thousands of iterations) is cancelled once it runs, the one
    # queued behind it before it runs
    big = core.Mesh.from_problem(None, synth.plate_problem(804, 805, 806, n_holes=4,
                                                           target_tris=100000))
    srv = core.Server(ctx, 1 << 30, max_slots=1)
    srv.submit(1, big, tol=1e-13, prec="fp64", krylov="classic", max_iter=10 ** 7)
    srv.submit(2, m, tol=1e-8)
    t0 = time.time()
    while srv.stats()["live"] < 1:
        assert time.time() - t0 < 30, "the long request was never admitted"
        time.sleep(0.001)
    srv.cancel(1)
    srv.cancel(2)
    _wait(srv, [1, 2], timeout=60)
    for i in (1, 2):
        _, r = srv.result(i)
        assert r["status"] == L.PFEM_E_CANCELLED
    srv.close()


def test_finished_at_admission_and_late_cancel(ctx):
    """A request whose warm start already meets tol_fine finishes when it is
    admitted (its result is its warm start, reported SKIPPED_FINE) and is
    collected like the others; a cancel that arrives after a request has
    finished leaves its result intact; every result equals its lone solve."""
    from paper_2601_03086_amd import _lib as L
    from paper_2601_03086_amd import core
    p = synth.plate_problem(901, 902, 903, n_holes=2, target_tris=3000)
    q = synth.plate_problem(904, 905, 906, n_holes=2, target_tris=5000)
    mp = core.Mesh.from_problem(ctx, p)
    ud, _, _ = mp.solve(tol=1e-11, prec="fp64")
    u1, r1, _ = core.Mesh.from_problem(ctx, q).solve(tol=1e-9, prec="fp32")
    hp, hq = core.Mesh.from_problem(None, p), core.Mesh.from_problem(None, q)
    srv = core.Server(ctx, 1 << 30, max_slots=2)
    srv.submit(0, hp, u0=ud, tol=1e-9, tol_fine=1e-6, prec="fp32")   # done at admission
    srv.submit(1, hq, tol=1e-9, prec="fp32")
    srv.submit(2, hp, u0=ud, tol=1e-9, tol_fine=1e-6, prec="fp32")
    _wait(srv, [0, 1, 2])
    srv.cancel(1)                       # too late: it has finished
    for i in (0, 2):
        u, r = srv.result(i)
        assert r["status"] == L.PFEM_SKIPPED_FINE
        assert np.array_equal(u, ud)
    u, r = srv.result(1)
    assert r["status"] == 0
    assert rel(u, u1) <= 1e-6
    st = srv.stats()
    assert st["live"] == 0 and st["bytes_in_use"] == 0
    assert st["admit_s"] >= 0 and st["tick_s"] > 0 and st["complete_s"] >= 0
    srv.close()
