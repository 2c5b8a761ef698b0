#!/usr/bin/env python3
"""Benchmark: warm-started solves served with continuous batching (one GPU).

Workload (default): a serving stream of 512 solve requests, each on its own
seeded mesh (70% plane-strain plates with 8 random holes, linear; 30%
1x1x4 boxes with 20 ellipsoidal voids, compressible Neo-Hookean), sizes
log-uniform in 1e4-5e5 elements, Poisson arrivals at 200/s.  Every request
carries a warm start (its reference solution + 1% smooth noise, standing
in for a network prediction) and is solved to a 1e-8 relative residual in
FP32 mode (FP32 element kernels and Krylov vectors, FP64 dots, residuals
and state).  Meshes, references (FP64, 1e-11, from zero) and guesses are
prepared before the timed region; the server uploads each mesh when it
admits the request.  The timed region is one open-loop replay of the whole
stream; its K steps are K windows of consecutive arrivals.

value = served solves/s (512 / (last completion - first submission)), with
p50 / p99 latency (completion - submission).  Beside it: the same stream
from zero starts under the same arrivals, the same requests solved one at a
time (warm and zero), batched K.v over all resident plates (a working set
beyond the caches), the 200k-triangle plate's solve, an oracle check of 16
served results, and the oracle timed on host cores.  The roofline object
describes the stream's dominant kernel, the fused PCG iteration batched
over the live requests: algorithmic bytes over the launches that did work
(counted by the library per solve and iteration) divided by their
duration, measured with HIP events on the server's stream.

Other modes (not the default line):
  --kv-only N        N back-to-back K.v launches, or with --kv-kernel fused
                     about N fused PCG iterations (for rocprofv3 counters)
  --parse-pmc DIR    mean counter values per kernel from rocprofv3 CSVs
  --config NAME      c1 | c2 | c3 | c4 | sweep | rotate | homog: the other
                     workloads (unit square, 200k-triangle plate alone, 3D
                     Neo-Hookean box, 64-mesh batch, K.v size sweep,
                     rotating-buffer K.v, 64^3 TPMS cell homogenisation),
                     one JSON line each
"""
import argparse
import glob
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Matrix-free K·v GDOF/s (% HBM roofline); solves/s + p99 latency at "
          "1e-8 rel")
HBM_PEAK_GBS = 8000.0
FAM_APPLY, FAM_FORCE, FAM_ENERGY, FAM_DIAG, FAM_UPDATE, FAM_DIRECTION, FAM_FUSED = range(7)
FAM_NAMES = ["apply", "force", "energy", "diag", "update", "direction", "fused_iter"]
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "pcg_iter_fp32_plate200k_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2601_03086_amd", "csrc", "elem_kernels.hip")
KERNEL_NAME = "k_fcg<2, float, false>"
KERNEL_MATCH = "k_fcg<2, float, false>"



# internal node numbering and owner-block size of every mesh the benchmark
# builds ("blocks" / "rcm"; 0 = automatic block size)
ORDER = "blocks"
BLOCK_NODES = 0


def new_mesh(ctx, prob, bn=0):
    from paper_2601_03086_amd import core
    return core.Mesh.from_problem(ctx, prob, bn, ORDER)

def kernel_hash():
    h = hashlib.sha256()
    # the kernels and the mesh layout they read (numbering, blocks, packing)
    for f in ("elem_kernels.hip", "elem_math.h", "reduce.h", "pfem_internal.h", "mesh.cpp"):
        h.update(open(os.path.join(ROOT, "paper_2601_03086_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def c2_problem():
    import synth
    return synth.plate_problem(2, 1002, 2002)   # geometry, material, BC seeds


def alg_bytes_kv(n_elems, n_nodes, dim, s=4, s_m=4):
    """Algorithmic bytes of one K.v: connectivity, one material value per
    element, coordinates, x read and y written once."""
    return 4 * (dim + 1) * n_elems + s_m * n_elems + 3 * dim * s * n_nodes


def alg_bytes_fused(n_elems, n_nodes, dim, s=4, s_m=4):
    """Algorithmic bytes of one fused PCG iteration: connectivity, one
    material value per element and the coordinates, each once; the node
    records {r, w, s, M^-1} read once and {r, w, s} written once; p and d
    read and written once."""
    return 4 * (dim + 1) * n_elems + s_m * n_elems + (1 + 4 + 3 + 4) * dim * s * n_nodes


# --------------------------------------------------------------- CPU baseline
# The oracle's whole warm solve is the CPU sample (about 4,100 K.v products
# to 1e-8); the cap only bounds a run that would not converge.
MAX_KV = 8000


def cpu_baseline_worker():
    """The FP64 oracle timed on host cores: Jacobi-PCG (scipy CSR SpMV) from
    the same warm start to 1e-8, the complete solve (at most MAX_KV K.v
    products)."""
    import numpy as np
    import synth
    from oracle import fe, solve as osolve
    prob = c2_problem()
    m = fe.Model(prob)
    Kff, Ff, uD = osolve.reduced_system(m)
    import scipy.sparse.linalg as spla
    uf = spla.spsolve(Kff.tocsc(), Ff)
    ustar = uD.copy()
    ustar[m.free_dofs] = uf
    u0 = synth.warm_start_guess(ustar, prob.coords, prob.dir_nodes, seed=3002)
    t0 = time.perf_counter()
    x, hist, kv, st = osolve.pcg(Kff, Ff, u0[m.free_dofs], 1e-8, max_iter=MAX_KV)
    t = time.perf_counter() - t0
    print(json.dumps({"seconds": t, "kv": kv, "n_dof": prob.n_dof, "status": st,
                      "final_rel": hist[-1], "threads": 1}))


def cpu_baseline():
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    r = subprocess.run([sys.executable, __file__, "--cpu-baseline-worker"], env=env,
                       capture_output=True, text=True, timeout=600)
    line = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or not line:
        return {"error": (r.stderr or r.stdout)[-400:]}
    d = json.loads(line[-1])
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": d["kv"] * d["n_dof"] / d["seconds"] / 1e9, "unit": "GDOF/s",
            "cores": d["threads"], "kind": "oracle",
            "host": {"cpu_model": model, "affinity_cpus": len(os.sched_getaffinity(0)),
                     "threads_env": {k: env[k] for k in ("OMP_NUM_THREADS",
                                                         "OPENBLAS_NUM_THREADS",
                                                         "MKL_NUM_THREADS")}},
            "sample": (f"oracle FP64 Jacobi-PCG (scipy CSR SpMV) on the same plate, "
                       f"same warm start, the whole solve to 1e-8: {d['kv']} K.v "
                       f"products in {d['seconds']:.1f} s (status {d['status']}, "
                       f"final rel {d['final_rel']:.1e}); 1 thread")}


# ------------------------------------------------------------------ traffic
def _short_kernel(name):
    import re
    m = re.match(r"(?:void )?(?:pfem::)?([A-Za-z_0-9]+)(<[^()]*>)?", name)
    return (m.group(1) + (m.group(2) or "")) if m else name[:40]


def parse_pmc(out_dir):
    """Mean counter value per dispatch, by kernel and counter, from the
    rocprofv3 counter CSVs under out_dir (pfem kernels, and device copies
    of at least 100000 KiB, which calibrate the byte counters)."""
    import csv
    vals = {}
    for f in glob.glob(os.path.join(out_dir, "**", "*counter_collection.csv"), recursive=True):
        for row in csv.DictReader(open(f)):
            name = row.get("Kernel_Name", "")
            ctr = row.get("Counter_Name", "")
            v = float(row.get("Counter_Value", 0))
            if "copyBuffer" in name and ctr in ("FETCH_SIZE", "WRITE_SIZE") and v > 100000:
                key = "copy_256MiB"
            elif "pfem::" in name:
                key = _short_kernel(name)
            else:
                continue
            vals.setdefault((key, ctr), []).append(v)
    return {f"{k} | {c}": round(sum(v) / len(v), 3) for (k, c), v in sorted(vals.items())}


def traffic_entry():
    if not os.path.exists(TRAFFIC_JSON):
        return None
    d = json.load(open(TRAFFIC_JSON))
    if d.get("kernel_hash") != kernel_hash():
        return None   # kernel changed since the counters were taken
    return d.get("traffic_bytes_per_launch")


# ------------------------------------------------------- per-config legs
def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _kv_rate(ctx, mesh, prec, reps=100, trials=5, warm=10, hvp_state=None):
    """Median over trials of the average K.v (or HVP at hvp_state) time in
    microseconds, internal layout, events around `reps` back-to-back launches."""
    import torch
    dt = torch.float32 if prec == "fp32" else torch.float64
    x = mesh.permute(torch.randn(mesh.n_dof, dtype=dt, device="cuda"), True, prec)
    y = torch.empty_like(x)
    u = None
    if hvp_state is not None:
        u = mesh.permute(torch.as_tensor(hvp_state, dtype=dt, device="cuda"), True, prec)
    call = ((lambda: mesh.hvp(u, x, prec=prec, layout="internal", out=y)) if u is not None
            else (lambda: mesh.apply_K(x, prec=prec, layout="internal", out=y)))
    for _ in range(warm):
        call()
    ts = []
    for _ in range(trials):
        ctx.set_timing([FAM_APPLY])
        ctx.reset_timing()
        for _ in range(reps):
            call()
        n, ms = ctx.kernel_time(FAM_APPLY)
        ts.append(ms / n * 1e3)
    ctx.set_timing(())
    ts.sort()
    return ts[len(ts) // 2]


def _timed_solve(mesh, **kw):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, rep, _ = mesh.solve(**kw)
    torch.cuda.synchronize()
    return u, rep, time.perf_counter() - t0


def run_c1():
    """Unit square, FP64: solves from zero and from a warm start to 1e-10,
    and the FP64 K.v rate."""
    import synth
    import torch
    from paper_2601_03086_amd import core
    prob = synth.unit_square_c1()
    ctx = core.Context(0)
    mesh = new_mesh(ctx, prob)
    uref, _, _ = mesh.solve(tol=1e-12, prec="fp64", device_io=True)
    u0 = synth.warm_start_guess(uref.cpu().numpy(), prob.coords, prob.dir_nodes, seed=11)
    out = {"config": "C1 unit square, 2048 triangles, plane stress, FP64 PCG to 1e-10"}
    for name, guess in (("zero", None), ("warm", u0)):
        best = None
        for _ in range(5):
            _, rep, t = _timed_solve(mesh, u0=guess, tol=1e-10, prec="fp64", history_cap=1)
            best = t if best is None else min(best, t)
        out[name] = {"ms": round(best * 1e3, 3), "kv": rep["kv_count"],
                     "rel_residual_initial": rep["rel_residual_initial"]}
    us = _kv_rate(ctx, mesh, "fp64")
    out["kv_fp64_us"] = round(us, 3)
    out["kv_fp64_GDOF_s"] = round(prob.n_dof / us * 1e-3, 3)
    print(json.dumps(out), flush=True)


def run_c3():
    """3D Neo-Hookean box, about 1e6 tets: FP32 HVP rate at the solution;
    zero-start (10 load steps) and warm-start (final step) FP32 Newton
    solves to 1e-8 next to the FP64 reference solve."""
    import synth
    import torch
    from paper_2601_03086_amd import core
    t0 = time.perf_counter()
    prob = synth.box_problem(3, 1003)
    _log(f"# C3 box: {prob.n_elems} tets, {prob.n_dof} DOFs, generated in "
         f"{time.perf_counter() - t0:.1f}s")
    ctx = core.Context(0)
    t0 = time.perf_counter()
    mesh = new_mesh(ctx, prob)
    _log(f"# preprocessed + uploaded in {time.perf_counter() - t0:.1f}s, "
         f"{mesh.info['n_blocks']} blocks of {mesh.info['block_nodes']}")
    uref, rref, tref = _timed_solve(mesh, tol=1e-10, prec="fp64", n_load_steps=10,
                                    device_io=True, history_cap=1)
    _log(f"# FP64 reference (zero start, 10 load steps, 1e-10): {tref:.2f}s "
         f"{rref['newton_iters']} Newton, {rref['kv_count']} HVP")
    uref_h = uref.cpu().numpy()
    u0 = synth.warm_start_guess(uref_h, prob.coords, prob.dir_nodes, seed=3003)
    out = {"config": f"C3 Neo-Hookean box, {prob.n_elems} tets / {prob.n_dof} DOFs",
           "fp64_zero_1e-10": {"s": round(tref, 3), "newton": rref["newton_iters"],
                               "hvp": rref["kv_count"], "status": rref["status_name"]}}
    for name, guess in (("zero", None), ("warm", u0)):
        if name == "warm":   # the solver's own HVP launches (element state cached per step)
            ctx.set_timing([FAM_APPLY])
            ctx.reset_timing()
        u, rep, t = _timed_solve(mesh, u0=guess, tol=1e-8, prec="fp32", n_load_steps=10,
                                 history_cap=1)
        if name == "warm":
            n_h, ms_h = ctx.kernel_time(FAM_APPLY)
            ctx.set_timing(())
            out["hvp_cached_in_warm_solve_us"] = round(ms_h / max(n_h, 1) * 1e3, 2)
            out["hvp_cached_launches_timed"] = n_h
        err = float(np.linalg.norm(u - uref_h) / np.linalg.norm(uref_h))
        out[f"fp32_{name}_1e-8"] = {
            "s": round(t, 3), "newton": rep["newton_iters"], "hvp": rep["kv_count"],
            "load_steps": rep["load_steps_done"], "line_search_evals": rep["line_search_evals"],
            "rel_residual_initial": rep["rel_residual_initial"],
            "rel_residual_final": rep["rel_residual_final"], "rel_err_vs_ref": err,
            "status": rep["status_name"],
            "hvp_GDOF_s_in_solve": round(rep["kv_count"] * prob.n_dof / t / 1e9, 3)}
        _log(f"# FP32 {name}: {t:.2f}s {rep['newton_iters']} Newton {rep['kv_count']} HVP")
    us = _kv_rate(ctx, mesh, "fp32", hvp_state=uref_h)
    b = alg_bytes_kv(prob.n_elems, prob.n_nodes, 3) + 3 * 4 * prob.n_nodes
    out["hvp_fp32_us"] = round(us, 2)
    out["hvp_fp32_GDOF_s"] = round(prob.n_dof / us * 1e-3, 2)
    out["hvp_fp32_alg_GBps"] = round(b / us * 1e-3, 1)
    us_lin = _kv_rate(ctx, mesh, "fp32")
    out["note"] = ("hvp_fp32_us: the stand-alone HVP (element state from the nodal state) at "
                   "the reference solution; hvp_at_zero: the same at u = 0; "
                   "hvp_cached_in_warm_solve_us: the solver's HVP launches, element state "
                   "read from the per-Newton-step cache")
    out["hvp_at_zero_fp32_us"] = round(us_lin, 2)
    print(json.dumps(out), flush=True)


def run_c4():
    """64 plates (5k-20k triangles, alternating linear / Neo-Hookean): the
    differentiable energy, its gradient and an HVP of the whole batch, one
    launch per kernel family."""
    import synth
    import torch
    from paper_2601_03086_amd import _lib as L, core
    members = synth.batch_c4(64)
    ctx = core.Context(0)
    meshes = [new_mesh(ctx, p) for p, _ in members]
    b = core.Batch(ctx, meshes)
    perms = [m.query(L.PFEM_Q_PERM) for m in meshes]
    parts = []
    for (p, u), pr in zip(members, perms):
        o = np.empty_like(u, dtype=np.float64)
        o.reshape(-1, 2)[pr] = u.reshape(-1, 2)
        parts.append(o)
    u = torch.tensor(np.concatenate(parts), device="cuda", dtype=torch.float32)
    v = torch.randn_like(u)
    n_dof = b.n_dof
    n_el = sum(p.n_elems for p, _ in members)
    res = {"config": f"C4 batch: 64 plates, {n_el} triangles, {n_dof} DOFs, FP32; "
                     "calls issued on the library stream"}
    torch.cuda.synchronize()
    stream_ctx = torch.cuda.stream(ctx.stream)
    stream_ctx.__enter__()
    for name, fn in (("energy", lambda: b.energy(u)), ("force", lambda: b.force(u)),
                     ("hvp", lambda: b.hvp(u, v))):
        for _ in range(5):
            fn()
        ts = []
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(ctx.stream)
            for _ in range(20):
                fn()
            e1.record(ctx.stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / 20 * 1e3)
        ts.sort()
        us = ts[2]
        res[name] = {"us": round(us, 2), "GDOF_s": round(n_dof / us * 1e-3, 2)}
    stream_ctx.__exit__(None, None, None)
    res["fwd_bwd_hvp_us"] = round(sum(res[k]["us"] for k in ("energy", "force", "hvp")), 2)
    print(json.dumps(res), flush=True)


def run_homog(n=64, seed=6001):
    """Homogenisation of a 64^3 TPMS cell (solid voxels of the level set, 6
    Kuhn tetrahedra each, periodic springs): the six cell problems solved
    together in FP32 mode to 1e-8 from zero and from warm starts (reference
    fluctuations, FP64 to 1e-11, plus 1% smooth noise), and the batched
    apply of the six right-hand sides, one element visit for all six."""
    import torch
    from synth import tpms
    from synth.fields import rff_field
    from paper_2601_03086_amd import core
    ctx = core.Context(0)
    t0 = time.perf_counter()
    cell = tpms.tpms_cell(seed, n=n)
    m = core.Mesh.from_cell(ctx, cell)
    _log(f"# cell {cell.name}: {cell.n_elems} tets, {len(cell.pairs)} pairs, "
         f"prepared in {time.perf_counter() - t0:.1f}s")
    Xr, EHr, _ = core.homogenize(m, tol=1e-11, prec="fp64")
    noise = np.stack([rff_field(cell.coords, seed + 10 + k, 0.2, 64, n_comp=3).reshape(-1)
                      for k in range(6)])
    noise[:, 3 * cell.pin:3 * cell.pin + 3] = 0.0
    u0 = Xr + (0.01 * np.linalg.norm(Xr, axis=1) / np.linalg.norm(noise, axis=1))[:, None] * noise
    out = {"cell": {**cell.meta, "tets": cell.n_elems, "nodes": cell.n_nodes,
                    "pairs": int(len(cell.pairs)), "block_nodes": m.info["block_nodes"]}}
    for name, start in (("zero", None), ("warm", u0)):
        core.homogenize(m, u0=start, tol=1e-8, prec="fp32")          # warm-up
        ctx.set_timing([FAM_APPLY])
        ctx.reset_timing()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        X, EH, reps = core.homogenize(m, u0=start, tol=1e-8, prec="fp32")
        t = time.perf_counter() - t1
        k = ctx.kernel_stats(FAM_APPLY)
        ctx.set_timing(())
        out[name] = {"ms": round(t * 1e3, 1), "kv": [r["kv_count"] for r in reps],
                     "status": [r["status_name"] for r in reps],
                     "EH_rel_err_vs_fp64": float(np.abs(EH - EHr).max() / np.abs(EHr).max()),
                     "apply": {"launches": k["launches_run"],
                               "avg_us": round(k["total_ms"] / max(k["launches_run"], 1) * 1e3, 2),
                               "alg_GBps": round(k["alg_bytes"] / (k["total_ms"] * 1e-3) / 1e9, 1)
                               if k["total_ms"] else 0.0}}
    out["EH"] = np.round(EHr, 6).tolist()
    print(json.dumps({"config": "homogenisation of a TPMS cell", **out}), flush=True)


def run_sweep(spec):
    """K.v roofline sweep over generator meshes of the given sizes
    ("2d:2e5,3d:1e6,..." = element counts)."""
    import torch
    import synth
    from paper_2601_03086_amd import core
    ctx = core.Context(0)
    # practical ceiling: a 1 GiB device-to-device copy (reads + writes)
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    gbs = 2 * a.numel() * 4 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    print(json.dumps({"copy_1GiB_GBps": round(gbs, 1),
                      "frac_of_8TBps": round(gbs / HBM_PEAK_GBS, 3)}), flush=True)
    del a, b
    for item in spec.split(","):
        kind, n = item.split(":")
        n = float(n)
        t0 = time.perf_counter()
        if kind == "2d":
            nx = int(round((n / 2) ** 0.5))
            prob = synth.structured_plate(nx, nx, seed=7)
        else:
            nx = int(round((n / 24) ** (1 / 3)))
            prob = synth.structured_box(nx, nx, 4 * nx, seed=7)
        _log(f"# {kind} {prob.n_elems} elements generated in {time.perf_counter() - t0:.1f}s")
        t0 = time.perf_counter()
        mesh = new_mesh(ctx, prob)
        _log(f"# preprocessed + uploaded in {time.perf_counter() - t0:.1f}s")
        d = prob.dim
        for prec in ("fp32", "fp64"):
            s = 4 if prec == "fp32" else 8
            us = _kv_rate(ctx, mesh, prec, reps=50, trials=5, warm=5)
            b_alg = alg_bytes_kv(prob.n_elems, prob.n_nodes, d, s=s, s_m=s)
            print(json.dumps({
                "mesh": f"{kind} {prob.n_elems} elems {prob.n_nodes} nodes", "prec": prec,
                "block_nodes": mesh.info["block_nodes"],
                "visits_per_elem": round(mesh.info["owner_elem_visits"] / prob.n_elems, 3),
                "alg_bytes": b_alg, "avg_us": round(us, 2),
                "alg_GBps": round(b_alg / us * 1e-3, 1),
                "frac_hbm": round(b_alg / us * 1e-3 / HBM_PEAK_GBS, 4),
                "GDOF_s": round(prob.n_dof / us * 1e-3, 2)}), flush=True)
        mesh.close()
        del prob, mesh
        torch.cuda.empty_cache()


def run_rotate(copies, kind="c2"):
    """K.v over `copies` distinct device copies of the plate (or the 3D box),
    applied round-robin so that no copy is in a cache when it is applied."""
    import torch
    import synth
    from paper_2601_03086_amd import core
    ctx = core.Context(0)
    prob = c2_problem() if kind == "c2" else synth.box_problem(3, 1003, model="lin_3d")
    meshes, xs, ys = [], [], []
    t0 = time.perf_counter()
    for i in range(copies):
        m = new_mesh(ctx, prob)
        meshes.append(m)
        xs.append(m.permute(torch.randn(prob.n_dof, dtype=torch.float32, device="cuda"),
                            True, "fp32"))
        ys.append(torch.empty_like(xs[-1]))
        if i % 16 == 15:
            _log(f"# {i + 1} copies in {time.perf_counter() - t0:.1f}s")
    d = prob.dim
    b_alg = alg_bytes_kv(prob.n_elems, prob.n_nodes, d)
    ws = b_alg * copies
    for r in range(2):
        for m, x, y in zip(meshes, xs, ys):
            m.apply_K(x, prec="fp32", layout="internal", out=y)
    ts = []
    for _ in range(5):
        ctx.set_timing([FAM_APPLY])
        ctx.reset_timing()
        for r in range(3):
            for m, x, y in zip(meshes, xs, ys):
                m.apply_K(x, prec="fp32", layout="internal", out=y)
        n, ms = ctx.kernel_time(FAM_APPLY)
        ts.append(ms / n * 1e3)
    ctx.set_timing(())
    ts.sort()
    us = ts[2]
    print(json.dumps({"mesh": f"{kind} x {copies} copies", "working_set_alg_bytes": ws,
                      "avg_us": round(us, 2), "alg_GBps": round(b_alg / us * 1e-3, 1),
                      "frac_hbm": round(b_alg / us * 1e-3 / HBM_PEAK_GBS, 4),
                      "GDOF_s": round(prob.n_dof / us * 1e-3, 2)}), flush=True)


# ------------------------------------------------------------ serving (C5)
SERVE_BUDGET_GB = 96      # device memory the server may hold for live solves
SERVE_SLOTS = 128         # live solves at once (512-request stream, warm: 64 slots
                          # 55.6 solves/s, 128 57.6, 256 56.6; one run each)
VERIFY_N = 16             # served results checked by the oracle
VERIFY_MAX_ELEMS = 30000  # ... drawn among requests of at most this size
CPU_SAMPLE_N = 24         # the oracle's timed sample: the first plates of the
CPU_SAMPLE_MAX_ELEMS = 100000   # stream with at most this many triangles


def _gen_request(desc):
    """Worker process: one request's problem and its unscaled warm-start
    noise (the scale needs the reference solution)."""
    import synth
    p = synth.serving_problem(desc)
    noise = synth.warm_start_noise(p.coords, p.dir_nodes, seed=desc["seed"] + 7,
                                   n_features=synth.SERVING_NOISE_FEATURES)
    return desc["id"], p, noise


def _host_workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def gen_stream(n_requests, rate):
    """The stream's request descriptors, problems and warm-start noises,
    generated in worker processes (largest first) before any GPU use."""
    import multiprocessing as mp
    import synth
    descs = synth.serving_stream(n_requests=n_requests, rate=rate)
    order = sorted(range(len(descs)), key=lambda i: -descs[i]["target_elems"])
    probs, noises = [None] * len(descs), [None] * len(descs)
    with mp.get_context("fork").Pool(_host_workers()) as pool:
        for i, p, nz in pool.imap_unordered(_gen_request, [descs[i] for i in order]):
            probs[i], noises[i] = p, nz
    return descs, probs, noises


def host_meshes(probs, block_nodes=None):
    """Finalized host-only meshes (the server uploads them on admission).
    block_nodes: {dim: nodes per owner block} (0 or missing: the library's
    automatic size); None: the --block-nodes value for every mesh."""
    import concurrent.futures as cf
    from paper_2601_03086_amd import core
    bn = (lambda p: BLOCK_NODES) if block_nodes is None else (lambda p: block_nodes.get(p.dim, 0))
    with cf.ThreadPoolExecutor(4) as ex:
        return list(ex.map(lambda p: core.Mesh.from_problem(None, p, bn(p), ORDER), probs))


def _solve_kw(p, tol, prec, precond="jacobi"):
    kw = dict(tol=tol, prec=prec, precond=precond)
    if p.nonlinear:
        kw["n_load_steps"] = p.n_load_steps
    return kw


def serve(ctx, meshes, probs, u0s, t_arrive, ids, tol=1e-8, prec="fp32", timing=False,
          keep=(), budget_gb=SERVE_BUDGET_GB, slots=None, precond="jacobi"):
    """Open-loop replay: request ids[k] is submitted at t_arrive[k] seconds
    after the server starts (u0s None: zero start).  Returns per-request
    reports (library timestamps: submission, admission, completion), the
    solutions of the ids in `keep`, server statistics and, with timing, the
    kernel statistics of the apply and fused-iteration families."""
    from paper_2601_03086_amd import core
    srv = core.Server(ctx, int(budget_gb * (1 << 30)),
                      max_slots=SERVE_SLOTS if slots is None else slots)
    if timing:
        srv.set_timing([FAM_APPLY, FAM_FUSED])
    n = len(ids)
    res, sols = {}, {}
    nxt = 0
    t0 = time.perf_counter()
    last_log = t0
    while len(res) < n:
        now = time.perf_counter() - t0
        while nxt < n and t_arrive[nxt] <= now:
            i = ids[nxt]
            srv.submit(i, meshes[i], u0=None if u0s is None else u0s[i],
                       **_solve_kw(probs[i], tol, prec, precond))
            nxt += 1
        for rid in srv.poll():
            u, r = srv.result(rid)
            res[rid] = r
            if rid in keep:
                sols[rid] = u
        if time.perf_counter() - last_log > 20:
            last_log = time.perf_counter()
            _log(f"#   {len(res)}/{n} done at {now:.1f}s")
        time.sleep(0.0003)
    st = srv.stats()
    ks = {}
    if timing:
        ks = {nm: srv.kernel_stats(f) for f, nm in ((FAM_APPLY, "apply"),
                                                   (FAM_FUSED, "fused_iter"))}
    srv.close()
    return res, sols, st, ks


def stream_summary(res, probs, ids):
    lat = np.sort([res[i]["t_done"] - res[i]["t_submit"] for i in ids])
    t_first = min(res[i]["t_submit"] for i in ids)
    t_last = max(res[i]["t_done"] for i in ids)
    wall = t_last - t_first
    kv = sum(res[i]["kv_count"] for i in ids)
    gdof = sum(res[i]["kv_count"] * probs[i].n_dof for i in ids) / wall / 1e9
    bad = [i for i in ids if res[i]["status"] not in (0, 2)]
    return {"solves_per_s": round(len(ids) / wall, 2), "wall_s": round(wall, 3),
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 1),
                           "p99": round(float(np.percentile(lat, 99)) * 1e3, 1),
                           "max": round(float(lat[-1]) * 1e3, 1)},
            "kv_per_request": round(kv / len(ids), 1), "kv_GDOF_s": round(gdof, 3),
            "failed": len(bad),
            "worst_rel_residual": max(res[i]["rel_residual_final"] for i in ids)}


def sequential(ctx, meshes, probs, u0s, ids, tol=1e-8, prec="fp32"):
    """The same requests solved one at a time with pfem_solve (mesh upload
    untimed, solve timed with its device-synchronising return)."""
    import torch
    tt, kv, lat = 0.0, 0, []
    for i in ids:
        m = meshes[i]
        m.upload(ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rep, _ = m.solve(u0=None if u0s is None else u0s[i], history_cap=1,
                            **_solve_kw(probs[i], tol, prec))
        dt = time.perf_counter() - t0
        m.release_device()
        assert rep["status"] in (0, 2), rep
        tt += dt
        kv += rep["kv_count"]
        lat.append(dt)
    return {"solves_per_s": round(len(ids) / tt, 2), "mean_ms": round(tt / len(ids) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 1),
            "kv_per_request": round(kv / len(ids), 1)}, lat


def batch_kv_point(ctx, meshes, probs, ids, prec, reps=20):
    """One batched K.v (HVP at u = 0 for Neo-Hookean meshes) over many
    resident meshes: a working set beyond the caches, every mesh a
    distinct seeded plate or box of the stream."""
    import torch
    from paper_2601_03086_amd import core
    ms = [meshes[i] for i in ids]
    for m in ms:
        m.upload(ctx)
    b = core.Batch(ctx, ms)
    dt = torch.float32 if prec == "fp32" else torch.float64
    x = torch.randn(b.n_dof, dtype=dt, device="cuda")
    nl = any(probs[i].nonlinear for i in ids)
    u = torch.zeros_like(x) if nl else None
    for _ in range(3):
        b.hvp(u, x, prec=prec)
    ctx.set_timing([FAM_APPLY])
    ctx.reset_timing()
    for _ in range(reps):
        b.hvp(u, x, prec=prec)
    n, t_ms = ctx.kernel_time(FAM_APPLY)
    ctx.set_timing(())
    us = t_ms / n * 1e3
    s = 4 if prec == "fp32" else 8
    b_alg = sum(alg_bytes_kv(probs[i].n_elems, probs[i].n_nodes, probs[i].dim, s=s, s_m=s)
                + (probs[i].dim * s * probs[i].n_nodes if probs[i].nonlinear else 0)
                for i in ids)
    b.close()
    for m in ms:
        m.release_device()
    n_dof = sum(probs[i].n_dof for i in ids)
    return {"meshes": len(ids), "elements": int(sum(probs[i].n_elems for i in ids)),
            "dim": probs[ids[0]].dim, "prec": prec,
            "op": "HVP at u=0 (Neo-Hookean)" if nl else "K.v (linear)",
            "alg_bytes": int(b_alg), "avg_us": round(us, 1),
            "alg_GBps": round(b_alg / (us * 1e-6) / 1e9, 1),
            "frac_hbm": round(b_alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "GDOF_s": round(n_dof / (us * 1e-6) / 1e9, 2)}


def _verify_one(args):
    """Oracle check of one served result (worker process): the oracle's
    relative residual of the served field, and its distance to the
    oracle's own solution (direct solve for linear plates, Newton with the
    request's load steps for Neo-Hookean boxes)."""
    i, p, u = args
    import scipy.sparse.linalg as spla
    from oracle import fe, solve as osolve
    om = fe.Model(p)
    if not p.nonlinear:
        Kff, Ff, uD = osolve.reduced_system(om)
        ud = uD.copy()
        ud[om.free_dofs] = spla.spsolve(Kff.tocsc(), Ff)
        rho = osolve.relative_residual(Kff, Ff, u[om.free_dofs])
    else:
        den = np.linalg.norm(om.gradient(om.lifted(1.0))[om.free_dofs])
        rho = np.linalg.norm(om.gradient(u)[om.free_dofs]) / den
        ud, _ = osolve.newton(p, tol=1e-11, n_load_steps=p.n_load_steps)
    err = float(np.linalg.norm(u - ud) / np.linalg.norm(ud))
    return i, float(rho), err


def verify_subset(probs, sols, ids):
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(len(ids), _host_workers())) as pool:
        out = pool.map(_verify_one, [(i, probs[i], sols[i]) for i in ids], chunksize=1)
    rho = max(o[1] for o in out)
    err = max(o[2] for o in out)
    return {"requests": len(ids), "ids": [int(o[0]) for o in out],
            "plates": sum(1 for i in ids if not probs[i].nonlinear),
            "boxes": sum(1 for i in ids if probs[i].nonlinear),
            "worst_oracle_rel_residual": rho, "worst_rel_error_vs_oracle_solution": err,
            "pass": bool(rho <= 1.05e-8 and err <= 1e-5)}


def cpu_sample_worker(path):
    """The FP64 oracle timed on one host core: Jacobi-PCG (scipy CSR SpMV)
    from each sampled plate's warm start to 1e-8 (problems and guesses read
    from the .npz written by the parent)."""
    from oracle import fe, solve as osolve
    import synth
    d = np.load(path, allow_pickle=False)
    n = int(d["n"])
    t_total, kv_total = 0.0, 0
    for k in range(n):
        p = synth.serving_problem({"id": int(d["ids"][k]), "kind": "2d",
                                   "target_elems": float(d["targets"][k]),
                                   "seed": int(d["seeds"][k])})
        u0 = d[f"u0_{k}"]
        m = fe.Model(p)
        Kff, Ff, _ = osolve.reduced_system(m)
        t0 = time.perf_counter()
        _, hist, kv, st = osolve.pcg(Kff, Ff, u0[m.free_dofs], 1e-8, max_iter=20000)
        t_total += time.perf_counter() - t0
        kv_total += kv
    print(json.dumps({"seconds": t_total, "solves": n, "kv": kv_total, "threads": 1}))


def cpu_sample(descs, u0s, ids):
    import tempfile
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "sample.npz")
        arrs = {"n": np.array(len(ids)), "ids": np.array(ids),
                "targets": np.array([descs[i]["target_elems"] for i in ids]),
                "seeds": np.array([descs[i]["seed"] for i in ids])}
        for k, i in enumerate(ids):
            arrs[f"u0_{k}"] = u0s[i]
        np.savez(path, **arrs)
        r = subprocess.run([sys.executable, __file__, "--cpu-sample-worker", path], env=env,
                           capture_output=True, text=True, timeout=900)
    line = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or not line:
        return {"error": (r.stderr or r.stdout)[-400:]}
    d = json.loads(line[-1])
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(d["solves"] / d["seconds"], 3), "unit": "solves/s",
            "cores": d["threads"], "kind": "oracle",
            "host": {"cpu_model": model, "affinity_cpus": len(os.sched_getaffinity(0)),
                     "threads_env": {k: env[k] for k in ("OMP_NUM_THREADS",
                                                         "OPENBLAS_NUM_THREADS",
                                                         "MKL_NUM_THREADS")}},
            "sample": (f"oracle FP64 Jacobi-PCG (scipy CSR SpMV, 1 thread) on the first "
                       f"{d['solves']} plates of the stream with <= {CPU_SAMPLE_MAX_ELEMS} "
                       f"triangles, each from its warm start to 1e-8: {d['kv']} K.v "
                       f"products in {d['seconds']:.1f} s")}


def serve_block_nodes(args):
    """Owner-block size of the served meshes, per dimension.  A served
    launch batches many meshes, so it has workgroups enough for the chip
    whatever their size, and bigger blocks spread each workgroup's fixed
    costs (partial sums, scalars, task descriptor) over more elements; a
    single latency-bound solve wants the library's smaller automatic blocks
    (the 200k-triangle plate: 58 ms at 224 nodes, 63 at 512, 90 at 1024)."""
    if args.block_nodes:
        return {2: args.block_nodes, 3: args.block_nodes}
    d2, d3 = (int(x) for x in args.serve_block_nodes.split(","))
    return {2: d2, 3: d3}


def run_c5(args):
    """The serving stream as the headline (see the module docstring)."""
    import torch
    import synth
    from paper_2601_03086_amd import core
    n_req, rate = args.requests, args.rate
    t_setup = time.perf_counter()
    descs, probs, noises = gen_stream(n_req, rate)
    n_el = np.array([p.n_elems for p in probs])
    _log(f"# generated {n_req} meshes ({int(n_el.sum())} elements, "
         f"{sum(p.dim == 2 for p in probs)} plates) in {time.perf_counter() - t_setup:.1f}s")
    t1 = time.perf_counter()
    meshes = host_meshes(probs, serve_block_nodes(args))
    _log(f"# preprocessed on the host in {time.perf_counter() - t1:.1f}s")
    ctx = core.Context(0)
    ids = list(range(n_req))
    t_arr = [d["t_arrive"] for d in descs]
    # references (untimed): every request from zero, FP64, to 1e-11, batched
    t1 = time.perf_counter()
    ref, refsol, _, _ = serve(ctx, meshes, probs, None, [0.0] * n_req, ids, tol=1e-11,
                              prec="fp64", keep=set(ids))
    bad = [i for i in ids if ref[i]["status"] != 0]
    assert not bad, ("reference solves failed", bad[:5], ref[bad[0]])
    u0s = [synth.warm_start_guess(refsol[i], probs[i].coords, probs[i].dir_nodes, 0,
                                  noise=noises[i]) for i in ids]
    del refsol
    _log(f"# references in {time.perf_counter() - t1:.1f}s")
    # warm-up: the first W windows of the stream, untimed
    w_ids = ids[:min(n_req, -(-args.warmup * n_req // args.steps))]
    if w_ids:
        serve(ctx, meshes, probs, u0s, t_arr[:len(w_ids)], w_ids)
    _log(f"# setup {time.perf_counter() - t_setup:.1f}s")
    # the timed stream: K windows of arrivals, one continuous replay
    rng = np.random.default_rng(5997)
    small = [i for i in ids if n_el[i] <= (VERIFY_MAX_ELEMS if probs[i].dim == 2
                                             else VERIFY_MAX_ELEMS * 2 // 3)]
    vset = sorted(rng.choice(small, size=min(VERIFY_N, len(small)), replace=False).tolist())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res_w, sols, st_w, ks = serve(ctx, meshes, probs, u0s, t_arr, ids, timing=True,
                                  keep=set(vset))
    torch.cuda.synchronize()
    t_timed = time.perf_counter() - t0
    warm = stream_summary(res_w, probs, ids)
    _log(f"# warm stream: {warm}")
    worker = {k: round(st_w[k], 3) for k in ("admit_s", "tick_s", "complete_s")}
    _log(f"# worker time: {worker}")
    fk = ks["fused_iter"]
    _log(f"# fused iteration: {fk}")
    if args.stream_only:       # profiling runs: setup, warm-up and the timed stream
        print(json.dumps({"served_warm": warm, "fused_iter": fk, "apply": ks["apply"],
                          "worker_s": worker,
                          "ms_per_step": round(t_timed / args.steps * 1e3, 3)}), flush=True)
        return
    res_z, _, st_z, _ = serve(ctx, meshes, probs, None, t_arr, ids)
    zero = stream_summary(res_z, probs, ids)
    _log(f"# zero-start stream: {zero}")
    # the same arrivals with the two-level preconditioner (rigid-body coarse
    # space per mesh, built on the host ahead of the stream like the rest of
    # each mesh's preprocessing)
    import concurrent.futures as cf
    t1 = time.perf_counter()
    with cf.ThreadPoolExecutor(4) as ex:
        n_c = list(ex.map(lambda m: m.prepare_coarse(), meshes))
    t_coarse = time.perf_counter() - t1
    _log(f"# coarse spaces of {n_req} meshes in {t_coarse:.1f}s (mean {np.mean(n_c):.0f} DOFs)")
    res_tl, _, _, _ = serve(ctx, meshes, probs, u0s, t_arr, ids, precond="two_level")
    warm_tl = stream_summary(res_tl, probs, ids)
    _log(f"# warm stream, two-level: {warm_tl}")
    res_tlz, _, _, _ = serve(ctx, meshes, probs, None, t_arr, ids, precond="two_level")
    zero_tl = stream_summary(res_tlz, probs, ids)
    _log(f"# zero-start stream, two-level: {zero_tl}")
    two_level = {"served_warm": warm_tl, "served_zero_start": zero_tl,
                 "coarse_setup_s_total": round(t_coarse, 1),
                 "coarse_dofs_mean": round(float(np.mean(n_c)), 1)}
    # one request at a time: meshes with the library's automatic blocks,
    # the better choice for a lone solve
    t1 = time.perf_counter()
    meshes_seq = host_meshes(probs, {2: 0, 3: 0})
    _log(f"# automatic-block meshes for the sequential legs in {time.perf_counter() - t1:.1f}s")
    seq_w, lat_sw = sequential(ctx, meshes_seq, probs, u0s, ids)
    _log(f"# sequential warm: {seq_w}")
    seq_z, _ = sequential(ctx, meshes_seq, probs, None, ids)
    for m in meshes_seq:
        m.close()
    del meshes_seq
    _log(f"# sequential zero: {seq_z}")
    plates = [i for i in ids if probs[i].dim == 2]
    boxes = [i for i in ids if probs[i].dim == 3]
    kv_points = [batch_kv_point(ctx, meshes, probs, plates, "fp32"),
                 batch_kv_point(ctx, meshes, probs, plates, "fp64"),
                 batch_kv_point(ctx, meshes, probs, boxes, "fp32")]
    _log(f"# batched K.v: {kv_points}")
    c2 = c2_leg(ctx, args)
    _log(f"# C2: {c2}")
    ver = verify_subset(probs, sols, vset)
    _log(f"# oracle check: {ver}")
    # the dominant kernel of the stream: the fused PCG iteration
    avg_ms = fk["total_ms"] / max(fk["launches_run"], 1)
    achieved = fk["alg_bytes"] / (fk["total_ms"] * 1e-3) / 1e9 if fk["total_ms"] else 0.0
    res = {
        "metric": METRIC,
        "value": warm["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_timed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"serving stream: {n_req} solve requests on {n_req} distinct seeded "
                         f"meshes, Poisson arrivals {rate:g}/s, 70% plane-strain plates with "
                         f"8 holes (linear) / 30% 1x1x4 boxes with 20 voids (Neo-Hookean), "
                         f"1e4-5e5 elements log-uniform, warm starts = reference + 1% smooth "
                         f"noise, tol 1e-8 relative residual, continuous batching under a "
                         f"{SERVE_BUDGET_GB} GiB / {SERVE_SLOTS}-slot budget; one step = one "
                         f"of {args.steps} arrival windows of the one timed stream"),
            "requests": n_req, "elements_total": int(n_el.sum()),
            "owner_block_nodes": {"2d": serve_block_nodes(args)[2] or "auto",
                                  "3d": serve_block_nodes(args)[3] or "auto"},
            "plates": len(plates), "boxes": len(boxes), "rate_per_s": rate, "tol": 1e-8,
            "precision": "fp32 element math and Krylov vectors; fp64 dots, residuals, "
                         "state, line-search energy and det F near compression",
        },
        "latency_ms": warm["latency_ms"],
        "served_warm": warm,
        "served_zero_start": zero,
        "sequential_warm": seq_w,
        "sequential_zero_start": seq_z,
        "server": {"peak_live": st_w["peak_live"], "peak_bytes": st_w["peak_bytes"],
                   "steps": st_w["steps"], "launches": st_w["launches"], "worker_s": worker},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_fcg (fused PCG iteration, batched over live requests)",
            "note": ("HBM is the roof; the batched launches' working sets (alg_bytes_per_"
                     "launch) fit the 256 MB Infinity Cache and each iteration is a chain "
                     "of dependent round trips, so latency keeps it below the roof"),
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "alg_bytes_per_launch": round(fk["alg_bytes"] / max(fk["launches_run"], 1)),
            "avg_launch_us": round(avg_ms * 1e3, 3),
            "launches_timed": fk["launches_timed"],
            "apply": ks["apply"],
        },
        "kv_large_working_set": kv_points,
        "two_level_preconditioner": two_level,
        "c2_plate_solve": c2,
        "oracle_verified": ver,
    }
    if not args.no_cpu_baseline:
        cs = [i for i in ids if probs[i].dim == 2 and n_el[i] <= CPU_SAMPLE_MAX_ELEMS]
        cs = cs[:CPU_SAMPLE_N]
        res["cpu_baseline"] = cpu_sample(descs, u0s, cs)
        res["cpu_baseline"]["gpu_sequential_same_sample_solves_per_s"] = round(
            len(cs) / sum(lat_sw[i] for i in cs), 2)
    print(json.dumps(res), flush=True)


# --------------------------------------------------------------------- main
def setup(args):
    import numpy as np
    import torch
    import synth
    from paper_2601_03086_amd import core
    prob = c2_problem()
    ctx = core.Context(0)
    mesh = new_mesh(ctx, prob, getattr(args, "block_nodes", 0) or 0)
    # reference (untimed): device FP64 solve at 1e-11, then 1% smooth noise
    uref, rep, hist = mesh.solve(tol=1e-11, prec="fp64", device_io=True)
    u0 = synth.warm_start_guess(uref.cpu().numpy(), prob.coords, prob.dir_nodes, seed=3002)
    u0_dev = torch.tensor(u0, device="cuda", dtype=torch.float64)
    return prob, ctx, mesh, u0_dev, uref, hist


def warm_start_prediction(mesh, uref, u0, hist):
    """Iteration saving of the warm start next to the estimate of App. C:
    CG needs about ln(|e0|_A / |e|_A) / R iterations at asymptotic rate R,
    so a start whose error is smaller by |e_zero|_A / |e_warm|_A saves
    ln(|e_zero|_A / |e_warm|_A) / R of them.  R is read off the FP64
    reference solve's residual history (between 1e-2 and 1e-9); the counts
    are FP64 PCG solves to 1e-8 from both starts."""
    import torch
    def anorm(e):
        ke = mesh.apply_K(e, prec="fp64", mask=3)   # free-DOF block of K
        return float(torch.sqrt(torch.dot(e, ke)).item())
    lift = torch.zeros_like(uref)
    e_zero = anorm(uref - lift)
    e_warm = anorm(u0 - uref)
    h = np.asarray(hist)
    k1 = int(np.argmax(h < 1e-2))
    k2 = int(np.argmax(h < 1e-9)) if (h < 1e-9).any() else len(h) - 1
    rate = (np.log(h[k1]) - np.log(h[k2])) / max(k2 - k1, 1)
    _, rz, _ = mesh.solve(u0=None, tol=1e-8, prec="fp64", history_cap=1, device_io=True)
    _, rw, _ = mesh.solve(u0=u0, tol=1e-8, prec="fp64", history_cap=1, device_io=True)
    return {"kv_zero_fp64": rz["kv_count"], "kv_warm_fp64": rw["kv_count"],
            "saving": rz["kv_count"] - rw["kv_count"],
            "predicted_saving": round(float(np.log(e_zero / e_warm) / rate), 1),
            "rate_per_iteration": round(float(rate), 6),
            "error_ratio_A_norm": round(e_zero / e_warm, 2)}


def run_crossover():
    """Warm FP32 solves to 1e-8, fused against classic PCG, on the meshes
    around the automatic choice between them: plates with 8 holes of 600k,
    1M and 2M triangles, Neo-Hookean and linear 1x1x4 boxes of 515k and 1M
    tetrahedra (automatic owner blocks).  The FP64 reference (zero start,
    1e-10, at most 400k products) gives the warm start, reference + 1%
    smooth noise; each form is timed as the median of 3 solves (device
    time on the library stream).  One JSON line per mesh."""
    import numpy as np
    import synth
    from paper_2601_03086_amd import core
    ctx = core.Context(0)
    cases = []
    for tt in (6e5, 1e6, 2e6):
        cases.append(("plate", lambda tt=tt: synth.plate_problem(2, 1002, 2002, target_tris=tt)))
    for npu in (28, 35):
        cases.append(("nh box", lambda npu=npu: synth.box_problem(3, 1003, n_per_unit=npu)))
        cases.append(("lin box", lambda npu=npu: synth.box_problem(3, 1003, n_per_unit=npu,
                                                                   model="lin_3d",
                                                                   n_load_steps=1)))
    for name, make in cases:
        t0 = time.perf_counter()
        prob = make()
        _log(f"# {name}: {prob.n_elems} elements generated in {time.perf_counter() - t0:.1f}s")
        mesh = core.Mesh.from_problem(ctx, prob)
        uref, rref, _ = mesh.solve(tol=1e-10, prec="fp64", max_iter=400000)
        assert rref["status"] == 0, rref
        u0 = synth.warm_start_guess(uref, prob.coords, prob.dir_nodes, seed=3002)
        out = {"config": "fused against classic PCG", "mesh": name, "elems": prob.n_elems,
               "blocks": mesh.info["n_blocks"], "block_nodes": mesh.info["block_nodes"]}
        for kr in ("fused", "classic", "auto"):
            ms = []
            for _ in range(3):
                u, rep, _ = mesh.solve(u0=u0, tol=1e-8, prec="fp32", krylov=kr, max_iter=400000)
                assert rep["status"] == 0 and rep["rel_residual_final"] <= 1e-8, rep
                ms.append(rep["t_device_ms"])
            out[kr] = {"ms": round(float(np.median(ms)), 2), "kv": rep["kv_count"],
                       "newton": rep["newton_iters"],
                       "rel_err": float(np.linalg.norm(u - uref) / np.linalg.norm(uref))}
        mesh.close()
        print(json.dumps(out), flush=True)
    ctx.close()


def run_quad(n=150, n_seq=10):
    """The paper's quadrilateral benchmarks (Sec. 'Nonlinear hyperelasticity'):
    n hyperelastic beams (50 x 50 Q4) and n Cook's membranes (30 x 30 Q8),
    Neo-Hookean plane strain, distinct seeded material fields and tractions.
    Per family: FP64 references (served, zero start, 5 load steps, 1e-10)
    give the warm starts (reference + 1% smooth noise); then all n requests
    are served at once (FP32 mode, 1e-8) from zero with 5 load steps, from
    zero with one load step (the paper's comparison) and from the warm
    starts at the final load; mean Newton iterations and Hessian-vector
    products per request, solves/s, and the HVP kernel's average duration;
    the first n_seq requests also one at a time."""
    import torch
    import synth
    from paper_2601_03086_amd import core
    ctx = core.Context(0)
    out = {}
    for fam, gen in (("beam_q4_50x50", lambda s: synth.beam_problem(s)),
                     ("cook_q8_30x30", lambda s: synth.cook_problem(s))):
        t0 = time.perf_counter()
        probs = [gen(7000 + i) for i in range(n)]
        meshes = host_meshes(probs)
        ids = list(range(n))
        ref, refsol, _, _ = serve(ctx, meshes, probs, None, [0.0] * n, ids, tol=1e-10, slots=64,
                                  prec="fp64", keep=set(ids))
        bad = [(i, ref[i]["status"], ref[i]["newton_iters"], ref[i]["rel_residual_final"])
               for i in ids if ref[i]["status"] != 0]
        assert not bad, (fam, len(bad), bad[:5])
        # smooth noise on the scale of the domain (correlation length 0.2 of
        # its size: the unit-size workloads use 0.2)
        size = float(np.ptp(probs[0].coords, axis=0).max())
        u0s = [synth.warm_start_guess(refsol[i], probs[i].coords, probs[i].dir_nodes, 100 + i,
                                      length=0.2 * size) for i in ids]
        _log(f"# {fam}: {n} meshes and references in {time.perf_counter() - t0:.1f}s")
        res = {"elements": probs[0].n_elems, "dofs": probs[0].n_dof}
        for label, starts, steps in (("zero_5_load_steps", None, 5),
                                     ("zero_1_load_step", None, 1),
                                     ("warm", u0s, 5)):
            for p in probs:
                p.n_load_steps = steps
            torch.cuda.synchronize()
            r, sols, st, ks = serve(ctx, meshes, probs, starts, [0.0] * n, ids, keep={0},
                                    slots=64)
            summ = stream_summary(r, probs, ids)
            summ["newton_per_request"] = round(float(np.mean([r[i]["newton_iters"]
                                                              for i in ids])), 2)
            summ["failed"] = sum(r[i]["status"] != 0 for i in ids)
            if label == "warm":
                # the HVP launches' durations from a second, event-timed run
                _, _, _, ks = serve(ctx, meshes, probs, starts, [0.0] * n, ids, timing=True,
                                    slots=64)
                k = ks["apply"]
                us = k["total_ms"] / max(k["launches_run"], 1) * 1e3
                b = k["alg_bytes"] / max(k["launches_run"], 1)
                summ["hvp_launch"] = {"avg_us": round(us, 3), "alg_bytes": round(b),
                                      "alg_GBps": round(b / us * 1e-3, 1) if us else 0.0}
                err = float(np.linalg.norm(sols[0] - refsol[0]) / np.linalg.norm(refsol[0]))
                summ["rel_error_vs_reference"] = err
            res[label] = summ
            _log(f"# {fam} {label}: {summ}")
        for p in probs:
            p.n_load_steps = 5
        seq_z, _ = sequential(ctx, meshes, probs, None, ids[:n_seq])
        seq_w, _ = sequential(ctx, meshes, probs, u0s, ids[:n_seq])
        res["sequential_zero_5_load_steps"] = seq_z
        res["sequential_warm"] = seq_w
        out[fam] = res
    print(json.dumps({"config": "quad", "requests_per_family": n, **out}), flush=True)
    ctx.close()


def run_kv_only(n, mesh_spec=None, kernel="owner", op="kv", block_nodes=0):
    """n launches of the K.v owner kernel (kernel="owner"; op="hvp": the
    Neo-Hookean Hessian-vector product at a smooth state, strains up to 6%)
    or about n fused PCG iterations of a capped zero-start FP32 solve
    (kernel="fused"), then five 256 MiB copies that calibrate byte
    counters."""
    import torch
    if mesh_spec:
        import synth
        from paper_2601_03086_amd import core
        kind, nx = mesh_spec.split(":")
        nx = int(nx)
        nh = op == "hvp"
        prob = (synth.structured_plate(nx, nx, seed=7,
                                       model="nh_plane_strain" if nh else "lin_plane_strain")
                if kind == "2d" else
                synth.structured_box(nx, nx, 4 * nx, seed=7, model="nh_3d" if nh else "lin_3d"))
        ctx = core.Context(0)
        mesh = new_mesh(ctx, prob, block_nodes)
    else:
        from paper_2601_03086_amd import core
        prob = c2_problem()
        ctx = core.Context(0)
        mesh = new_mesh(ctx, prob)
    if kernel == "fused":
        mesh.solve(u0=None, tol=1e-8, prec="fp32", max_iter=n, history_cap=1, krylov="fused")
    else:
        x = mesh.permute(torch.randn(prob.n_dof, dtype=torch.float32, device="cuda"),
                         True, "fp32")
        y = torch.empty_like(x)
        if op == "hvp":
            X = torch.tensor(prob.coords, device="cuda")
            u = 0.02 * torch.sin(3.0 * X)                      # smooth, strains up to 6%
            ui = mesh.permute(u.reshape(-1).float().contiguous(), True, "fp32")
            for _ in range(n):
                mesh.hvp(ui, x, prec="fp32", layout="internal", out=y)
        else:
            for _ in range(n):
                mesh.apply_K(x, prec="fp32", layout="internal", out=y)
    a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")   # 256 MiB copy
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"kv_launches": n, "copy_bytes": a.numel() * 4}))


def fused_iteration_time(ctx, mesh, prob):
    """(launches, ms) of the fused FP32 PCG iterations of a solve capped at
    600 matvecs from a random start (a nonzero residual on any mesh)."""
    import numpy as np
    from paper_2601_03086_amd import core
    ctx.set_timing([FAM_FUSED])
    ctx.reset_timing()
    try:
        u0 = np.random.default_rng(0).normal(size=prob.n_dof)
        mesh.solve(u0=u0, tol=1e-14, prec="fp32", krylov="fused", max_iter=600,
                   history_cap=1)
    except core.L.PfemError:
        pass                       # the iteration cap ends the solve
    nf, msf = ctx.kernel_time(FAM_FUSED)
    ctx.set_timing(())
    return nf, msf


def run_kv_sweep(sizes, mesh_spec=None):
    """Average K.v time (FP32 and FP64, internal layout) per owner-block size,
    and the average fused PCG iteration of a capped FP32 solve.  mesh_spec:
    None (the 200k-triangle plate) or "2d:NX" / "3d:NX" structured meshes."""
    import numpy as np
    import torch
    from paper_2601_03086_amd import core
    if mesh_spec:
        import synth
        kind, nx = mesh_spec.split(":")
        nx = int(nx)
        prob = (synth.structured_plate(nx, nx, seed=7) if kind == "2d"
                else synth.structured_box(nx, nx, 4 * nx, seed=7))
    else:
        prob = c2_problem()
    ctx = core.Context(0)
    b_alg = alg_bytes_kv(prob.n_elems, prob.n_nodes, prob.dim)
    for bn in sizes:
        mesh = new_mesh(ctx, prob, bn)
        if mesh.info["n_blocks"] > 4096:   # the fused form is for small meshes only
            nf, msf = 0, 0.0
        else:
            nf, msf = fused_iteration_time(ctx, mesh, prob)
        print(json.dumps({"block_nodes": mesh.info["block_nodes"], "order": ORDER,
                          "blocks": mesh.info["n_blocks"], "fused_launches": nf,
                          "fused_avg_us": round(msf / max(nf, 1) * 1e3, 3)}), flush=True)
        for prec in ("fp32", "fp64"):
            dt = torch.float32 if prec == "fp32" else torch.float64
            x = mesh.permute(torch.randn(prob.n_dof, dtype=dt, device="cuda"), True, prec)
            y = torch.empty_like(x)
            for _ in range(20):
                mesh.apply_K(x, prec=prec, layout="internal", out=y)
            ctx.set_timing([FAM_APPLY])
            ctx.reset_timing()
            for _ in range(200):
                mesh.apply_K(x, prec=prec, layout="internal", out=y)
            n, ms = ctx.kernel_time(FAM_APPLY)
            ctx.set_timing(())
            us = ms / n * 1e3
            print(json.dumps({"block_nodes": mesh.info["block_nodes"], "prec": prec,
                              "order": ORDER,
                              "blocks": mesh.info["n_blocks"],
                              "visits_per_elem": round(mesh.info["owner_elem_visits"] / prob.n_elems, 3),
                              "avg_us": round(us, 3),
                              "alg_GBps": round(b_alg / (us * 1e-6) / 1e9, 1)}), flush=True)
        mesh.close()


def run_kv_large(spec, reps=50):
    """K.v at working sets far beyond the caches: structured-topology plates
    and boxes with jittered interior nodes and a random node relabelling
    (so the library's RCM does the ordering work).  spec: "2d:NX,3d:NX"."""
    import numpy as np
    import torch
    import synth
    from paper_2601_03086_amd import core
    ctx = core.Context(0)
    for item in spec.split(","):
        kind, n = item.split(":")
        n = int(n)
        t0 = time.perf_counter()
        if kind == "2d":
            prob = synth.structured_plate(n, n, seed=7)
        else:
            prob = synth.structured_box(n, n, 4 * n, seed=7)
        t_gen = time.perf_counter() - t0
        print(f"# generated {kind} {prob.n_elems} elements in {t_gen:.1f}s", file=sys.stderr,
              flush=True)
        t0 = time.perf_counter()
        mesh = new_mesh(ctx, prob, BLOCK_NODES)
        t_prep = time.perf_counter() - t0
        print(f"# preprocessed in {t_prep:.1f}s", file=sys.stderr, flush=True)
        d = prob.dim
        for prec in ("fp32", "fp64"):
            s = 4 if prec == "fp32" else 8
            dt = torch.float32 if prec == "fp32" else torch.float64
            x = mesh.permute(torch.randn(prob.n_dof, dtype=dt, device="cuda"), True, prec)
            y = torch.empty_like(x)
            for _ in range(5):
                mesh.apply_K(x, prec=prec, layout="internal", out=y)
            ctx.set_timing([FAM_APPLY])
            ctx.reset_timing()
            for _ in range(reps):
                mesh.apply_K(x, prec=prec, layout="internal", out=y)
            nl, ms = ctx.kernel_time(FAM_APPLY)
            ctx.set_timing(())
            us = ms / nl * 1e3
            b_alg = alg_bytes_kv(prob.n_elems, prob.n_nodes, d, s=s, s_m=s)
            print(json.dumps({
                "mesh": f"{kind} {prob.n_elems} elems {prob.n_nodes} nodes",
                "prec": prec, "block_nodes": mesh.info["block_nodes"], "order": ORDER,
                "bandwidth": mesh.info["bandwidth_internal"],
                "visits_per_elem": round(mesh.info["owner_elem_visits"] / prob.n_elems, 3),
                "alg_bytes": b_alg, "avg_us": round(us, 2),
                "alg_GBps": round(b_alg / (us * 1e-6) / 1e9, 1),
                "frac_hbm": round(b_alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                "GDOF_s": round(prob.n_dof / (us * 1e-6) / 1e9, 2),
                "gen_s": round(t_gen, 1), "prep_s": round(t_prep, 1)}), flush=True)
            del x, y
        mesh.close()
        del prob


def run_c2(args):
    """The 200k-triangle plate alone: warm FP32 solves (one JSON line)."""
    import torch
    t_setup = time.perf_counter()
    prob, ctx, mesh, u0, uref, ref_hist = setup(args)
    out = mesh.new_vec("fp64")
    info = mesh.info
    print(f"# setup {time.perf_counter() - t_setup:.1f}s: {prob.n_elems} triangles, "
          f"{prob.n_dof} DOFs, {info['n_blocks']} blocks of {info['block_nodes']} nodes",
          file=sys.stderr, flush=True)
    two_level = args.precond == "two_level"
    if two_level:
        mesh.prepare_coarse()
    opts = dict(tol=1e-8, prec=args.prec, krylov="classic" if two_level else "fused",
                precond=args.precond, device_io=True, out=out, history_cap=1)
    for _ in range(args.warmup):
        mesh.solve(u0=u0, **opts)
    # zero-start reference solve (not timed in the headline)
    _, rz, _ = mesh.solve(u0=None, **opts)
    # the dominant kernel's duration: HIP events around each chunk of
    # consecutive fused-iteration launches of the timed solves (chunks that
    # ran past convergence are discarded), divided by the launches in it
    dom = FAM_APPLY if two_level else FAM_FUSED
    # the classic loop's applies are single launches: time one in 16 so the
    # events do not slow the solves they measure
    ctx.set_timing([dom], sample_every=16 if two_level else 1)
    ctx.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kv_total = 0
    reps = []
    lat = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, rep, _ = mesh.solve(u0=u0, **opts)
        lat.append(time.perf_counter() - ts)
        kv_total += rep["kv_count"]
        reps.append(rep)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    n_apply, ms_apply = ctx.kernel_time(dom)
    k_dom = ctx.kernel_stats(dom)
    # per-family breakdown from two extra solves with every family timed
    ctx.set_timing(range(7))
    ctx.reset_timing()
    for _ in range(2):
        mesh.solve(u0=u0, **opts)
    breakdown = {}
    for f, nm in enumerate(FAM_NAMES):
        n_f, ms_f = ctx.kernel_time(f)
        if n_f:
            breakdown[nm] = {"launches_per_solve": n_f / 2, "avg_us": round(ms_f / n_f * 1e3, 3)}
    ctx.set_timing(())
    # the same warm solves with the three-launch PCG loop, for comparison
    opts["krylov"] = "classic"
    torch.cuda.synchronize()
    tc0 = time.perf_counter()
    n_cls = max(2, args.steps // 4)
    kv_cls = 0
    for _ in range(n_cls):
        _, rc, _ = mesh.solve(u0=u0, **opts)
        kv_cls += rc["kv_count"]
    torch.cuda.synchronize()
    t_cls = time.perf_counter() - tc0
    assert all(r["status"] == 0 and r["rel_residual_final"] <= 1e-8 for r in reps), reps[-1]
    value = kv_total * prob.n_dof / t / 1e9
    avg_ms = ms_apply / max(n_apply, 1)
    s_val = 4 if args.prec == "fp32" else 8
    if two_level:
        b_alg = k_dom["alg_bytes"] / max(k_dom["launches_run"], 1)
        kernel = f"k_owner<2, {'float' if args.prec == 'fp32' else 'double'}, K.v>"
    else:
        b_alg = alg_bytes_fused(prob.n_elems, prob.n_nodes, 2, s=s_val, s_m=s_val)
        kernel = f"k_fcg<2, {'float' if args.prec == 'fp32' else 'double'}, false>"
    achieved = b_alg / (avg_ms * 1e-3) / 1e9
    lat_sorted = sorted(lat)
    res = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": ("plane-strain plate, 8 random holes, "
                         f"{prob.n_elems} P1 triangles / {prob.n_dof} DOFs, lognormal E, "
                         "warm start = reference + 1% smooth noise, "
                         + ("two-level-PCG" if two_level else "Jacobi-PCG") + " to 1e-8 "
                         + ("(FP32 Krylov, FP64 residual refinement)" if args.prec == "fp32"
                            else "(FP64)")
                         + (", classic loop" if two_level else ", fused one-launch iteration")),
            "n_elems": prob.n_elems, "n_dof": prob.n_dof, "tol": 1e-8,
            "precision": ("fp32 element math and Krylov vectors; fp64 dots, residuals, x"
                          if args.prec == "fp32" else "fp64 throughout"),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_entry() if kernel == KERNEL_NAME else None,
            "alg_bytes_per_launch": b_alg,
            "avg_launch_us": round(avg_ms * 1e3, 3),
            "launches_timed": n_apply,
        },
        "solves_per_s": round(args.steps / t, 2),
        "solve_latency_ms": {"p50": round(lat_sorted[len(lat) // 2] * 1e3, 3),
                             "p99": round(lat_sorted[min(len(lat) - 1,
                                                         int(0.99 * len(lat)))] * 1e3, 3)},
        "kernel_breakdown": breakdown,
        "classic_pcg": {"ms_per_solve": round(t_cls / n_cls * 1e3, 3),
                        "GDOF_s": round(kv_cls * prob.n_dof / t_cls / 1e9, 3),
                        "kv_per_solve": kv_cls / n_cls},
        "kv_per_solve_warm": kv_total / args.steps,
        "kv_per_solve_zero": rz["kv_count"],
        "outer_sweeps_warm": reps[-1]["outer_sweeps"],
        "rel_residual_initial_warm": reps[-1]["rel_residual_initial"],
        "warm_start_vs_app_c": warm_start_prediction(mesh, uref, u0, ref_hist),
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline()
    print(json.dumps(res))


def c2_leg(ctx, args, n_solves=5):
    """The 200k-triangle plate (C2) inside the default run: warm solves to
    1e-8 in FP32 mode (fused iteration) and in FP64 (fused), K.v rate and
    time to solution of each, and the fused FP32 iteration's roofline from
    HIP events on the library stream."""
    import torch
    import synth
    prob = c2_problem()
    mesh = new_mesh(ctx, prob)
    uref, _, _ = mesh.solve(tol=1e-11, prec="fp64", device_io=True)
    u0 = torch.tensor(synth.warm_start_guess(uref.cpu().numpy(), prob.coords, prob.dir_nodes,
                                             seed=3002), device="cuda", dtype=torch.float64)
    out = mesh.new_vec("fp64")
    res = {"mesh": f"{prob.n_elems} triangles, {prob.n_dof} DOFs"}
    for prec in ("fp32", "fp64"):
        opts = dict(tol=1e-8, prec=prec, krylov="fused", device_io=True, out=out,
                    history_cap=1)
        for _ in range(2):
            mesh.solve(u0=u0, **opts)
        ctx.set_timing([FAM_FUSED])
        ctx.reset_timing()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kv = 0
        for _ in range(n_solves):
            _, rep, _ = mesh.solve(u0=u0, **opts)
            assert rep["status"] == 0 and rep["rel_residual_final"] <= 1e-8, rep
            kv += rep["kv_count"]
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        k = ctx.kernel_stats(FAM_FUSED)
        ctx.set_timing(())
        us = k["total_ms"] / max(k["launches_run"], 1) * 1e3
        b = k["alg_bytes"] / max(k["launches_run"], 1)
        res[prec] = {"ms_per_solve": round(t / n_solves * 1e3, 2),
                     "kv_per_solve": kv / n_solves,
                     "GDOF_s": round(kv * prob.n_dof / t / 1e9, 2),
                     "fused_iter": {"alg_bytes_per_launch": round(b), "avg_us": round(us, 3),
                                    "alg_GBps": round(b / us * 1e-3, 1),
                                    "frac_hbm": round(b / us * 1e-3 / HBM_PEAK_GBS, 4)}}
    # the two-level preconditioner (rigid-body coarse space on owner blocks):
    # warm and zero starts, FP32 mode, classic loop
    t0 = time.perf_counter()
    n_c = mesh.prepare_coarse()
    res["two_level"] = {"coarse_dofs": n_c, "setup_s": round(time.perf_counter() - t0, 3)}
    for name, start in (("warm", u0), ("zero", None)):
        opts = dict(tol=1e-8, prec="fp32", precond="two_level", device_io=True, out=out,
                    history_cap=1)
        mesh.solve(u0=start, **opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kv = 0
        for _ in range(n_solves):
            _, rep, _ = mesh.solve(u0=start, **opts)
            assert rep["status"] == 0 and rep["rel_residual_final"] <= 1e-8, rep
            kv += rep["kv_count"]
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        res["two_level"][name] = {"ms_per_solve": round(t / n_solves * 1e3, 2),
                                  "kv_per_solve": kv / n_solves}
    for name, start in (("jacobi_zero", None),):
        opts = dict(tol=1e-8, prec="fp32", krylov="fused", device_io=True, out=out, history_cap=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rep, _ = mesh.solve(u0=start, **opts)
        torch.cuda.synchronize()
        res["fp32"][name] = {"ms": round((time.perf_counter() - t0) * 1e3, 2),
                             "kv": rep["kv_count"]}
    mesh.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-worker", action="store_true")
    ap.add_argument("--kv-only", type=int, default=0)
    ap.add_argument("--parse-pmc", default=None)
    ap.add_argument("--kv-sweep", default=None,
                    help="comma-separated owner-block sizes to time K.v with")
    ap.add_argument("--block-nodes", type=int, default=0)
    ap.add_argument("--order", default="blocks", choices=["blocks", "rcm"],
                    help="internal node numbering of every mesh")
    ap.add_argument("--precond", default="jacobi", choices=["jacobi", "two_level"],
                    help="--config c2 preconditioner")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"],
                    help="solve precision (fp32: FP32 Krylov + FP64 refinement)")
    ap.add_argument("--kv-mesh", default=None, help='mesh for --kv-only, e.g. "3d:40"')
    ap.add_argument("--kv-op", default="kv", choices=["kv", "hvp"],
                    help="--kv-only owner kernel: K.v or the Neo-Hookean HVP")
    ap.add_argument("--kv-kernel", default="owner", choices=["owner", "fused"],
                    help="--kv-only: K.v launches or fused PCG iterations")
    ap.add_argument("--kv-large", default=None,
                    help='e.g. "2d:2000,3d:60": K.v roofline sweep on large meshes')
    ap.add_argument("--config", default=None,
                    choices=["c1", "c2", "c3", "c4", "sweep", "rotate", "homog", "quad",
                             "crossover"],
                    help="other workloads (one JSON line each, not the headline)")
    ap.add_argument("--sizes", default="2d:2e5,2d:1e6,2d:4e6,2d:1.6e7,3d:1e6,3d:4e6,3d:1.6e7",
                    help="--config sweep sizes (element counts)")
    ap.add_argument("--copies", type=int, default=192, help="--config rotate copies")
    ap.add_argument("--requests", type=int, default=512, help="serving stream requests")
    ap.add_argument("--rate", type=float, default=200.0, help="serving arrivals per second")
    ap.add_argument("--cpu-sample-worker", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--serve-slots", type=int, default=0,
                    help="live solves at once in the served streams (0: 128)")
    ap.add_argument("--serve-block-nodes", default="768,256",
                    help="owner-block nodes of the served meshes, 2D,3D (0: automatic)")
    ap.add_argument("--stream-only", action="store_true",
                    help="serving: stop after the timed stream (for profiler runs)")
    args = ap.parse_args()
    global SERVE_SLOTS
    if args.serve_slots > 0:
        SERVE_SLOTS = args.serve_slots
    global ORDER, BLOCK_NODES
    ORDER, BLOCK_NODES = args.order, args.block_nodes
    if args.cpu_baseline_worker:
        cpu_baseline_worker()
        return
    if args.cpu_sample_worker:
        cpu_sample_worker(args.cpu_sample_worker)
        return
    if args.parse_pmc:
        d = parse_pmc(args.parse_pmc)
        print(json.dumps(d, indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.kv_only:
        run_kv_only(args.kv_only, args.kv_mesh, args.kv_kernel, args.kv_op, args.block_nodes)
        return
    if args.kv_sweep:
        run_kv_sweep([int(s) for s in args.kv_sweep.split(",")], args.kv_mesh)
        return
    if args.kv_large:
        run_kv_large(args.kv_large)
        return
    if args.config:
        {"c1": run_c1, "c2": lambda: run_c2(args), "c3": run_c3, "c4": run_c4,
         "sweep": lambda: run_sweep(args.sizes),
         "rotate": lambda: run_rotate(args.copies),
         "homog": run_homog, "quad": run_quad,
         "crossover": run_crossover}[args.config]()
        return
    run_c5(args)


if __name__ == "__main__":
    main()
