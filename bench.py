#!/usr/bin/env python3
"""Benchmark: matrix-free K.v throughput inside warm-started solves (one GPU).

Workload (default): the plane-strain plate with 8 random holes, about 2e5 P1
triangles, lognormal E field, clamped bottom edge and a random traction
segment on the top edge.  One step is one warm-started solve to a 1e-8
relative residual (FP32 Jacobi-PCG with FP64 residual refinement), starting
from a synthetic network prediction (reference solution + 1% smooth noise).
Inputs are resident in device memory before the timed region.

value = sum over timed solves of (K.v products * n_dof) / wall time, in
GDOF/s.  The PCG runs in its fused form: one launch per iteration does the
element pass (K.v) and every vector update.  The roofline object
describes that kernel: algorithmic bytes per launch (K.v inputs plus the
fused vector pass) divided by its average launch time, measured with HIP
events on the library stream during the timed solves.

Other modes (not the default line):
  --kv-only N        N back-to-back K.v launches, or with --kv-kernel fused
                     about N fused PCG iterations (for rocprofv3 counters)
  --parse-pmc DIR    turn rocprofv3 FETCH_SIZE / WRITE_SIZE CSVs into the
                     traffic summary under profiles/
"""
import argparse
import glob
import hashlib
import json
import os
import subprocess
import sys
import time

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


def kernel_hash():
    h = hashlib.sha256()
    for f in ("elem_kernels.hip", "elem_math.h", "reduce.h", "pfem_internal.h"):
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
def cpu_baseline_worker():
    """The FP64 oracle timed on host cores: Jacobi-PCG (scipy CSR SpMV) from
    the same warm start to 1e-8, capped at 3000 K.v products."""
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
    x, hist, kv, st = osolve.pcg(Kff, Ff, u0[m.free_dofs], 1e-8, max_iter=3000)
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
    return {"value": d["kv"] * d["n_dof"] / d["seconds"] / 1e9, "unit": "GDOF/s",
            "cores": d["threads"], "kind": "oracle",
            "sample": (f"oracle FP64 Jacobi-PCG (scipy CSR SpMV) on the same plate, "
                       f"same warm start, to 1e-8: {d['kv']} K.v products in "
                       f"{d['seconds']:.1f} s (status {d['status']}, final rel "
                       f"{d['final_rel']:.1e}); 1 thread")}


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


# --------------------------------------------------------------------- main
def setup(args):
    import numpy as np
    import torch
    import synth
    from paper_2601_03086_amd import core
    prob = c2_problem()
    ctx = core.Context(0)
    mesh = core.Mesh.from_problem(ctx, prob, getattr(args, "block_nodes", 0) or 0)
    # reference (untimed): device FP64 solve at 1e-11, then 1% smooth noise
    uref, rep, _ = mesh.solve(tol=1e-11, prec="fp64", device_io=True)
    u0 = synth.warm_start_guess(uref.cpu().numpy(), prob.coords, prob.dir_nodes, seed=3002)
    u0_dev = torch.tensor(u0, device="cuda", dtype=torch.float64)
    return prob, ctx, mesh, u0_dev


def run_kv_only(n, mesh_spec=None, kernel="owner"):
    """n launches of the K.v owner kernel (kernel="owner") or about n fused
    PCG iterations of a capped zero-start FP32 solve (kernel="fused"), then
    five 256 MiB copies that calibrate byte counters."""
    import torch
    if mesh_spec:
        import synth
        from paper_2601_03086_amd import core
        kind, nx = mesh_spec.split(":")
        nx = int(nx)
        prob = (synth.structured_plate(nx, nx, seed=7) if kind == "2d"
                else synth.structured_box(nx, nx, 4 * nx, seed=7))
        ctx = core.Context(0)
        mesh = core.Mesh.from_problem(ctx, prob)
    else:
        from paper_2601_03086_amd import core
        prob = c2_problem()
        ctx = core.Context(0)
        mesh = core.Mesh.from_problem(ctx, prob)
    if kernel == "fused":
        mesh.solve(u0=None, tol=1e-8, prec="fp32", max_iter=n, history_cap=1)
    else:
        x = mesh.permute(torch.randn(prob.n_dof, dtype=torch.float32, device="cuda"),
                         True, "fp32")
        y = torch.empty_like(x)
        for _ in range(n):
            mesh.apply_K(x, prec="fp32", layout="internal", out=y)
    a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")   # 256 MiB copy
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"kv_launches": n, "copy_bytes": a.numel() * 4}))


def run_kv_sweep(sizes):
    """Average K.v time (FP32 and FP64, internal layout) per owner-block size."""
    import torch
    from paper_2601_03086_amd import core
    prob = c2_problem()
    ctx = core.Context(0)
    b_alg = alg_bytes_kv(prob.n_elems, prob.n_nodes, 2)
    for bn in sizes:
        mesh = core.Mesh.from_problem(ctx, prob, bn)
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
        mesh = core.Mesh.from_problem(ctx, prob)
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
                "prec": prec, "block_nodes": mesh.info["block_nodes"],
                "visits_per_elem": round(mesh.info["owner_elem_visits"] / prob.n_elems, 3),
                "alg_bytes": b_alg, "avg_us": round(us, 2),
                "alg_GBps": round(b_alg / (us * 1e-6) / 1e9, 1),
                "frac_hbm": round(b_alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                "GDOF_s": round(prob.n_dof / (us * 1e-6) / 1e9, 2),
                "gen_s": round(t_gen, 1), "prep_s": round(t_prep, 1)}), flush=True)
            del x, y
        mesh.close()
        del prob


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-worker", action="store_true")
    ap.add_argument("--kv-only", type=int, default=0)
    ap.add_argument("--parse-pmc", default=None)
    ap.add_argument("--kv-sweep", default=None,
                    help="comma-separated owner-block sizes to time K.v with")
    ap.add_argument("--block-nodes", type=int, default=0)
    ap.add_argument("--kv-mesh", default=None, help='mesh for --kv-only, e.g. "3d:40"')
    ap.add_argument("--kv-kernel", default="owner", choices=["owner", "fused"],
                    help="--kv-only: K.v launches or fused PCG iterations")
    ap.add_argument("--kv-large", default=None,
                    help='e.g. "2d:2000,3d:60": K.v roofline sweep on large meshes')
    args = ap.parse_args()
    if args.cpu_baseline_worker:
        cpu_baseline_worker()
        return
    if args.parse_pmc:
        d = parse_pmc(args.parse_pmc)
        print(json.dumps(d, indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build never uses a second GPU); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.kv_only:
        run_kv_only(args.kv_only, args.kv_mesh, args.kv_kernel)
        return
    if args.kv_sweep:
        run_kv_sweep([int(s) for s in args.kv_sweep.split(",")])
        return
    if args.kv_large:
        run_kv_large(args.kv_large)
        return
    import torch
    t_setup = time.perf_counter()
    prob, ctx, mesh, u0 = setup(args)
    out = mesh.new_vec("fp64")
    info = mesh.info
    print(f"# setup {time.perf_counter() - t_setup:.1f}s: {prob.n_elems} triangles, "
          f"{prob.n_dof} DOFs, {info['n_blocks']} blocks of {info['block_nodes']} nodes",
          file=sys.stderr, flush=True)
    opts = dict(tol=1e-8, prec="fp32", device_io=True, out=out, history_cap=1)
    for _ in range(args.warmup):
        mesh.solve(u0=u0, **opts)
    # zero-start reference solve (not timed in the headline)
    _, rz, _ = mesh.solve(u0=None, **opts)
    # the dominant kernel's duration: HIP events around each chunk of
    # consecutive fused-iteration launches of the timed solves (chunks that
    # ran past convergence are discarded), divided by the launches in it
    ctx.set_timing([FAM_FUSED])
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
    n_apply, ms_apply = ctx.kernel_time(FAM_FUSED)
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
    torch.cuda.synchronize()
    tc0 = time.perf_counter()
    n_cls = max(2, args.steps // 4)
    kv_cls = 0
    for _ in range(n_cls):
        _, rc, _ = mesh.solve(u0=u0, krylov="classic", **opts)
        kv_cls += rc["kv_count"]
    torch.cuda.synchronize()
    t_cls = time.perf_counter() - tc0
    assert all(r["status"] == 0 and r["rel_residual_final"] <= 1e-8 for r in reps), reps[-1]
    value = kv_total * prob.n_dof / t / 1e9
    avg_ms = ms_apply / max(n_apply, 1)
    b_alg = alg_bytes_fused(prob.n_elems, prob.n_nodes, 2)
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
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("plane-strain plate, 8 random holes, "
                         f"{prob.n_elems} P1 triangles / {prob.n_dof} DOFs, lognormal E, "
                         "warm start = reference + 1% smooth noise, Jacobi-PCG to 1e-8 "
                         "(FP32 Krylov, FP64 residual refinement)"),
            "n_elems": prob.n_elems, "n_dof": prob.n_dof, "tol": 1e-8,
            "precision": "fp32 element math and Krylov vectors; fp64 dots, residuals, x",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": KERNEL_NAME,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_entry(),
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
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
