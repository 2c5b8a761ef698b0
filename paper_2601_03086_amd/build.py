"""Build libpfem.so (HIP for gfx950) in-tree.

    python -m paper_2601_03086_amd.build            # incremental
    python -m paper_2601_03086_amd.build --force    # rebuild everything

Every source under csrc/ is compiled by hipcc for gfx950 and linked into
paper_2601_03086_amd/libpfem.so.  Object files go to _build/ at the
repository root.
"""
import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libpfem.so")
ARCH = os.environ.get("PFEM_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
          "-I" + os.path.join(ROOT, "include")]
DEVICE = ["--offload-arch=" + ARCH, "-munsafe-fp-atomics",
          # no packed-FP32 instructions anywhere in device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def sources():
    out = []
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".cpp")):
            out.append(os.path.join(CSRC, f))
    return out


def headers_mtime():
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hs.append(os.path.join(ROOT, "include", "pfem.h"))
    return max(os.path.getmtime(h) for h in hs)


def compile_one(src, force, hmt):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if (not force and os.path.exists(obj)
            and os.path.getmtime(obj) >= max(os.path.getmtime(src), hmt)):
        return obj, None
    cmd = [hipcc()] + COMMON + DEVICE + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [hipcc()] + COMMON + DEVICE + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        return obj, "FAILED: " + " ".join(cmd) + "\n" + r.stdout + r.stderr
    return obj, r.stderr.strip() or None


def build(force=False, verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    hmt = headers_mtime()
    srcs = sources()
    jobs = jobs or min(8, len(srcs))
    objs, errors = [], []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for obj, msg in ex.map(lambda s: compile_one(s, force, hmt), srcs):
            objs.append(obj)
            if msg and msg.startswith("FAILED"):
                errors.append(msg)
            elif msg and verbose:
                print(msg, file=sys.stderr)
    if errors:
        raise RuntimeError("\n".join(errors))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: " + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    print(build(a.force, a.verbose))


if __name__ == "__main__":
    main()
