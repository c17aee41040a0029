"""Build libns.so (HIP, gfx950) in-tree.

    python -m paper_2603_08892_amd.build          # or build() from Python

hipcc cross-compiles without a GPU.  Every translation unit (the C ABI and the
size-generic passes in ns_host.hip, one unit per specialised grid size) is
compiled to an object file in parallel, then linked.  Packed FP32 instructions
are disabled (-packed-fp32-ops) for every HIP translation unit.
"""

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libns.so")
OBJ = os.path.join(PKG, "_build")


def sources():
    return [os.path.join(CSRC, "ns_host.hip")] + sorted(glob.glob(os.path.join(CSRC, "fast_*.hip")))


def headers():
    return sorted(glob.glob(os.path.join(CSRC, "*.hpp"))) + [os.path.join(ROOT, "include", "ns.h")]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libns.so)")


FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def compile_command(src, obj, extra=()):
    return [hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), *extra, "-c", "-o", obj, src]


def link_command(objs, out):
    return [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out, *objs]


def _obj(src):
    return os.path.join(OBJ, os.path.splitext(os.path.basename(src))[0] + ".o")


def build(verbose=True, jobs=None, only_changed=False, extra=()):
    """Compile every translation unit and link libns.so (atomic replace of the old
    file).  only_changed=True recompiles only units older than their source or any
    header (for development; the default always compiles everything)."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    newest_header = max(os.path.getmtime(h) for h in headers())
    todo = []
    for s in srcs:
        o = _obj(s)
        if only_changed and os.path.exists(o) and os.path.getmtime(o) > max(os.path.getmtime(s), newest_header):
            continue
        todo.append(s)
    jobs = jobs or min(len(todo) or 1, os.cpu_count() or 1, 16)

    def one(s):
        cmd = compile_command(s, _obj(s) + ".tmp", extra)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode == 0:
            os.replace(_obj(s) + ".tmp", _obj(s))
        return s, cmd, r

    failed = []
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        for s, cmd, r in ex.map(one, todo):
            if verbose:
                print(" ".join(cmd), flush=True)
            errs = "\n".join(ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln)
            if errs.strip():
                print(errs, file=sys.stderr, flush=True)
            if r.returncode != 0:
                failed.append(os.path.basename(s))
    if failed:
        raise RuntimeError("compilation failed: " + ", ".join(failed))
    tmp = LIB + ".tmp"
    cmd = link_command([_obj(s) for s in srcs], tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, only_changed="--changed" in sys.argv)
    sys.exit(0)
