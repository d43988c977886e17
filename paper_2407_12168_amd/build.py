"""Builds libensf.so (HIP kernels for gfx950 + the C-ABI host code) in-tree.

    python -m paper_2407_12168_amd.build [--jobs N]

Every HIP translation unit is compiled with packed-FP32 instruction selection disabled
(the code has no hand-written packed-FP32 arithmetic, and the compiler is told not to
form those instructions either).
"""
import argparse
import hashlib
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libensf.so")
ARCH = os.environ.get("ENSF_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
HIP_FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-munsafe-fp-atomics"]


def sources():
    out = []
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".hip"):
            out.append((os.path.join(CSRC, name), True))
        elif name.endswith(".cpp"):
            out.append((os.path.join(CSRC, name), False))
    return out


_QUOTE_INCLUDE = re.compile(r'^\s*#\s*include\s+"([^"]+)"', re.M)


def _local_headers(src):
    """The project headers `src` includes with #include "...", transitively."""
    seen, todo = set(), [src]
    while todo:
        f = todo.pop()
        with open(f) as fh:
            names = _QUOTE_INCLUDE.findall(fh.read())
        for n in names:
            h = os.path.normpath(os.path.join(os.path.dirname(f), n))
            if os.path.exists(h) and h not in seen:
                seen.add(h)
                todo.append(h)
    return sorted(seen)


def _digest(src, cmd):
    """Hash of the command and of the source and included header texts as read before
    compiling."""
    h = hashlib.sha256(" ".join(cmd).encode())
    for f in [src] + _local_headers(src):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _compile(src, is_hip, hipcc, incremental=False):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc] + COMMON + (HIP_FLAGS if is_hip else [f"--offload-arch={ARCH}"]) + ["-c", src, "-o", obj]
    stamp = obj + ".sha256"
    digest = _digest(src, cmd)
    if incremental and os.path.exists(obj) and os.path.exists(stamp):
        with open(stamp) as fh:
            if fh.read().strip() == digest:
                return obj
    if os.path.exists(stamp):
        os.remove(stamp)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    with open(stamp, "w") as fh:
        fh.write(digest)
    return obj


def build(jobs=4, verbose=False, incremental=False):
    """Compiles every source (incremental=True: only those whose text, header texts or
    command changed since their object file was built) and links libensf.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: _compile(s[0], s[1], hipcc, incremental), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lhipfft", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--incremental", action="store_true",
                    help="recompile only sources whose text, headers or command changed")
    a = ap.parse_args()
    build(a.jobs, verbose=True, incremental=a.incremental)
    sys.exit(0)
