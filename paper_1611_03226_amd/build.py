"""Build libdfhip.so (HIP kernels + C ABI) for gfx950, in-tree.

    python -m paper_1611_03226_amd.build [--jobs N] [--arch gfx950]

Every source under csrc/ is compiled by hipcc to an object in _build/, then
linked into paper_1611_03226_amd/libdfhip.so.  build() recompiles every
source; ``--incremental`` reuses objects whose source, headers and flags are
unchanged (keyed by content hash).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libdfhip.so")

SOURCES = ["runtime.cpp", "stateless.cpp", "k_scan.hip", "k_dpd.hip", "k_motion.hip",
           "k_adjoint.hip", "persist.hip", "k_copy.hip", "k_mdp.hip", "k_dpd_net.hip", "noalloc.hip"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags(arch: str) -> list[str]:
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={arch}",
            # packed FP32 VALU ops are disabled for every HIP object
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # matrix-core results in VGPRs (no accumulator-register copies)
            "-Xarch_device", "-mllvm=-amdgpu-mfma-vgpr-form",
            "-Wall", "-Wno-unused-result", f"-I{INCLUDE}", f"-I{CSRC}"]


def _headers_digest() -> str:
    h = hashlib.sha256()
    for d in (CSRC, INCLUDE):
        for f in sorted(os.listdir(d)):
            if f.endswith(".h"):
                with open(os.path.join(d, f), "rb") as fh:
                    h.update(fh.read())
    return h.hexdigest()


def _compile(src: str, arch: str, hdr: str, force: bool) -> str:
    path = os.path.join(CSRC, src)
    fl = flags(arch)
    with open(path, "rb") as fh:
        key = hashlib.sha256(fh.read() + hdr.encode() + " ".join(fl).encode()).hexdigest()[:16]
    obj = os.path.join(BUILD, f"{os.path.splitext(src)[0]}.{key}.o")
    if os.path.exists(obj) and not force:
        return obj
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [hipcc(), *fl, *lang, "-c", path, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if "warning" in warn:
        print(f"{src}:\n{warn}", file=sys.stderr)
    os.replace(obj + ".tmp", obj)
    return obj


def build(arch: str = "gfx950", jobs: int | None = None, verbose: bool = True,
          incremental: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hdr = _headers_digest()
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, arch, hdr, not incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={arch}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--arch", default="gfx950")
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--incremental", action="store_true")
    a = ap.parse_args()
    build(a.arch, a.jobs, incremental=a.incremental)


if __name__ == "__main__":
    main()
