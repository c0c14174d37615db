"""Builds libfmm.so for gfx950 in-tree (paper_2005_12351_amd/libfmm.so).

Steps: generate the unrolled M2L kernels (csrc/gen_m2l.py) into _build/gen,
compile every translation unit with hipcc (in parallel), link the shared
library.  Host-only tree code is compiled without floating-point contraction
so that the quantisation and acceptance tests round as specified.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
GEN = os.path.join(BUILD, "gen")
LIB = os.path.join(HERE, "libfmm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


def _sources(gen_dir, gen_opt):
    sys.path.insert(0, CSRC)
    import gen_bh  # noqa: E402
    import gen_m2l  # noqa: E402
    gen = gen_m2l.main(gen_dir, gen_opt)
    gen_bh_tus = gen_bh.main(gen_dir)
    sys.path.pop(0)
    srcs = [(os.path.join(CSRC, "p2p_lo.hip"), []),
            (os.path.join(CSRC, "p2p_oct.hip"), []),
            (os.path.join(CSRC, "kernels.hip"), []),
            (os.path.join(CSRC, "m2l.hip"), []),
            (os.path.join(CSRC, "fmm_capi.cpp"), ["-ffp-contract=off"]),
            (os.path.join(CSRC, "tree_host.cpp"), ["-ffp-contract=off"]),
            (os.path.join(CSRC, "m2l_dispatch.cpp"), []),
            (os.path.join(CSRC, "serve.cpp"), [])]
    for extra in ("bh.hip", "tree_gpu.hip", "derivs.hip", "sort.hip"):
        f = os.path.join(CSRC, extra)
        if os.path.exists(f):
            srcs.append((f, []))
    # the Barnes-Hut instantiations first: the longest units
    srcs = [(g, []) for g in gen_bh_tus] + srcs + [(g, []) for g in gen]
    return srcs


def _headers_digest(build_dir):
    """digest of every header a translation unit may include and of this script"""
    paths = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h"))
    gen = os.path.join(build_dir, "gen")
    paths += sorted(os.path.join(gen, f) for f in os.listdir(gen) if f.endswith(".h"))
    paths.append(os.path.join(os.path.dirname(HERE), "include", "fmm.h"))
    paths.append(os.path.abspath(__file__))
    h = hashlib.sha256()
    for p in paths:
        if os.path.exists(p):
            with open(p, "rb") as f:
                h.update(os.path.basename(p).encode() + b"\0" + f.read())
    return h.hexdigest()


def _compile(src, extra, verbose, build_dir, headers=None):
    """compile one unit; with `headers` (incremental build) an object whose
    recorded digest of its source, the headers and the flags matches is kept"""
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    stamp = obj + ".digest"
    digest = None
    if headers is not None:
        h = hashlib.sha256(headers.encode())
        with open(src, "rb") as f:
            h.update(f.read())
        h.update(" ".join(COMMON + extra).encode())
        digest = h.hexdigest()
        if os.path.exists(obj) and os.path.exists(stamp) and open(stamp).read() == digest:
            return obj
        if os.path.exists(stamp):
            os.remove(stamp)
    cmd = [HIPCC, "-x", "hip", "-c", src, "-o", obj] + COMMON + ["-I", os.path.join(build_dir, "gen")] + extra
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stderr[-6000:]}")
    if digest is not None:
        with open(stamp, "w") as f:
            f.write(digest)
    return obj


def build(verbose: bool = False, jobs: int | None = None, out: str = LIB, build_dir: str = BUILD,
          gen_opt: dict | None = None, incremental: bool = False) -> str:
    """Build the library into `out` (default: the in-tree libfmm.so).
    `gen_opt` overrides code-shape options of the generated M2L kernels.
    `incremental` keeps an object compiled from the same source, headers and
    flags (recorded beside it; the default compiles everything)."""
    gen_dir = os.path.join(build_dir, "gen")
    os.makedirs(gen_dir, exist_ok=True)
    srcs = _sources(gen_dir, gen_opt)
    headers = _headers_digest(build_dir) if incremental else None
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda a: _compile(a[0], a[1], verbose, build_dir, headers), srcs))
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stderr[-4000:]}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
