"""Build libfkt.so in-tree for gfx950 (hipcc for device code, g++ for the
pure host plan builder).

Usage: python paper_2106_04487_amd/build.py [--jobs N]   (run as a script: importing
the package would first load the library being rebuilt)
"""
from __future__ import annotations

import argparse
import hashlib
import os
import re
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfkt.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 instructions are kept out of the device code on purpose.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include")]


def _jobs():
    dev = [HIPCC, *COMMON, f"--offload-arch={ARCH}", *DEVICE_FLAGS]
    jobs = [
        # the FP64 far-test predicate must not be contracted into FMAs
        (["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-c",
          os.path.join(CSRC, "plan_host.cpp"), "-o", os.path.join(BUILD, "plan_host.o")]),
        ([HIPCC, *COMMON, "-c", os.path.join(CSRC, "fkt_api.cpp"), "-o", os.path.join(BUILD, "fkt_api.o")]),
        ([*dev, "-c", os.path.join(CSRC, "mvm.hip"), "-o", os.path.join(BUILD, "mvm.o")]),
        ([*dev, "-c", os.path.join(CSRC, "cg.hip"), "-o", os.path.join(BUILD, "cg.o")]),
        (["g++", "-O3", "-std=c++17", "-fPIC", "-Wall", "-I" + os.path.join(ROOT, "include"), "-c",
          os.path.join(CSRC, "learn_host.cpp"), "-o", os.path.join(BUILD, "learn_host.o")]),
        (["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-I" + os.path.join(ROOT, "include"), "-c",
          os.path.join(CSRC, "radial_host.cpp"), "-o", os.path.join(BUILD, "radial_host.o")]),
        ([*dev, "-c", os.path.join(CSRC, "learn.hip"), "-o", os.path.join(BUILD, "learn.o")]),
        ([*dev, "-c", os.path.join(CSRC, "mrhs.hip"), "-o", os.path.join(BUILD, "mrhs.o")]),
        ([*dev, "-c", os.path.join(CSRC, "coarse.hip"), "-o", os.path.join(BUILD, "coarse.o")]),
    ]
    # one source-to-multipole object per (dimension, precision)
    for d in (3, 4, 5):
        for prec in (0, 1):
            jobs.append([*dev, f"-DFKT_S2M_D={d}", f"-DFKT_S2M_PREC={prec}", "-c", os.path.join(CSRC, "stage_s2m.hip"),
                         "-o", os.path.join(BUILD, f"stage_s2m_d{d}_p{prec}.o")])
    # one multipole-to-target object per kernel kind (fkt_kernel_kind 0..6)
    for kind in range(7):
        jobs.append([*dev, f"-DFKT_M2T_KIND={kind}", "-c", os.path.join(CSRC, "stage_m2t.hip"),
                     "-o", os.path.join(BUILD, f"stage_m2t_{kind}.o")])
    # persistent near + far field launches, one object per kernel kind
    for kind in range(7):
        jobs.append([*dev, f"-DFKT_FUSED_KIND={kind}", "-c", os.path.join(CSRC, "stage_fused.hip"),
                     "-o", os.path.join(BUILD, f"stage_fused_{kind}.o")])
    # many-RHS source-to-multipole on the matrix cores, one object per dimension
    for d in (3, 4, 5):
        jobs.append([*dev, f"-DFKT_S2M_D={d}", "-c", os.path.join(CSRC, "s2m_mrhs.hip"),
                     "-o", os.path.join(BUILD, f"s2m_mrhs_d{d}.o")])
    # many-RHS multipole-to-target on the matrix cores, one object per kernel kind
    for kind in range(7):
        jobs.append([*dev, f"-DFKT_M2T_KIND={kind}", "-c", os.path.join(CSRC, "m2t_mrhs.hip"),
                     "-o", os.path.join(BUILD, f"m2t_mrhs_{kind}.o")])
    # longest compiles first (the high-order d = 5 moment kernels)
    jobs.sort(key=lambda j: 0 if ("-DFKT_S2M_D=5" in j or any(("m2t" in a or "fused" in a) and a.endswith(".hip")
                                                                for a in j)) else 1)
    return jobs


def _objects():
    return [j[j.index("-o") + 1] for j in _jobs()]


_INCLUDE = re.compile(r'^\s*#\s*include\s*"([^"]+)"', re.M)
_COMMENTS = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


def _deps(src):
    """The source and every header it includes with quotes, transitively."""
    seen, todo = [], [os.path.abspath(src)]
    while todo:
        f = todo.pop()
        if f in seen or not os.path.exists(f):
            continue
        seen.append(f)
        for inc in _INCLUDE.findall(open(f).read()):
            todo.append(os.path.abspath(os.path.join(os.path.dirname(f), inc)))
    return seen


def _fingerprint(cmd):
    """Hash of the command and of its inputs with comments and blank space
    removed: an edit that only touches comments leaves objects current."""
    h = hashlib.sha256(" ".join(cmd).encode())
    for src in [a for a in cmd if a.endswith((".cpp", ".hip"))]:
        for f in _deps(src):
            text = " ".join(_COMMENTS.sub(" ", open(f).read()).split())
            h.update(f.encode() + b"\0" + text.encode())
    return h.hexdigest()


def _stale(cmd) -> bool:
    """An object is stale when it is missing or its fingerprint changed."""
    out = cmd[cmd.index("-o") + 1]
    fp = out + ".fp"
    if not os.path.exists(out) or not os.path.exists(fp):
        return True
    return open(fp).read().strip() != _fingerprint(cmd)


def build(jobs: int = 8, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every object (or, with incremental, only the stale ones) and
    link libfkt.so."""
    os.makedirs(BUILD, exist_ok=True)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        out = cmd[cmd.index("-o") + 1]
        fp = _fingerprint(cmd) if out.endswith(".o") else None  # inputs as compiled
        t0 = time.perf_counter()
        r = subprocess.run(cmd, capture_output=True, text=True)
        if verbose:
            print(f"{time.perf_counter() - t0:7.1f} s  {out}", flush=True)
        if r.returncode != 0:
            raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
        if fp:
            with open(out + ".fp", "w") as f:
                f.write(fp + "\n")
        return r

    todo = [j for j in _jobs() if not incremental or _stale(j)]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(run, todo))
    tmp = LIB + ".tmp"
    run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *_objects(), "-o", tmp, "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("--incremental", action="store_true",
                    help="recompile only objects whose inputs changed (comments aside)")
    a = ap.parse_args()
    print(build(a.jobs, a.v, a.incremental))
    sys.exit(0)
