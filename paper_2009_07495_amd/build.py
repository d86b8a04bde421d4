"""Build the gfx950 HIP library ``libigmres.so`` in place with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libigmres.so")
# the cycle kernels first: they take longest to compile
SOURCES = ["igm_cycle.hip", "igm_cycle_lanes.hip", "igm_cycle_merge.hip", "igm_batch.hip", "igm_kernels.hip",
           "igm_api.cpp", "igm_setup.cpp", "igm_bsched.cpp", "igm_batch.cpp", "igm_serve.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # every FP64 step must round exactly as written: no FMA contraction
    "-ffp-contract=off",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
    return res.returncode, out


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link
    paper_2009_07495_amd/libigmres.so (always rebuilds)."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, s + ".o") for s in SOURCES]
    cmds = [[HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        results = list(ex.map(_run, cmds))
    for (rc, out), s in zip(results, SOURCES):
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {s} ({rc}):\n{out}")
        if verbose and out.strip():
            print(out)
    tmp = LIB + ".tmp"
    # roctx: host trace ranges of the solvers
    rc, out = _run([HIPCC, *FLAGS, "-shared", *objs, "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-o", tmp])
    if rc != 0:
        raise RuntimeError(f"link failed ({rc}):\n{out}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
