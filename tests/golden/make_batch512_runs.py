"""Write tests/golden/batch512_oracle.json: the oracle's whole solve of every
one of the 512 systems of the batched workload (seed 4; Jacobi, GMRES(30),
tol 1e-10): status, refinement and iteration counts, final relative residual
and a SHA-256 of the solution bytes.

Calls only the oracle (oracle/) and the seeded input generators; the systems
are solved one per process over the host cores (each oracle solve is
single-threaded and deterministic, so the split changes no bit). Run it from
the repository root: python tests/golden/make_batch512_runs.py [processes]
"""
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

COUNT, SEED, M, PRESET = 512, 4, 30, "jacobi"


def solve_one(i: int) -> dict:
    from oracle import oracle as O
    from paper_2009_07495_amd import workloads as W

    # each worker regenerates only system i (child i of SeedSequence(SEED))
    sysm = W.batch_system(i, SEED)
    x, st = O.OracleSystem.from_system(sysm, O.policy(PRESET, m=M)).solve()
    return dict(index=i, name=sysm.name, n=sysm.n, nnz=sysm.nnz, status=st["status"],
                refinements=st["refinements"], iterations=st["iterations"], relres_orig=st["relres_orig"],
                x_sha256=hashlib.sha256(x.tobytes()).hexdigest())


if __name__ == "__main__":
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=procs) as ex:
        runs = list(ex.map(solve_one, range(COUNT), chunksize=4))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch512_oracle.json")
    json.dump({"workload": "batch512", "seed": SEED, "count": COUNT, "preset": PRESET, "m": M, "tol": 1e-10,
               "systems": runs}, open(out, "w"), indent=0)
    print(f"{COUNT} systems in {time.time() - t0:.0f} s; max relres {max(r['relres_orig'] for r in runs):.3e}")
