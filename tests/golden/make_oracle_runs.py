"""Write tests/golden/oracle_runs.json: whole-solve results of the oracle on
the three named workloads (refinements, iterations, final relative residuals,
per-refinement history and a SHA-256 of the solution bytes), and the
iteration count of the oracle's FP64 GMRES(m) comparator on each.

Calls only the oracle (oracle/) and the seeded input generators; run it from
the repository root: python tests/golden/make_oracle_runs.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2009_07495_amd import workloads as W  # noqa: E402


def run(name):
    gen, preset, m = W.WORKLOADS[name]
    sysm = gen()
    pol = O.policy(preset, m=m)
    osys = O.OracleSystem.from_system(sysm, pol)
    t0 = time.time()
    x, st = osys.solve()
    dt = time.time() - t0
    # the paper's comparator ("Double"): FP64 GMRES(m) with the FP64 form of
    # the same preconditioner, relres checked once per restart
    _, fp_it, fp_rc = osys.gmres64(m=m)
    return dict(workload=name, preset=preset, m=m, n=sysm.n, nnz=sysm.nnz, status=st["status"],
                fp64_gmres_iterations=fp_it, fp64_gmres_restarts=-(-fp_it // m), fp64_gmres_status=fp_rc,
                refinements=st["refinements"], iterations=st["iterations"], relres_orig=st["relres_orig"],
                relres_scaled=st["relres_scaled"], hist_relres_orig=[float(v) for v in st["hist_relres_orig"]],
                hist_gamma=[float(v) for v in st["hist_gamma"]], hist_rho=[float(v) for v in st["hist_rho"]],
                x_sha256=hashlib.sha256(x.tobytes()).hexdigest(), oracle_seconds=round(dt, 2))


if __name__ == "__main__":
    names = sys.argv[1:] or list(W.WORKLOADS)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_runs.json")
    data = json.load(open(out)) if os.path.exists(out) else {}
    for nm in names:
        data[nm] = run(nm)
        print(nm, data[nm]["refinements"], data[nm]["relres_orig"], data[nm]["oracle_seconds"], flush=True)
        json.dump(data, open(out, "w"), indent=1)
