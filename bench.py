"""Benchmark: integer-GMRES(m) + FP64 iterative refinement solves per second on
one MI355X.

A step is one whole solve (Fig. 1 of the paper: refinements until the FP64
relative residual of the original system is below 1e-10) of the
convection-diffusion workload (64^3 grid, 7-point stencil, n = 262,144,
nnz = 1,810,432, Jacobi preconditioner, GMRES(50)), with the system and the
solution vector resident in HBM. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s

# Sources the persistent cycle kernel is compiled from: a traffic figure
# measured with hardware counters is reported only while they are unchanged.
CYCLE_SOURCES = ("igm_cycle.hip", "igm_sweep.hpp", "igm_sync.hpp", "igm_rows.hpp", "igm_device.hpp", "igm_internal.hpp")


def cycle_sources_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    for name in CYCLE_SOURCES:
        with open(os.path.join(ROOT, "paper_2009_07495_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str, grid_blocks: int):
    """HBM bytes per cycle-kernel launch from the FETCH_SIZE / WRITE_SIZE
    counter summary in profiles/, if it was taken on the current kernel
    sources, this workload and this workgroup count; else None."""
    path = os.path.join(ROOT, "profiles", f"k_cycle_{workload}.md")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"^\s*([a-z_0-9]+)\s*=\s*(\S+)\s*$", line)
            if m:
                kv[m.group(1)] = m.group(2)
    try:
        ok = (kv["kernel_sources_sha256"] == cycle_sources_digest() and int(kv["grid_blocks"]) == grid_blocks)
        return float(kv["traffic_bytes_per_launch"]) if ok else None
    except KeyError:
        return None


def cycle_bytes(n: int, nnz: int, m_steps: int, precond: int, nnz_l: int, nnz_u: int, nterms: int) -> float:
    """Algorithmic HBM bytes of one int-GMRES call of the persistent kernel:
    per Arnoldi step j the matrix stream (8 B value per term + 4 B column per
    nonzero) and one read of v_j, the preconditioner operands, j reads of the
    basis for modified Gram-Schmidt (w stays in registers), one write of
    v_{j+1}; then the closing least-squares step reads the basis once and
    updates x."""
    per_step = nnz * (8 * nterms + 4) + 8 * n + 8 * n  # matrix, v_j gather, v_{j+1} write
    if precond == 1:
        per_step += 16 * n  # two integer diagonals
    elif precond == 2:
        per_step += 12 * (nnz_l + nnz_u) + 16 * (n + 1) + 40 * n  # factors, row pointers, z/y/u traffic
    mgs = 8 * n * m_steps * (m_steps + 1) / 2
    update = 8 * n * m_steps + 16 * n
    return m_steps * per_step + mgs + update


def cpu_baseline(sysm, preset: str, m: int, refinements: int, cycles: int = 2) -> dict:
    """The oracle (single-threaded C) on a bounded sample: the first `cycles`
    refinements of one solve, scaled to solves/s with the solve's refinement count."""
    from oracle import oracle as O

    o = O.OracleSystem.from_system(sysm, O.policy(preset, m=m, max_refine=cycles))
    t0 = time.perf_counter()
    _, st = o.solve()
    dt = time.perf_counter() - t0
    per_cycle = dt / max(st["refinements"], 1)
    return {"value": 1.0 / (per_cycle * refinements), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{st['refinements']} of the {refinements} refinements of one solve ({dt:.1f} s), "
                      f"scaled by the refinement count"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="convdiff3d_64")
    ap.add_argument("--grid-blocks", type=int, default=0, help="cycle-kernel workgroups (0 = autotune)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernels", action="store_true", help="skip timing the standalone SpMV and dot kernels")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-system batched solver section")
    ap.add_argument("--no-serve", action="store_true", help="skip the served solver section")
    ap.add_argument("--serve-requests", type=int, default=48, help="requests in the served trace")
    ap.add_argument("--serve-distinct", type=int, default=24, help="distinct systems the trace draws from")
    ap.add_argument("--batch-steps", type=int, default=3, help="timed solves of the whole batch")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a known-size kernel for "
                         "calibrating hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2009_07495_amd import binding as B
    from paper_2009_07495_amd import workloads as W

    assert torch.cuda.is_available()
    if args.copy_mib:
        src = torch.ones(args.copy_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    gen, preset, m = W.WORKLOADS[args.workload]
    progress(f"single-system solver: {args.workload}")
    sysm = gen()

    # autotune the workgroup count of the cycle kernel (bits do not depend on it)
    candidates = [args.grid_blocks] if args.grid_blocks else [64, 128, 256]
    best = None
    x = torch.zeros(sysm.n, dtype=torch.float64, device="cuda")
    g = B.System.from_system(sysm, preset, m=m)
    for gb in candidates:
        try:
            g.set_policy(B.make_policy(preset, m=m, grid_blocks=gb))
        except B.IgmError as e:  # too few workgroups for this many rows
            if e.status != B.ERR_UNSUPPORTED:
                raise
            continue
        x.zero_()
        assert g.solve_device(x) == B.OK
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        assert g.solve_device(x) == B.OK
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if best is None or dt < best[1]:
            best = (gb, dt)
    g.set_policy(B.make_policy(preset, m=m, grid_blocks=best[0]))
    st = g.stats()

    for _ in range(args.warmup):
        x.zero_()
        assert g.solve_device(x) == B.OK
    torch.cuda.synchronize()
    cyc_ms, refs, iters, relres = 0.0, 0, 0, 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x.zero_()
        rc = g.solve_device(x)
        s = g.stats()
        assert rc == B.OK and s["relres_orig"] <= 1e-10, (rc, s["relres_orig"])
        cyc_ms += s["time_cycle_ms"]
        refs += s["refinements"]
        iters += s["iterations"]
        relres = max(relres, s["relres_orig"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps

    pol = g.pol
    steps_per_cycle = iters / refs
    nnz_l = nnz_u = 0
    if preset == "paper_ilu":
        nnz_l = nnz_u = (sysm.nnz - sysm.n) // 2
    byts = cycle_bytes(sysm.n, sysm.nnz, int(round(steps_per_cycle)), pol.precond, nnz_l, nnz_u, st["nterms"])
    avg_cycle_s = cyc_ms / refs / 1000.0
    achieved = byts / avg_cycle_s / 1e9
    traffic = measured_traffic(args.workload, st["grid_blocks"])
    out = {
        "metric": "GMRES-IR solves/s at relres 1e-10 (integer GMRES(m) inner solver)",
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: n={sysm.n}, nnz={sysm.nnz}, preset={preset}, GMRES({m})+FP64 IR, "
                               f"tol 1e-10", "refinements_per_solve": refs / args.steps,
                   "grid_blocks": st["grid_blocks"], "rows_per_thread": st["rows_per_thread"],
                   "max_relres": relres},
        "roofline": {"kernel": "k_cycle (persistent int-GMRES call)", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": byts, "avg_launch_ms": avg_cycle_s * 1000.0},
    }
    # where the time goes: one more solve with the phase clock on (not timed)
    g.set_policy(B.make_policy(preset, m=m, grid_blocks=best[0], phase_clock=1))
    x.zero_()
    assert g.solve_device(x) == B.OK
    ph = g.stats()["phase_us"]
    out["cycle_phases_us"] = dict(zip(["spmv_precond", "mgs_local", "mgs_grid_wait", "norm", "normalize",
                                       "givens", "step_barrier", "total"], [round(v, 1) for v in ph]))
    if not args.no_kernels:
        progress("standalone SpMV and dot kernels")
        out["kernels"] = kernel_rates(torch, B, W)
    if not args.no_batch:
        progress("batched solver: 512 systems")
        out["batched"] = batched(torch, B, W, args.batch_steps, not args.no_cpu_baseline)
    if not args.no_serve:
        progress("served solver: request stream")
        out["served"] = served(B, W, args.serve_requests, args.serve_distinct)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sysm, preset, m, int(round(refs / args.steps)))
    print(json.dumps(out))


def batch_bytes(n: int, nnz: int, m: int, refinements: int) -> float:
    """Algorithmic HBM bytes of one system's solve in the batched kernel
    (Jacobi, one term): per refinement the int-GMRES call (see cycle_bytes)
    plus the FP64 residual (20 B per nonzero, row pointers, b, bhat, x, 48 B
    per row) and the start step with the cast of v1 (x, diagonals, v1)."""
    return refinements * (cycle_bytes(n, nnz, m, 1, 0, 0, 1) + 20 * nnz + 48 * n + 40 * n)


def batched(torch, B, W, steps: int, with_cpu: bool) -> dict:
    """The 512-system workload (2D/3D convection-diffusion, n log-uniform in
    [1k, 64k], Jacobi, GMRES(30)) solved by the batched persistent kernel,
    beside the plain loop of single-system solves on the same GPU."""
    systems = W.batch_systems(512, seed=4)
    m = 30
    bt = B.Batch(systems, "jacobi", m=m)
    block, rows = bt.autotune()
    x = torch.zeros(bt.total_n, dtype=torch.float64, device="cuda")
    x.zero_()
    assert bt.solve_device(x) == B.OK
    times = []
    for _ in range(steps):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = bt.solve_device(x)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        assert rc == B.OK, rc
    res = bt.results()
    st = bt.stats()
    t = float(np.median(times))
    bt.set_phase_clock(True)
    x.zero_()
    assert bt.solve_device(x) == B.OK
    names = ["spmv_precond", "mgs_local", "mgs_wait", "norm", "normalize", "fp64_refinement", "step_barrier", "total"]
    ph = np.sum([r["phase_us"] for r in bt.results()], axis=0) / max(sum(r["refinements"] for r in res), 1)
    byts = sum(batch_bytes(r["n"], r["nnz"], m, r["refinements"]) for r in res)
    lat = np.array([r["time_solve_ms"] for r in res])
    bt.close()
    # plain loop: one single-system solve after another (system resident, setup not timed)
    g0 = B.System.from_system(systems[0], "jacobi", m=m)
    xw = torch.zeros(systems[0].n, dtype=torch.float64, device="cuda")
    g0.solve_device(xw)
    g0.close()
    plain = 0.0
    for s in systems:
        g = B.System.from_system(s, "jacobi", m=m)
        xs = torch.zeros(s.n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = g.solve_device(xs)
        torch.cuda.synchronize()
        plain += time.perf_counter() - t0
        assert rc == B.OK, rc
        g.close()
    out = {"workload": f"batch512: 512 systems, n log-uniform [1k, 64k] (sum n {bt.total_n}), 2D 5-point / 3D 7-point "
                       f"convection-diffusion, jacobi, GMRES({m})+FP64 IR, tol 1e-10",
           "solves_per_s": len(systems) / t, "ms_per_batch": 1000.0 * t, "kernel_ms": st["time_kernel_ms"],
           "plain_loop_solves_per_s": len(systems) / plain, "plain_loop_s": plain,
           "speedup_vs_plain_loop": plain / t, "block": block, "rows_per_thread": rows,
           "grid_blocks": st["grid_blocks"], "refinements": st["refinements"],
           "max_relres": max(r["relres_orig"] for r in res),
           "algorithmic_gb_s": byts / t / 1e9, "per_system_ms_p50": float(np.percentile(lat, 50)),
           "per_system_ms_p99": float(np.percentile(lat, 99)),
           "phases_us_per_refinement": dict(zip(names, [round(float(v), 1) for v in ph]))}
    if with_cpu:
        from oracle import oracle as O

        sample = systems[:6]
        t0 = time.perf_counter()
        for s in sample:
            O.OracleSystem.from_system(s, O.policy("jacobi", m=m)).solve()
        dt = time.perf_counter() - t0
        # the oracle's refinement counts equal the GPU's (bit-exact), so the
        # work of a system scales with rows x refinements
        work = [r["n"] * r["refinements"] for r in res]
        scale = sum(work) / sum(work[: len(sample)])
        out["cpu_baseline"] = {"value": len(systems) / (dt * scale), "unit": "solves/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"first {len(sample)} of the 512 systems ({dt:.1f} s), scaled by "
                                         f"rows x refinements to the whole batch"}
    return out


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def served(B, W, count: int, distinct: int, rate: float = 2000.0) -> dict:
    """The served workload: Poisson arrivals (mean 2000 requests/s) of solves
    with n log-uniform in [4096, 1M] from the three families (2D/3D
    convection-diffusion with Jacobi, 27-point random with ILU(0)),
    GMRES(30), through the server; latency = submission to result, host setup
    included. Beside it the plain per-request loop (create, solve, destroy)
    over the same trace."""
    import itertools

    pool = list(itertools.islice(W.served_requests(distinct, seed=5), distinct))
    reqs = [pool[i % distinct] for i in range(count)]
    arrivals = W.arrival_times(count, rate, seed=5)
    sv = B.Server()
    w = sv.submit(W.convdiff2d(40, 40, seed=1), "jacobi", m=30)  # warm-up
    sv.wait(w, 120000)
    t0 = time.perf_counter()
    subs = []
    for (s, preset), ta in zip(reqs, arrivals):
        d = t0 + ta - time.perf_counter()
        if d > 0:
            time.sleep(d)
        subs.append((sv.submit(s, preset, m=30), time.perf_counter() - t0))
    lat, setup, dev, ok, relres = [], [], [], 0, 0.0
    last = 0.0
    for t, ts in subs:
        _, st = sv.wait(t, 600000)
        lat.append(st["time_solve_ms"])
        setup.append(st["time_setup_ms"])
        dev.append(st["time_kernel_ms"])
        ok += st["status"] == B.OK
        relres = max(relres, st["relres_orig"])
        last = max(last, ts + st["time_solve_ms"] / 1000.0)
    sst = sv.stats()
    sv.close()
    progress(f"served {count} requests in {last:.2f} s; plain per-request loop next")
    plain = 0.0
    for s, preset in reqs:
        t = time.perf_counter()
        g = B.System.from_system(s, preset, m=30)
        _, st = g.solve()
        g.close()
        plain += time.perf_counter() - t
        assert st == B.OK
    lat = np.array(lat)
    return {"workload": f"served: {count} requests (drawn from {distinct} distinct systems, n log-uniform "
                        f"[4096, 1M], 2D/3D convection-diffusion with jacobi and 27-point random with ILU(0), "
                        f"GMRES(30)+FP64 IR, tol 1e-10), Poisson arrivals at {rate:.0f}/s",
            "solves_per_s": count / last, "completed_ok": ok, "requests": count, "max_relres": relres,
            "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
            "setup_ms_p50": float(np.percentile(setup, 50)), "setup_ms_p99": float(np.percentile(setup, 99)),
            "device_ms_p50": float(np.percentile(dev, 50)), "device_ms_p99": float(np.percentile(dev, 99)),
            "plain_loop_solves_per_s": count / plain, "speedup_vs_plain_loop": plain / last,
            "sustainable_at_offered_rate": bool(count / last >= 0.95 * rate),
            "workgroups": sst["workgroups"], "pool_peak_bytes": sst["pool_peak"]}


def kernel_rates(torch, B, W) -> dict:
    """Standalone SpMV and Gram-Schmidt inner-product kernels (Fig. 2) on the
    27-point 1M-row matrix, timed with HIP events around the kernels."""
    sysm = W.random27(128, 128, 64, seed=3)
    g = B.System.from_system(sysm, "jacobi", m=2)
    n, nnz = sysm.n, sysm.nnz
    rng = np.random.default_rng(0)
    v = torch.from_numpy(rng.integers(-(1 << 30), 1 << 30, n)).cuda()
    z = torch.zeros(n, dtype=torch.int64, device="cuda")
    res = {}
    for name, fn, byts in (("spmv", lambda: g.spmv(v, z), 12 * nnz + 16 * n + 4 * (n + 1)),
                           ("dot", lambda: g.dot(v, v), 16 * n)):  # Q30 words: no product overflows
        for _ in range(3):
            fn()
        ts = []
        for _ in range(20):
            fn()
            ts.append(g.stats()["time_kernel_ms"])
        t = float(np.median(ts)) / 1000.0
        res[name] = {"gb_s": byts / t / 1e9, "frac": byts / t / 1e9 / HBM_PEAK_GBS, "ms": t * 1000.0,
                     "bytes": byts, "workload": f"random27 n={n} nnz={nnz}"}
    return res


if __name__ == "__main__":
    main()
