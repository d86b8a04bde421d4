"""Benchmark: integer-GMRES(m) + FP64 iterative refinement solves per second on
one MI355X.

A step is one whole solve (Fig. 1 of the paper: refinements until the FP64
relative residual of the original system is below 1e-10) of the 1M-row
27-point system (128 x 128 x 64 grid, n = 1,048,576, nnz = 27,725,560,
fixed-point ILU(0) preconditioner with level-scheduled sweeps, GMRES(30)),
with the system and the solution vector resident in HBM. Prints one JSON
line; sections beside the headline: the 262K-row convection-diffusion
system, the 512-system batched solver, the served solver, the standalone
SpMV and inner-product kernels and a device copy (measured bandwidth peak).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
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
# measured with hardware counters is reported only while their code (comments
# aside) is unchanged.
# sources of the single-system cycle kernels (every mapping) and what they include
CYCLE_SOURCES = ("igm_cycle.hip", "igm_cycle_lanes.hip", "igm_cycle_merge.hip", "igm_cycle.hpp", "igm_bsweep.hpp",
                 "igm_sync.hpp", "igm_rows.hpp", "igm_device.hpp", "igm_internal.hpp", "../../include/igmres.h")


def strip_comments(src: str) -> str:
    """C/C++ source without its comments and with runs of blank space made one
    space (string and character literals kept), so that the digest below
    changes with the code, not with its comments."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def cycle_sources_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    for name in CYCLE_SOURCES:
        with open(os.path.join(ROOT, "paper_2009_07495_amd", "csrc", name), encoding="utf-8") as f:
            h.update(strip_comments(f.read()).encode())
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


def path_bytes(n: int, nnz: int, steps: int, precond: int, nnz_lu: int, nterms: int) -> float:
    """Algorithmic HBM bytes of one int-GMRES call with `steps` Arnoldi steps
    (int64 words, int32 indices, every vector read or written once): per step
    j the SpMV (12 nnz + 4(n+1) + 16n, plus 12 nnz + 4(n+1) + 8n per further
    matrix term), the preconditioner apply (ILU(0): 12 (nnz(L)+nnz(U)) +
    8(n+1) + 32n with both factors' diagonals counted in nnz_lu; Jacobi: the
    two diagonals, 16n), modified Gram-Schmidt reading the j basis vectors
    (8n j; w stays on chip), the norm (8n) and the normalisation (16n); then
    the closing least-squares step reads the basis once and updates x
    (8n steps + 16n)."""
    spmv = 12 * nnz + 4 * (n + 1) + 16 * n + (nterms - 1) * (12 * nnz + 4 * (n + 1) + 8 * n)
    pre = {0: 0, 1: 16 * n, 2: 12 * nnz_lu + 8 * (n + 1) + 32 * n}[precond]
    per_step = spmv + pre + 8 * n + 16 * n
    mgs = 8 * n * steps * (steps + 1) / 2
    return steps * per_step + mgs + 8 * n * steps + 16 * n


def host_cpu() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cores": len(os.sched_getaffinity(0))}


def pinned_to_one_core(fn):
    """Run fn() with this thread pinned to one core (the first of its
    affinity set); returns (result, core)."""
    before = os.sched_getaffinity(0)
    core = min(before)
    os.sched_setaffinity(0, {core})
    try:
        return fn(), core
    finally:
        os.sched_setaffinity(0, before)


def cpu_baseline(sysm, preset: str, m: int, refinements: int, cycles: int) -> dict:
    """The oracle (single-threaded C, pinned to one core) on a bounded
    sample: the first `cycles` refinements of one solve, scaled to solves/s
    with the solve's refinement count."""
    from oracle import oracle as O

    o = O.OracleSystem.from_system(sysm, O.policy(preset, m=m, max_refine=cycles))

    def run():
        t0 = time.perf_counter()
        _, st = o.solve()
        return time.perf_counter() - t0, st

    (dt, st), core = pinned_to_one_core(run)
    per_cycle = dt / max(st["refinements"], 1)
    return {"value": 1.0 / (per_cycle * refinements), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{st['refinements']} of the {refinements} refinements of one solve ({dt:.1f} s on core "
                      f"{core}), scaled by the refinement count", **host_cpu()}


def golden_context(workload: str) -> dict | None:
    """The paper's comparator on this workload, from the oracle's recorded
    runs: FP64 GMRES(m) iterations beside the integer solver's refinements."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_runs.json")
    try:
        with open(path) as f:
            rec = json.load(f)[workload]
    except (OSError, KeyError, ValueError):
        return None
    out = {"int_gmres_refinements": rec["refinements"], "int_gmres_iterations": rec["iterations"]}
    if "fp64_gmres_iterations" in rec:
        out.update(fp64_gmres_iterations=rec["fp64_gmres_iterations"],
                   fp64_gmres_restarts=rec["fp64_gmres_restarts"])
    return out


def stream_copy(torch, mib: int = 2048, reps: int = 10) -> dict:
    """Measured device bandwidth: a device-to-device copy of `mib` MiB
    (read + write bytes), median of `reps` launches timed with HIP events."""
    src = torch.ones(mib << 17, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1000.0)
    t = float(np.median(ts))
    del src, dst
    torch.cuda.empty_cache()
    return {"gb_s": 2.0 * (mib << 20) / t / 1e9, "bytes_moved": 2 * (mib << 20), "ms": t * 1000.0}


def single(torch, B, W, workload: str, steps: int, warmup: int, grid_blocks: int = 0) -> dict:
    """Whole solves of one named workload by the single-system solver, the
    system and x resident in HBM; the cycle kernel's workgroup count is
    autotuned first (bits do not depend on it). Returns the measured figures
    and the roofline of the int-GMRES call."""
    gen, preset, m = W.WORKLOADS[workload]
    sysm = gen()
    candidates = [grid_blocks] if grid_blocks else [64, 128, 256]
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

    for _ in range(warmup):
        x.zero_()
        assert g.solve_device(x) == B.OK
    torch.cuda.synchronize()
    cyc_ms, refs, iters, relres, calls = 0.0, 0, 0, 0.0, 0
    t0 = time.perf_counter()
    for _ in range(steps):
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

    pol = g.pol
    steps_per_call = iters / refs
    nnz_lu = sysm.nnz + sysm.n if pol.precond == B.PRE_ILU0 else 0
    byts = path_bytes(sysm.n, sysm.nnz, int(round(steps_per_call)), pol.precond, nnz_lu, st["nterms"])
    avg_call_s = cyc_ms / refs / 1000.0
    achieved = byts / avg_call_s / 1e9
    out = {
        "workload": f"{workload}: n={sysm.n}, nnz={sysm.nnz}, preset={preset}, GMRES({m})+FP64 IR, tol 1e-10",
        "solves_per_s": steps / elapsed, "ms_per_solve": 1000.0 * elapsed / steps,
        "refinements_per_solve": refs / steps, "grid_blocks": st["grid_blocks"],
        "block_threads": st["block_threads"], "rows_per_thread": st["rows_per_thread"], "max_relres": relres,
        "roofline": {"kernel": "k_cycle (persistent int-GMRES call)", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(workload, st["grid_blocks"]), "bytes_per_launch": byts,
                     "avg_launch_ms": avg_call_s * 1000.0, "launches_timed": refs},
        "paper_context": golden_context(workload),
    }
    # where the time goes: one more solve with the phase clock on (not timed)
    g.set_policy(B.make_policy(preset, m=m, grid_blocks=best[0], phase_clock=1))
    x.zero_()
    assert g.solve_device(x) == B.OK
    ph = g.stats()["phase_us"]
    out["cycle_phases_us"] = dict(zip(["spmv_precond", "mgs_local", "mgs_grid_wait", "norm", "normalize",
                                       "givens", "step_barrier", "total"], [round(v, 1) for v in ph]))
    # the basis streamed by the local Gram-Schmidt work of that call (workgroup
    # 0's clock): steps (steps + 1) / 2 columns of n words
    last_steps = int([j for j in g.history()["jstar"] if j >= 0][-1])
    mgs_bytes = 8 * sysm.n * last_steps * (last_steps + 1) / 2
    out["mgs_local_stream"] = {"steps": last_steps, "bytes": mgs_bytes,
                               "gb_s": mgs_bytes / (ph[1] * 1e-6) / 1e9 if ph[1] > 0 else None,
                               "frac": mgs_bytes / (ph[1] * 1e-6) / 1e9 / HBM_PEAK_GBS if ph[1] > 0 else None}
    g.close()
    return out, sysm, preset, m


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="random27_1m")
    ap.add_argument("--grid-blocks", type=int, default=0, help="cycle-kernel workgroups (0 = autotune)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernels", action="store_true", help="skip timing the standalone SpMV and dot kernels")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-system batched solver section")
    ap.add_argument("--no-serve", action="store_true", help="skip the served solver section")
    ap.add_argument("--no-second", action="store_true", help="skip the 262K-row convection-diffusion section")
    ap.add_argument("--serve-requests", type=int, default=1000, help="requests in the served trace")
    ap.add_argument("--serve-distinct", type=int, default=96, help="distinct systems the trace draws from")
    ap.add_argument("--batch-steps", type=int, default=3, help="timed solves of the whole batch")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a known-size kernel for "
                         "calibrating hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU (sharding is design only); --gpus must be 1"}))
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
    progress(f"single-system solver: {args.workload}")
    head, sysm, preset, m = single(torch, B, W, args.workload, args.steps, args.warmup, args.grid_blocks)
    progress("device copy (measured bandwidth)")
    copy = stream_copy(torch)
    roof = head.pop("roofline")
    roof["frac_of_measured_copy"] = roof["achieved"] / copy["gb_s"]
    out = {
        "metric": "GMRES-IR solves/s at relres 1e-10 (integer GMRES(m) inner solver)",
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {k: head[k] for k in ("workload", "refinements_per_solve", "grid_blocks", "block_threads",
                                         "rows_per_thread", "max_relres")},
        "roofline": roof,
        "stream_copy": copy,
        "paper_context": head["paper_context"],
        "cycle_phases_us": head["cycle_phases_us"],
        "mgs_local_stream": head["mgs_local_stream"],
    }
    if not args.no_second and args.workload != "convdiff3d_64":
        progress("single-system solver: convdiff3d_64")
        out["convdiff3d_64"] = single(torch, B, W, "convdiff3d_64", 10, 2)[0]
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
        progress("oracle on one host core (bounded sample)")
        refs = int(round(head["refinements_per_solve"]))
        out["cpu_baseline"] = cpu_baseline(sysm, preset, m, refs, max(1, min(2, refs // 2)))
    print(json.dumps(out), flush=True)


def batch_bytes(n: int, nnz: int, m: int, refinements: int) -> float:
    """Algorithmic HBM bytes of one system's solve in the batched kernel
    (Jacobi, one term): per refinement the int-GMRES call (see path_bytes)
    plus the FP64 residual (20 B per nonzero, row pointers, b, bhat, x, 48 B
    per row) and the start step with the cast of v1 (x, diagonals, v1)."""
    return refinements * (path_bytes(n, nnz, m, 1, 0, 1) + 20 * nnz + 48 * n + 40 * n)


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

        def run():
            t0 = time.perf_counter()
            for s in sample:
                O.OracleSystem.from_system(s, O.policy("jacobi", m=m)).solve()
            return time.perf_counter() - t0

        dt, core = pinned_to_one_core(run)
        # the oracle's refinement counts equal the GPU's (bit-exact), so the
        # work of a system scales with rows x refinements
        work = [r["n"] * r["refinements"] for r in res]
        scale = sum(work) / sum(work[: len(sample)])
        out["cpu_baseline"] = {"value": len(systems) / (dt * scale), "unit": "solves/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"first {len(sample)} of the 512 systems ({dt:.1f} s on core {core}), "
                                         f"scaled by rows x refinements to the whole batch", **host_cpu()}
    return out


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def served_trace(B, reqs, arrivals, timeout_ms: float = 600000.0) -> dict:
    """Submit the requests at their arrival times to a fresh server and wait
    for every one; every request must finish OK at relres <= 1e-10.
    Latency = submission to result (host setup included)."""
    sv = B.Server()
    from paper_2009_07495_amd import workloads as W

    w = sv.submit(W.convdiff2d(40, 40, seed=1), "jacobi", m=30)  # warm-up
    sv.wait(w, 120000)
    t0 = time.perf_counter()
    subs = []
    for (s, preset), ta in zip(reqs, arrivals):
        d = t0 + ta - time.perf_counter()
        if d > 0:
            time.sleep(d)
        subs.append((sv.submit(s, preset, m=30), time.perf_counter() - t0))
    lat, setup, dev, relres, last = [], [], [], 0.0, 0.0
    for t, ts in subs:
        _, st = sv.wait(t, timeout_ms)
        assert st["status"] == B.OK and st["relres_orig"] <= 1e-10, (st["status"], st["relres_orig"])
        lat.append(st["time_solve_ms"])
        setup.append(st["time_setup_ms"])
        dev.append(st["time_kernel_ms"])
        relres = max(relres, st["relres_orig"])
        last = max(last, ts + st["time_solve_ms"] / 1000.0)
    sst = sv.stats()
    sv.close()
    pct = lambda v, p: float(np.percentile(v, p))  # noqa: E731
    return {"completed_ok": len(subs), "solves_per_s": len(subs) / last, "makespan_s": last, "max_relres": relres,
            "offered_per_s": len(subs) / float(arrivals[-1]) if len(arrivals) else 0.0,
            "latency_ms_p50": pct(lat, 50), "latency_ms_p99": pct(lat, 99),
            "setup_ms_p50": pct(setup, 50), "setup_ms_p99": pct(setup, 99),
            "device_ms_p50": pct(dev, 50), "device_ms_p99": pct(dev, 99),
            "workgroups": sst["workgroups"], "pool_peak_bytes": sst["pool_peak"]}


def served(B, W, count: int, distinct: int, rate: float = 2000.0, plain_sample: int = 100) -> dict:
    """The served workload: Poisson arrivals (mean 2000 requests/s) of solves
    with n log-uniform in [4096, 1M] from the three families (2D/3D
    convection-diffusion with Jacobi, 27-point random with ILU(0)),
    GMRES(30), through the server. The offered rate is far above one GPU's
    capacity, so the server runs saturated and its completion rate is the
    largest sustainable rate; a second, shorter trace at 80% of that rate
    gives the latency without a standing queue. Beside it the plain
    per-request loop (create, solve, destroy), timed on a uniform sample of
    the same trace."""
    import itertools

    pool = list(itertools.islice(W.served_requests(distinct, seed=5), distinct))
    reqs = [pool[i % distinct] for i in range(count)]
    arrivals = W.arrival_times(count, rate, seed=5)
    sat = served_trace(B, reqs, arrivals)
    progress(f"served {count} requests in {sat['makespan_s']:.2f} s; trace at 80% of that rate next")
    cap = sat["solves_per_s"]
    n2 = max(32, min(count // 4, int(cap * 15)))  # about 15 s of offered work
    arr2 = W.arrival_times(n2, 0.8 * cap, seed=6)
    below = served_trace(B, reqs[:n2], arr2)
    progress("plain per-request loop on a sample of the trace")
    step = max(1, count // plain_sample)
    sample = reqs[::step][:plain_sample]
    plain = 0.0
    for s, preset in sample:
        t = time.perf_counter()
        g = B.System.from_system(s, preset, m=30)
        _, st = g.solve()
        g.close()
        plain += time.perf_counter() - t
        assert st == B.OK
    plain_rate = len(sample) / plain
    return {"workload": f"served: {count} requests (drawn in turn from {distinct} distinct systems of the stream: "
                        f"n log-uniform [4096, 1M], 2D/3D convection-diffusion with jacobi and 27-point random with "
                        f"ILU(0), GMRES(30)+FP64 IR, tol 1e-10), Poisson arrivals offered at {rate:.0f}/s",
            "requests": count, **{k: v for k, v in sat.items()},
            "max_sustainable_per_s": cap,
            "sustainable_at_offered_rate": bool(cap >= 0.95 * rate),
            "at_80pct_of_capacity": below,
            "plain_loop_solves_per_s": plain_rate,
            "plain_loop_sample": f"every {step}th request of the trace ({len(sample)} requests, {plain:.1f} s)",
            "speedup_vs_plain_loop": cap / plain_rate}


def dot_by_length(torch, B, rng) -> dict:
    """The inner-product kernel (k_reduce, the kernel of igm_dot and
    igm_norm) on two distinct int64 vectors of 2^20 to 2^26 words, through
    the allocation-free entry point (whose launch also runs a one-thread
    clearing kernel): HIP events on the stream around 50 back-to-back calls.
    At 2^20 words (16.8 MB) the fixed cost of a launch and of the completion
    ticket (about 5 us) dominates; from 2^24 words on the kernel streams."""
    stream = torch.cuda.current_stream()
    out = {}
    for lg in (20, 22, 24, 26):
        n = 1 << lg
        w = torch.from_numpy(rng.integers(-(1 << 30), 1 << 30, n)).cuda()
        v = torch.from_numpy(rng.integers(-(1 << 30), 1 << 30, n)).cuda()
        res = torch.zeros(2, dtype=torch.int64, device="cuda")
        for _ in range(5):
            assert B.igm_reduce_noalloc(0, n, w, v, 0, 30, res, stream) == B.OK
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(50):
            B.igm_reduce_noalloc(0, n, w, v, 0, 30, res, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1000.0 / 50
        out[str(n)] = {"us_per_call": us, "bytes": 16 * n, "gb_s": 16 * n / us / 1e3,
                       "frac": 16 * n / us / 1e3 / HBM_PEAK_GBS}
        del w, v, res
    return out


def kernel_rates(torch, B, W) -> dict:
    """Standalone SpMV and Gram-Schmidt inner-product kernels (Fig. 2), timed
    with HIP events around the kernels: the SpMV with each row-to-lane mapping
    (1: one thread per row over SELL-64; 2: each workgroup's rows split evenly
    by entries; 4, 8, 16, 32, 64 lanes per row over CSR) on the
    27-point 1M-row matrix, the 7-point 64^3 matrix and a heavy-tailed 1M-row
    matrix, with the mapping the automatic rule and the setup-time measurement
    pick; the inner product on the 27-point matrix's vector length."""

    def med_ms(g, fn):
        for _ in range(3):
            fn()
        ts = []
        for _ in range(20):
            fn()
            ts.append(g.stats()["time_kernel_ms"])
        return float(np.median(ts))

    res = {"spmv_mappings": {}}
    rng = np.random.default_rng(0)
    for wl, gen in (("random27_1m", lambda: W.random27(128, 128, 64, seed=3)),
                    ("convdiff3d_64", lambda: W.convdiff3d(64)),
                    ("skewed_1m", lambda: W.skewed(1 << 20, seed=6))):
        sysm = gen()
        n, nnz = sysm.n, sysm.nnz
        byts = 12 * nnz + 16 * n + 4 * (n + 1)
        v = torch.from_numpy(rng.integers(-(1 << 30), 1 << 30, n)).cuda()
        z = torch.zeros(n, dtype=torch.int64, device="cuda")
        row = {"n": n, "nnz": nnz, "bytes": byts, "lanes": {}}
        for lanes in (1, 2, 4, 8, 16, 32, 64):
            g = B.System.from_system(sysm, "jacobi", spmv_lanes=lanes)
            ms = med_ms(g, lambda: g.spmv(v, z))
            row["lanes"][str(lanes)] = {"ms": ms, "gb_s": byts / ms / 1e6, "frac": byts / ms / 1e6 / HBM_PEAK_GBS}
            # a whole Jacobi-preconditioned GMRES(30) solve with this mapping in the
            # cycle kernel and the residual (the second of two; same bits for all)
            for _ in range(2):
                x, st = g.solve()
            gs = g.stats()
            row["lanes"][str(lanes)].update(solve_ms=gs["time_solve_ms"], refinements=gs["refinements"],
                                            relres=gs["relres_orig"], x_sha256=hashlib.sha256(x.tobytes()).hexdigest())
            if wl == "random27_1m" and lanes == 1:
                res["spmv"] = dict(row["lanes"]["1"], bytes=byts, workload=f"random27 n={n} nnz={nnz}")
                w2 = torch.from_numpy(rng.integers(-(1 << 30), 1 << 30, n)).cuda()
                dms = med_ms(g, lambda: g.dot(w2, v))  # Q30 words: no product overflows
                res["dot"] = {"ms": dms, "gb_s": 16 * n / dms / 1e6, "frac": 16 * n / dms / 1e6 / HBM_PEAK_GBS,
                              "bytes": 16 * n, "workload": f"random27 n={n}, two distinct vectors"}
                res["dot_by_length"] = dot_by_length(torch, B, rng)
                del w2
            g.close()
        for key, lanes in (("auto", 0), ("measured", -1)):
            g = B.System.from_system(sysm, "jacobi", m=2, spmv_lanes=lanes)
            row[key] = g.stats()["spmv_lanes"]
            g.close()
        best = min(row["lanes"], key=lambda k: row["lanes"][k]["ms"])
        row["fastest"] = int(best)
        row["same_x_every_mapping"] = len({r["x_sha256"] for r in row["lanes"].values()}) == 1
        res["spmv_mappings"][wl] = row
        progress(f"spmv mappings {wl}: " + ", ".join(f"{k}: {r['gb_s']:.0f} GB/s" for k, r in row["lanes"].items())
            + f"; auto {row['auto']}, measured {row['measured']}")
    return res

if __name__ == "__main__":
    main()
