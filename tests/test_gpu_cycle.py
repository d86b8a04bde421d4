"""GPU parity of the persistent int-GMRES(m) kernel and of whole solves.

The cycle trace (rotated H, c, s, g, the whole basis V, j*, breakdown, steps,
overflow code) must equal the oracle's bit for bit for every launch shape the
library can pick (workgroup count and rows per thread), and whole solves must
return the oracle's x bit for bit (the FP64 steps follow the same fixed
operation order and the norms are order-free)."""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_2009_07495_amd import binding as B
from paper_2009_07495_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = [
    ("poisson_37x29", lambda: W.poisson2d(37, 29), "paper_noprec", dict(m=20)),
    ("cd_12x11x9", lambda: W.convdiff3d(12, 11, 9, seed=7), "jacobi", dict(m=25)),
    ("r27_9x8x6", lambda: W.random27(9, 8, 6, seed=8), "paper_ilu", dict(m=20)),
    ("dd_257", lambda: W.random_dd(257, 0.03, 9), "paper_ilu", dict(m=30)),
    ("cd_multiterm", lambda: W.convdiff3d(9, 8, 7, seed=10), "jacobi", dict(m=15, alpha_a=24, s_terms=2)),
]
# cases whose refinement loop need not converge: cycle traces only
TRACE_ONLY = [
    # Jacobi with cast diagonals that are not powers of two, of both signs
    ("dd_weakdiag_jacobi", lambda: W.random_dd(257, 0.05, 7, dominance=0.1, nonneg_diag=False), "jacobi", dict(m=12)),
]


@pytest.fixture(scope="module")
def torch():
    import torch as T

    assert T.cuda.is_available(), "GPU tests need a HIP device"
    return T


def first_v1(o, n):
    r, _ = o.residual(np.zeros(n))
    return o.start_vector(r)["v1"]


def assert_trace_equal(tg, to, n):
    for k in ("jstar", "breakdown", "steps", "first_ovf"):
        assert tg[k] == to[k], (k, tg[k], to[k])
    assert np.array_equal(tg["H"], to["H"])
    assert np.array_equal(tg["c"], to["c"]) and np.array_equal(tg["s"], to["s"])
    assert np.array_equal(tg["g"], to["g"])
    assert np.array_equal(tg["V"], to["V"])


@pytest.mark.parametrize("name,gen,preset,kw", CASES + TRACE_ONLY)
@pytest.mark.parametrize("grid", [0, 1, 3, 7])
def test_cycle_trace_bit_exact_for_every_launch_shape(orc, torch, name, gen, preset, kw, grid):
    s = gen()
    o = orc.OracleSystem.from_system(s, orc.policy(preset, **kw))
    v1 = first_v1(o, s.n)
    to = o.cycle(v1)
    g = B.System.from_system(s, preset, grid_blocks=grid, **kw)
    st = g.stats()
    if grid:
        assert st["grid_blocks"] <= grid
    tg = g.int_cycle(v1)
    assert_trace_equal(tg, to, s.n)
    # a second call on the same system gives the same bits (no state leaks, no races)
    tg2 = g.int_cycle(v1)
    assert_trace_equal(tg2, to, s.n)


def test_cycle_trace_at_the_largest_m(orc, torch):
    """m = 1024, the policy's maximum: all 1024 Arnoldi steps run (no
    breakdown, no overflow) on a ragged 1100-row system, so the kernel's
    per-call arrays (H column, rotations, g, one synchronisation slot per
    grid sum) are exercised at their largest size."""
    s = W.random_dd(1100, 0.005, 77)
    o = orc.OracleSystem.from_system(s, orc.policy("jacobi", m=1024))
    v1 = first_v1(o, s.n)
    to = o.cycle(v1)
    assert to["steps"] == 1024 and to["breakdown"] == 0
    g = B.System.from_system(s, "jacobi", m=1024)
    assert_trace_equal(g.int_cycle(v1), to, s.n)


def test_cycle_breakdown_cases(orc, torch):
    n = 20
    b = np.zeros(n)
    b[5] = -2.0
    s = W.from_dense(3.0 * np.eye(n), b)
    for preset, kw in (("jacobi", dict(m=10)),):
        o = orc.OracleSystem.from_system(s, orc.policy(preset, **kw))
        g = B.System.from_system(s, preset, **kw)
        v1 = first_v1(o, n)
        to, tg = o.cycle(v1), g.int_cycle(v1)
        assert to["breakdown"] == 1
        assert_trace_equal(tg, to, n)
        x, st = g.solve()
        xo, sto = o.solve()
        assert st == B.OK and np.array_equal(x, xo)
    a = np.array([[1.0, 1.0], [1.0, 1.0]])
    s = W.from_dense(a, np.array([1.0, -1.0]))
    o = orc.OracleSystem.from_system(s, orc.policy("paper_noprec", m=5))
    g = B.System.from_system(s, "paper_noprec", m=5)
    v1 = first_v1(o, 2)
    to, tg = o.cycle(v1), g.int_cycle(v1)
    assert to["breakdown"] == 2 and to["jstar"] == 0
    assert_trace_equal(tg, to, 2)
    x, st = g.solve()
    assert st == B.ERR_BREAKDOWN and np.all(x == 0)


def test_overflow_code_matches(orc, torch):
    s = W.poisson2d(16)
    o = orc.OracleSystem.from_system(s, orc.policy("paper_noprec", alpha_a=40))
    g = B.System.from_system(s, "paper_noprec", alpha_a=40)
    v1 = first_v1(o, s.n)
    to, tg = o.cycle(v1), g.int_cycle(v1)
    assert to["first_ovf"] != orc.NO_EVENT
    assert_trace_equal(tg, to, s.n)
    xo, sto = o.solve()
    x, st = g.solve()
    assert st == B.ERR_OVERFLOW and sto["status"] == orc.ERR_OVERFLOW
    assert g.stats()["first_ovf"] == sto["first_ovf"]
    assert np.array_equal(x, xo)


SOLVES = [
    ("poisson_32", lambda: W.poisson2d(32), "paper_noprec", dict(m=30)),
    ("cd_16", lambda: W.convdiff3d(16, seed=2), "jacobi", dict(m=50)),
    ("r27_16x16x8", lambda: W.random27(16, 16, 8, seed=3), "paper_ilu", dict(m=30)),
    ("dd_64", lambda: W.random_dd(64, 0.2, 11, nonneg_diag=False), "paper_ilu", dict(m=10)),
    ("cd_multiterm", lambda: W.convdiff3d(9, 8, 7, seed=10), "jacobi", dict(m=15, alpha_a=24, s_terms=2)),
]
# cases whose refinement loop need not converge: cycle traces only
TRACE_ONLY = [
    # Jacobi with cast diagonals that are not powers of two, of both signs
    ("dd_weakdiag_jacobi", lambda: W.random_dd(257, 0.05, 7, dominance=0.1, nonneg_diag=False), "jacobi", dict(m=12)),
]


@pytest.mark.parametrize("name,gen,preset,kw", SOLVES)
def test_whole_solve_bit_exact(orc, torch, name, gen, preset, kw):
    s = gen()
    o = orc.OracleSystem.from_system(s, orc.policy(preset, **kw))
    xo, sto = o.solve()
    g = B.System.from_system(s, preset, **kw)
    x, st = g.solve()
    gs = g.stats()
    assert st == sto["status"] == B.OK
    assert gs["refinements"] == sto["refinements"] and gs["iterations"] == sto["iterations"]
    assert np.array_equal(x, xo)
    h = g.history()
    assert np.array_equal(h["relres_orig"], sto["hist_relres_orig"])
    k = gs["refinements"]
    assert np.array_equal(h["gamma"][:k], sto["hist_gamma"][:k])
    assert np.array_equal(h["rho"][:k], sto["hist_rho"][:k])
    assert np.array_equal(h["jstar"][:k], sto["hist_jstar"][:k])
    assert gs["relres_orig"] < 1e-10
    # device entry point with a torch buffer: same bits
    xd = torch.zeros(s.n, dtype=torch.float64, device="cuda")
    assert g.solve_device(xd) == B.OK
    assert np.array_equal(xd.cpu().numpy(), xo)


def test_resume_is_bit_identical(orc, torch):
    s = W.convdiff3d(12, seed=4)
    g = B.System.from_system(s, "jacobi", m=20)
    full, st = g.solve()
    g.set_policy(B.make_policy("jacobi", m=20, max_refine=2))
    part, st2 = g.solve()
    assert st2 == B.NOT_CONVERGED
    g.set_policy(B.make_policy("jacobi", m=20))
    rest, st3 = g.solve(part)
    assert st3 == B.OK and np.array_equal(rest, full)


def test_stream_and_rhs_updates(orc, torch):
    s = W.convdiff3d(10, seed=12)
    g = B.System.from_system(s, "jacobi", m=20)
    stream = torch.cuda.Stream()
    g.set_stream(stream)
    rng = np.random.default_rng(13)
    b2 = rng.uniform(-1, 1, s.n)
    g.set_rhs(b2)
    x, st = g.solve()
    s2 = W.System("cd", s.n, s.row_ptr, s.col, s.val, b2)
    xo, sto = orc.OracleSystem.from_system(s2, orc.policy("jacobi", m=20)).solve()
    assert st == B.OK and np.array_equal(x, xo)
    torch.cuda.synchronize()


def test_setup_thread_count_does_not_change_bits(torch, monkeypatch):
    """The host setup splits its passes (and the FP64 ILU(0) by level sets)
    over threads; one thread and many must give the same solve bit for bit
    (64,000 rows: above the size where the passes run in parallel)."""
    s = W.random27(40, 40, 40, seed=21)
    out = []
    for threads in ("1", "8"):
        monkeypatch.setenv("IGM_SETUP_THREADS", threads)
        g = B.System.from_system(s, "paper_ilu", m=30)
        x, st = g.solve()
        assert st == B.OK
        out.append((x, g.stats()["refinements"]))
        g.close()
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


ZERO_SHIFTS = dict(b_dot=0, b_axpy=0, b_norm=0, b_rot=0, b_tmp=0)
SHIFT_KEYS = ("b_dot", "b_axpy", "b_norm", "b_div_num", "b_div_den", "b_rot", "b_tmp", "b_cs_num", "b_cs_den")


@pytest.mark.parametrize("retries", [40, 3])
def test_shift_retry_matches_oracle(orc, torch, retries):
    """Overflow-driven shift retries (igm_policy.shift_retry): the same
    retries, the same adjusted shifts, the same status, event code and x bit
    for bit as the oracle, both when the retries repair the overflow (40) and
    when the limit ends the solve (3)."""
    s = W.poisson2d(32)
    kw = dict(ZERO_SHIFTS, shift_retry=retries)
    o = orc.OracleSystem.from_system(s, orc.policy("paper_noprec", **kw))
    xo, so = o.solve()
    g = B.System.from_system(s, "paper_noprec", **kw)
    x = torch.zeros(s.n, dtype=torch.float64, device="cuda")
    st = g.solve_device(x)
    gs = g.stats()
    assert st == so["status"] and gs["shift_retries"] == so["shift_retries"] > 0
    assert gs["refinements"] == so["refinements"] and gs["first_ovf"] == so["first_ovf"]
    pol = g.policy()
    assert all(pol[k] == o.policy_now()[k] for k in SHIFT_KEYS)
    assert np.array_equal(x.cpu().numpy(), xo)


def check_batched_result(r, x, xo, so, name):
    for k in ("status", "refinements", "iterations", "first_ovf", "shift_retries", "relres_orig", "relres_scaled"):
        assert r[k] == so[k], (name, k, r[k], so[k])
    assert np.array_equal(x, xo), (name, np.abs(x - xo).max())


def retry_systems():
    """Systems whose calls overflow with all product shifts at 0; the retries
    each needs differ (12 to 20), so the teams' shifts diverge; the 3000-row
    one is shared by two workgroups at 2048 rows each."""
    return [W.poisson2d(32), W.poisson2d(45, 37), W.poisson2d(7, 5), W.poisson2d(60, 50),
            W.from_dense(np.array([[2.5]]), np.array([-1.5]))]


@pytest.mark.parametrize("retries,shape", [(40, (256, 8)), (3, (256, 8)), (40, (1024, 4))])
def test_shift_retry_batched_matches_oracle(orc, torch, retries, shape):
    """Overflow-driven shift retries inside the batched kernel: each system's
    team adjusts its own working shifts and repeats the call; every system
    returns the oracle's status, retry count, event code, counts and x bit for
    bit, when the retries repair the overflow (40) and when the limit ends
    the solve (3)."""
    systems = retry_systems()
    kw = dict(ZERO_SHIFTS, shift_retry=retries, m=30)
    refs = [orc.OracleSystem.from_system(s, orc.policy("paper_noprec", **kw)).solve() for s in systems]
    assert all(so["shift_retries"] > 0 for _, so in refs)
    assert retries < 12 or len({so["shift_retries"] for _, so in refs}) > 1
    bt = B.Batch(systems, "paper_noprec", **kw)
    assert bt.set_shape(*shape) == B.OK
    if shape == (256, 8):
        assert bt.result(3)["grid_blocks"] == 2
    x, _ = bt.solve()
    for i, (s, (xo, so)) in enumerate(zip(systems, refs)):
        check_batched_result(bt.result(i), x[bt.offsets[i]:bt.offsets[i + 1]], xo, so, s.name)
    bt.close()


@pytest.mark.parametrize("retries", [40, 3])
def test_shift_retry_served_matches_oracle(orc, torch, retries):
    """The same retries for served requests, solved side by side."""
    systems = retry_systems()
    kw = dict(ZERO_SHIFTS, shift_retry=retries, m=30)
    sv = B.Server()
    try:
        tickets = [sv.submit(s, "paper_noprec", **kw) for s in systems]
        out = [sv.wait(t, 120000) for t in tickets]
    finally:
        sv.close(30000)
    for s, (x, st) in zip(systems, out):
        xo, so = orc.OracleSystem.from_system(s, orc.policy("paper_noprec", **kw)).solve()
        check_batched_result(st, x, xo, so, s.name)


@pytest.mark.parametrize("preset,gen", [("paper_noprec", lambda: W.poisson2d(37, 29)),
                                        ("jacobi", lambda: W.convdiff3d(14, 13, 12, seed=33)),
                                        ("paper_ilu", lambda: W.random27(12, 11, 10, seed=34))])
def test_two_sided_scaling_matches_oracle(orc, torch, preset, gen):
    """Eq. (eq2) with D1 = D2 = Dhat^(1/2) (igm_policy.two_sided): whole solves
    bit for bit against the oracle, residual history included."""
    s = gen()
    xo, so = orc.OracleSystem.from_system(s, orc.policy(preset, two_sided=1)).solve()
    g = B.System.from_system(s, preset, two_sided=1)
    x, st = g.solve()
    assert st == so["status"] == B.OK
    assert g.stats()["refinements"] == so["refinements"]
    h = g.history()
    assert np.array_equal(h["relres_orig"], so["hist_relres_orig"])
    assert np.array_equal(h["relres_scaled"], so["hist_relres_scaled"])
    assert np.array_equal(x, xo)


TWO_SIDED = [("paper_noprec", [lambda: W.poisson2d(37, 29), lambda: W.poisson2d(70, 60)]),
             ("jacobi", [lambda: W.convdiff3d(14, 13, 12, seed=33), lambda: W.convdiff2d(91, 77, seed=35)]),
             ("paper_ilu", [lambda: W.random27(12, 11, 10, seed=34), lambda: W.random27(20, 20, 12, seed=36)])]


@pytest.mark.parametrize("preset,gens", TWO_SIDED)
def test_two_sided_scaling_batched_and_served(orc, torch, preset, gens):
    """Eq. (eq2) in the batched kernel (the second system of each pair is
    shared by several workgroups) and in the served solver, with the scaling
    computed by the request's team on the device and on the host: every
    system returns the oracle's x bit for bit."""
    systems = [g() for g in gens]
    refs = [orc.OracleSystem.from_system(s, orc.policy(preset, two_sided=1)).solve() for s in systems]
    bt = B.Batch(systems, preset, two_sided=1)
    assert bt.set_shape(256, 8) == B.OK
    assert bt.result(1)["grid_blocks"] > 1
    x, _ = bt.solve()
    for i, (s, (xo, so)) in enumerate(zip(systems, refs)):
        assert so["status"] == B.OK
        check_batched_result(bt.result(i), x[bt.offsets[i]:bt.offsets[i + 1]], xo, so, s.name)
    bt.close()
    for host in (False, True):
        sv = B.Server(host_setup=host)
        try:
            out = [sv.wait(t, 120000) for t in [sv.submit(s, preset, two_sided=1) for s in systems]]
        finally:
            sv.close(30000)
        for s, (xs, st), (xo, so) in zip(systems, out, refs):
            check_batched_result(st, xs, xo, so, (s.name, host))


@pytest.mark.parametrize("gen", [lambda: W.convdiff2d(91, 77, seed=41), lambda: W.random27(20, 20, 12, seed=42),
                                 lambda: W.random27(40, 40, 40, seed=43)])
def test_gauss_seidel_matches_oracle(orc, torch, gen):
    """The Gauss-Seidel splitting (igm_policy.gauss_seidel) through the
    single-system and the batched solver: whole solves bit for bit against the
    oracle (the last case, 64,000 rows, builds its factors on several host
    threads and sweeps with the level counters)."""
    s = gen()
    xo, so = orc.OracleSystem.from_system(s, orc.policy("paper_ilu", gauss_seidel=1)).solve()
    g = B.System.from_system(s, "paper_ilu", gauss_seidel=1)
    x, st = g.solve()
    assert st == so["status"] == B.OK and g.stats()["refinements"] == so["refinements"]
    assert g.stats()["levels_bwd"] == 1  # Ubar is diagonal
    assert np.array_equal(x, xo)
    bt = B.Batch([s], "paper_ilu", gauss_seidel=1)
    xb, stb = bt.solve()
    assert stb == B.OK and np.array_equal(xb, xo)


def test_abi_error_statuses_match_oracle(orc, torch):
    """The failure statuses of the C ABI, forced from the host, equal the
    oracle's: an all-zero row, a NaN entry, unsorted columns, a structurally
    zero ILU pivot, a bad policy; and non-convergence (one refinement at
    tol 1e-14) returns the oracle's best iterate bit for bit."""
    s = W.random_dd(10, 0.3, 15)
    cases = []
    val = s.val.copy()
    val[s.row_ptr[3]:s.row_ptr[4]] = 0.0
    cases.append((W.System("zero row", s.n, s.row_ptr, s.col, val, s.b), "paper_noprec", {}))
    val = s.val.copy()
    val[0] = np.nan
    cases.append((W.System("nan", s.n, s.row_ptr, s.col, val, s.b), "paper_noprec", {}))
    col = s.col.copy()
    col[s.row_ptr[2]], col[s.row_ptr[2] + 1] = col[s.row_ptr[2] + 1], col[s.row_ptr[2]]
    cases.append((W.System("unsorted", s.n, s.row_ptr, col, s.val, s.b), "paper_noprec", {}))
    cases.append((W.from_dense(np.array([[0.0, 1.0], [1.0, 1.0]]), np.ones(2)), "paper_ilu", {}))
    cases.append((s, "paper_noprec", dict(df=70)))
    for sysm, preset, kw in cases:
        with pytest.raises(orc.OracleError) as eo:
            orc.OracleSystem.from_system(sysm, orc.policy(preset, **kw))
        with pytest.raises(B.IgmError) as eg:
            B.System.from_system(sysm, preset, **kw)
        assert eg.value.status == eo.value.status, (sysm.name, eg.value.status, eo.value.status)
    big = W.convdiff3d(12, seed=9)
    xo, so = orc.OracleSystem.from_system(big, orc.policy("jacobi", m=10, max_refine=1, tol=1e-14)).solve()
    g = B.System.from_system(big, "jacobi", m=10, max_refine=1, tol=1e-14)
    x, st = g.solve()
    assert st == so["status"] == B.NOT_CONVERGED
    assert np.array_equal(x, xo) and g.stats()["relres_orig"] == so["relres_orig"]


def _golden():
    path = os.path.join(HERE, "golden", "oracle_runs.json")
    return json.load(open(path)) if os.path.exists(path) else {}


@pytest.mark.parametrize("name", ["poisson2d_64", "convdiff3d_64", "random27_1m"])
def test_full_size_workload_matches_recorded_oracle_run(torch, name):
    """Full-size workloads against the oracle's recorded whole-solve results
    (tests/golden/make_oracle_runs.py): same refinement count, same residual
    history, and the solution's bytes hash to the oracle's."""
    gold = _golden().get(name)
    if gold is None:
        pytest.skip("no recorded oracle run")
    gen, preset, m = W.WORKLOADS[name]
    s = gen()
    g = B.System.from_system(s, preset, m=m)
    x, st = g.solve()
    gs = g.stats()
    print(name, gs)
    assert st == B.OK and gs["relres_orig"] <= 1e-10
    assert gs["refinements"] == gold["refinements"] and gs["iterations"] == gold["iterations"]
    h = g.history()
    assert [float(v) for v in h["relres_orig"]] == gold["hist_relres_orig"]
    if name == "random27_1m":  # level sets of the ILU(0) factors of this matrix
        assert gs["levels_fwd"] == 634 and gs["levels_bwd"] == 634
    assert hashlib.sha256(x.tobytes()).hexdigest() == gold["x_sha256"]


@pytest.mark.parametrize("lanes", [1, 2, 16])
def test_full_size_skewed_solve_every_mapping(torch, lanes):
    """The 1M-row heavy-tailed matrix (the SpMV mappings' benchmark matrix)
    solved at full size with one thread per row over SELL-64, the merge split
    and 16 lanes per row: each matches the oracle's recorded whole solve
    (refinements, residual history, solution hash)."""
    gold = _golden().get("skewed_1m")
    if gold is None:
        pytest.skip("no recorded oracle run")
    gen, preset, m = W.WORKLOADS["skewed_1m"]
    g = B.System.from_system(gen(), preset, m=m, spmv_lanes=lanes)
    x, st = g.solve()
    gs = g.stats()
    assert st == B.OK and gs["relres_orig"] <= 1e-10 and gs["spmv_lanes"] == lanes
    assert gs["refinements"] == gold["refinements"] and gs["iterations"] == gold["iterations"]
    assert [float(v) for v in g.history()["relres_orig"]] == gold["hist_relres_orig"]
    assert hashlib.sha256(x.tobytes()).hexdigest() == gold["x_sha256"]
    g.close()


ILU_SWEEP_CASES = [
    ("r27_11x9x8", lambda: W.random27(11, 9, 8, seed=31), dict(m=12)),
    ("dd_301_ragged", lambda: W.random_dd(301, 0.04, 32), dict(m=10)),
    ("cd_13x12x7_ilu", lambda: W.convdiff3d(13, 12, 7, seed=33), dict(m=12)),
]


@pytest.mark.parametrize("name,gen,kw", ILU_SWEEP_CASES)
@pytest.mark.parametrize("rows,lanes", [(64, 4), (64, 8), (64, 16), (128, 8), (192, 16), (320, 4), (0, 0)])
def test_ilu_blocked_sweeps_any_block_size(orc, torch, name, gen, kw, rows, lanes):
    """The ILU(0) preconditioner apply runs block by block (Sec. VI; blocks of
    `rows` consecutive rows; every accepted `sweep_lanes` value): small blocks force many
    blocks, waits on earlier blocks' progress across workgroups and, with
    fewer workgroups than blocks, workgroups that run several blocks in turn.
    The cycle trace (whole basis included) and a whole solve (whose FP64
    start step runs the same schedules) equal the oracle's bit for bit."""
    s = gen()
    o = orc.OracleSystem.from_system(s, orc.policy("paper_ilu", **kw))
    v1 = first_v1(o, s.n)
    to = o.cycle(v1)
    for grid in (0, 2):
        g = B.System.from_system(s, "paper_ilu", grid_blocks=grid, sweep_rows=rows, sweep_lanes=lanes, **kw)
        assert_trace_equal(g.int_cycle(v1), to, s.n)
        x, st = g.solve()
        xo, so = o.solve()
        assert st == so["status"] and np.array_equal(x, xo), (name, rows, lanes, grid)
        g.close()


@pytest.mark.parametrize("rule", [0, 1])
def test_s_schedule_matches_oracle(orc, torch, rule):
    """s(k) of eq. (AA): the call of refinement k uses Abar_0 and s(k)
    correction matrices (rule 1: s(k) = min(S, k - 1)). The cycle traces of
    refinements 1 to 3 and a whole solve equal the oracle's bit for bit."""
    s = W.convdiff3d(9, 8, 7, seed=10)
    kw = dict(m=15, alpha_a=24, s_terms=2, s_rule=rule)
    o = orc.OracleSystem.from_system(s, orc.policy("jacobi", **kw))
    g = B.System.from_system(s, "jacobi", **kw)
    v1 = first_v1(o, s.n)
    for k in (1, 2, 3):
        assert_trace_equal(g.int_cycle(v1, k=k), o.cycle(v1, k=k), s.n)
    x, st = g.solve()
    xo, so = o.solve()
    assert st == so["status"] == B.OK and np.array_equal(x, xo)
    assert g.stats()["refinements"] == so["refinements"]


SPMV_LANE_CASES = [
    ("poisson_37x29", lambda: W.poisson2d(37, 29), "paper_noprec", dict(m=20)),
    ("skewed_3001", lambda: W.skewed(3001, seed=12), "jacobi", dict(m=20)),
    ("skewed_2500_multiterm", lambda: W.skewed(2500, mean_len=30.0, seed=13), "jacobi",
     dict(m=15, alpha_a=24, s_terms=2)),
    ("r27_9x8x6", lambda: W.random27(9, 8, 6, seed=8), "paper_ilu", dict(m=20)),
    ("arrow_3000", lambda: W.arrow(3000), "jacobi", dict(m=20)),
    ("arrow_2100_ilu", lambda: W.arrow(2100, seed=9), "paper_ilu", dict(m=12)),
]


@pytest.mark.parametrize("name,gen,preset,kw", SPMV_LANE_CASES)
@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64, -1])
def test_spmv_lane_mappings_bit_exact(orc, torch, name, gen, preset, kw, lanes):
    """The integer SpMV inside the cycle kernel with one thread per row over
    SELL-64 (1), each workgroup's rows split evenly by entries (2), or 4, 16,
    64 lanes per row over CSR (-1: the mapping measured at setup), and the
    FP64 residual of the refinement loop with its mapping: the cycle trace
    (whole basis) and a whole solve equal the oracle's bit for bit, with the
    library's own and with 3 workgroups."""
    s = gen()
    o = orc.OracleSystem.from_system(s, orc.policy(preset, **kw))
    v1 = first_v1(o, s.n)
    to = o.cycle(v1)
    xo, so = o.solve()
    for grid in (0, 3):
        g = B.System.from_system(s, preset, grid_blocks=grid, spmv_lanes=lanes, **kw)
        got = g.stats()["spmv_lanes"]
        assert got == lanes if lanes > 0 else got in (1, 2, 4, 8, 16, 32, 64)
        assert_trace_equal(g.int_cycle(v1), to, s.n)
        x, st = g.solve()
        assert st == so["status"] and np.array_equal(x, xo), (name, lanes, grid)
        g.close()


def test_automatic_spmv_lanes_follow_the_row_lengths(torch):
    """The automatic mapping: one thread per row for stencils (SELL-64 pads
    little), the even split by entries for heavy-tailed row lengths (SELL-64
    would load more than twice the entries)."""
    for gen, want in ((lambda: W.poisson2d(40, 30), 1), (lambda: W.random27(9, 8, 6, seed=8), 1),
                      (lambda: W.skewed(3001, seed=12), 2), (lambda: W.skewed(2500, mean_len=30.0, seed=13), 2),
                      (lambda: W.arrow(3000), 2)):
        g = B.System.from_system(gen(), "jacobi")
        assert g.stats()["spmv_lanes"] == want
        g.close()
