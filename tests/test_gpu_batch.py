"""GPU parity of the batched solver (many independent systems, one persistent
launch).

Every system of a batch must come back with the oracle's solution bit for bit
and the oracle's status, refinement and iteration counts and final relative
residuals, whatever its team size (workgroups per system), the launch shape,
and the other systems in the batch. The full 512-system workload is checked on
sampled systems the oracle solves one by one, plus the convergence of all."""
import numpy as np
import pytest

from paper_2009_07495_amd import binding as B
from paper_2009_07495_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPES = [(1024, 8), (1024, 4), (512, 8), (512, 16), (256, 8), (256, 16)]


@pytest.fixture(scope="module")
def torch():
    import torch as T

    assert T.cuda.is_available(), "GPU tests need a HIP device"
    return T


def mixed_jacobi():
    """Ragged sizes (not multiples of 64), 2D and 3D stencils, one
    unstructured system, one single-row system."""
    return [
        W.convdiff2d(37, 29, seed=11),
        W.convdiff3d(12, 11, 9, seed=12),
        W.random_dd(301, 0.02, 13),
        W.convdiff2d(91, 77, seed=14),       # 7007 rows: two workgroups at 4096 rows each
        W.from_dense(np.array([[2.5]]), np.array([-1.5])),
        W.convdiff3d(23, 19, 17, seed=15),   # 7429 rows
        W.convdiff2d(5, 3, seed=16),
    ]


def oracle_solve(orc, s, preset, **kw):
    o = orc.OracleSystem.from_system(s, orc.policy(preset, **kw))
    return o.solve()


def check_against_oracle(bt, x, systems, refs):
    for i, (s, (xo, so)) in enumerate(zip(systems, refs)):
        r = bt.result(i)
        xi = x[bt.offsets[i]:bt.offsets[i + 1]]
        assert r["status"] == so["status"], (i, s.name, r["status"], so["status"])
        assert r["refinements"] == so["refinements"], (i, s.name)
        assert r["iterations"] == so["iterations"], (i, s.name)
        assert r["first_ovf"] == so["first_ovf"], (i, s.name)
        assert r["relres_orig"] == so["relres_orig"] and r["relres_scaled"] == so["relres_scaled"], (i, s.name)
        assert np.array_equal(xi, xo), (i, s.name, np.abs(xi - xo).max())


@pytest.mark.parametrize("block,rows", SHAPES)
def test_batch_bit_exact_every_shape(orc, torch, block, rows):
    systems = mixed_jacobi()
    refs = [oracle_solve(orc, s, "jacobi", m=20) for s in systems]
    bt = B.Batch(systems, "jacobi", m=20)
    assert bt.set_shape(block, rows) == B.OK
    teams = [bt.result(i)["grid_blocks"] for i in range(bt.nsys)]
    assert teams == [-(-s.n // (block * rows)) for s in systems]
    x = torch.zeros(bt.total_n, dtype=torch.float64, device="cuda")
    assert bt.solve_device(x) == B.OK
    check_against_oracle(bt, x.cpu().numpy(), systems, refs)
    # a second solve of the same batch from zero gives the same bits
    x.zero_()
    assert bt.solve_device(x) == B.OK
    check_against_oracle(bt, x.cpu().numpy(), systems, refs)


def test_batch_teams_of_many_workgroups(orc, torch):
    """Systems split over up to 25 workgroups of 256 threads x 8 rows (and
    8 workgroups of 256 x 16)."""
    systems = [W.convdiff2d(181, 179, seed=21), W.convdiff3d(20, 20, 13, seed=22), W.convdiff2d(30, 30, seed=23),
               W.convdiff3d(37, 37, 37, seed=24)]
    refs = [oracle_solve(orc, s, "jacobi", m=30) for s in systems]
    bt = B.Batch(systems, "jacobi", m=30)
    for shape, teams in (((256, 16), [8, 2, 1, 13]), ((256, 8), [16, 3, 1, 25])):
        assert bt.set_shape(*shape) == B.OK
        assert [bt.result(i)["grid_blocks"] for i in range(4)] == teams
        x, st = bt.solve()
        assert st == B.OK
        check_against_oracle(bt, x, systems, refs)


@pytest.mark.parametrize("block,rows", [(1024, 4), (256, 8)])
def test_batch_ilu_bit_exact(orc, torch, block, rows):
    """ILU(0) preconditioned systems (Sec. VI): level-scheduled integer sweeps
    and the FP64 substitution of the start step inside a team, including teams of
    several workgroups (the 4800- and 7007-row systems at 2048 rows each)."""
    systems = [W.random27(9, 8, 6, seed=61), W.random_dd(300, 0.05, 62), W.random27(20, 20, 12, seed=63),
               W.convdiff2d(91, 77, seed=64), W.random27(5, 4, 3, seed=65)]
    refs = [oracle_solve(orc, s, "paper_ilu", m=30) for s in systems]
    bt = B.Batch(systems, "paper_ilu", m=30)
    assert bt.set_shape(block, rows) == B.OK
    x, st = bt.solve()
    assert st == B.OK
    check_against_oracle(bt, x, systems, refs)


def test_batch_paper_noprec_preset(orc, torch):
    systems = [W.poisson2d(37, 29), W.poisson2d(20, 20), W.poisson2d(64)]
    refs = [oracle_solve(orc, s, "paper_noprec", m=30) for s in systems]
    bt = B.Batch(systems, "paper_noprec", m=30)
    x, st = bt.solve()
    assert st == B.OK
    check_against_oracle(bt, x, systems, refs)
    # Poisson right-hand sides are A * ones
    assert np.abs(x - 1.0).max() < 1e-8


@pytest.mark.parametrize("rule", [0, 1])
def test_batch_s_schedule(orc, torch, rule):
    """s(k) of eq. (AA) in the batched kernel: each system's call of
    refinement k uses Abar_0 and s(k) correction matrices (rule 1:
    min(S, k - 1)); every system equals the oracle bit for bit."""
    systems = [W.convdiff3d(9, 8, 7, seed=10), W.convdiff2d(31, 27, seed=11), W.convdiff3d(12, 10, 6, seed=12)]
    kw = dict(m=15, alpha_a=24, s_terms=2, s_rule=rule)
    refs = [oracle_solve(orc, s, "jacobi", **kw) for s in systems]
    bt = B.Batch(systems, "jacobi", **kw)
    x, st = bt.solve()
    assert st == B.OK
    check_against_oracle(bt, x, systems, refs)


def test_batch_matches_single_system_solver(torch):
    systems = [W.convdiff3d(14, 13, 12, seed=31), W.convdiff2d(70, 61, seed=32)]
    bt = B.Batch(systems, "jacobi", m=25)
    xb, st = bt.solve()
    assert st == B.OK
    for i, s in enumerate(systems):
        g = B.System.from_system(s, "jacobi", m=25)
        xs, st1 = g.solve()
        assert st1 == B.OK
        assert np.array_equal(xb[bt.offsets[i]:bt.offsets[i + 1]], xs)
        assert bt.result(i)["refinements"] == g.stats()["refinements"]


def test_batch_status_cases(orc, torch):
    """A breakdown system, a system stopped by the refinement limit and a
    normal one in the same batch: each gets its own status; the batch returns
    the first non-OK status in system order."""
    n = 20
    b = np.zeros(n)
    b[5] = -2.0
    brk = W.from_dense(3.0 * np.eye(n), b)        # A = cI: exact after one column
    slow = W.convdiff3d(11, 10, 9, seed=41)
    ok = W.convdiff2d(16, 15, seed=42)
    systems = [ok, slow, brk]
    kw = dict(m=5, max_refine=3)
    refs = [oracle_solve(orc, s, "jacobi", **kw) for s in systems]
    bt = B.Batch(systems, "jacobi", **kw)
    x, st = bt.solve()
    check_against_oracle(bt, x, systems, refs)
    statuses = [r["status"] for r in bt.results()]
    first_bad = next((s for s in statuses if s != B.OK), B.OK)
    assert st == first_bad
    assert refs[1][1]["status"] == B.NOT_CONVERGED


def test_batch_start_iterate(orc, torch):
    systems = [W.convdiff2d(33, 31, seed=51), W.convdiff3d(9, 9, 9, seed=52)]
    bt = B.Batch(systems, "jacobi", m=10)
    rng = np.random.default_rng(5)
    x0 = rng.uniform(-1, 1, bt.total_n)
    x, st = bt.solve(x0)
    assert st == B.OK
    for i, s in enumerate(systems):
        o = orc.OracleSystem.from_system(s, orc.policy("jacobi", m=10))
        xo, so = o.solve(x0[bt.offsets[i]:bt.offsets[i + 1]])
        assert np.array_equal(x[bt.offsets[i]:bt.offsets[i + 1]], xo)
        assert bt.result(i)["refinements"] == so["refinements"]


def test_batch_rejects_bad_input(torch):
    good = W.convdiff2d(8, 8, seed=1)
    bad = W.convdiff2d(8, 8, seed=2)
    bad.col = bad.col.copy()
    bad.col[3] = 10_000  # column out of range
    with pytest.raises(B.IgmError) as e:
        B.Batch([good, bad], "jacobi", m=10)
    assert e.value.status == B.ERR_ARG and "system 1" in str(e.value)
    with pytest.raises(B.IgmError) as e:
        B.Batch([good], "jacobi", m=65)  # H of the call lives in LDS: m <= 64
    assert e.value.status == B.ERR_UNSUPPORTED
    bt = B.Batch([good], "jacobi", m=10)
    assert bt.set_shape(300, 8) == B.ERR_ARG
    assert bt.set_shape(1024, 8) == B.OK


def test_batch_full_512_every_system(orc, torch):
    """The 512-system workload at full size: every system converges, the
    launch shape is autotuned, and every system's solution equals the
    oracle's bit for bit (SHA-256 of x, refinement and iteration counts and
    the final relative residual from tests/golden/batch512_oracle.json,
    written by tests/golden/make_batch512_runs.py, which calls only the
    oracle); two systems are also solved by the oracle here."""
    import hashlib
    import json
    import os

    with open(os.path.join(os.path.dirname(__file__), "golden", "batch512_oracle.json")) as f:
        golden = json.load(f)
    systems = W.batch_systems(512, seed=4)
    assert golden["count"] == len(systems) and golden["m"] == 30 and golden["preset"] == "jacobi"
    bt = B.Batch(systems, "jacobi", m=30)
    block, rows = bt.autotune()
    assert (block, rows) in SHAPES
    x = torch.zeros(bt.total_n, dtype=torch.float64, device="cuda")
    assert bt.solve_device(x) == B.OK
    res = bt.results()
    xh = x.cpu().numpy()
    for i, (s, r, gd) in enumerate(zip(systems, res, golden["systems"])):
        assert gd["index"] == i and gd["name"] == s.name and gd["n"] == s.n, i
        assert r["status"] == gd["status"] == B.OK and r["relres_orig"] == gd["relres_orig"] < 1e-10, i
        assert r["refinements"] == gd["refinements"] and r["iterations"] == gd["iterations"], i
        xi = np.ascontiguousarray(xh[bt.offsets[i]:bt.offsets[i + 1]])
        assert hashlib.sha256(xi.tobytes()).hexdigest() == gd["x_sha256"], (i, s.name)
    for i in (7, 301):  # the recorded hashes match a fresh oracle solve
        xo, so = oracle_solve(orc, systems[i], "jacobi", m=30)
        assert hashlib.sha256(xo.tobytes()).hexdigest() == golden["systems"][i]["x_sha256"]
    bt.close()
