"""Pins for the oracle's whole solve (Fig. 1 around Fig. 2): dense FP64 solves
on small systems, the known solution of the Poisson workload, the paper's
qualitative claims (gamma decreasing, counts in multiples of m, at most about
one extra refinement over FP64 GMRES(m)) and the error/resume paths."""
import numpy as np
import pytest

from paper_2009_07495_amd import workloads as W


def make(orc, sysm, preset, **kw):
    return orc.OracleSystem.from_system(sysm, orc.policy(preset, **kw))


def true_relres(sysm, x):
    return np.linalg.norm(sysm.b - sysm.matvec(x)) / np.linalg.norm(sysm.b)


@pytest.mark.parametrize("preset", ["paper_noprec", "paper_ilu", "jacobi"])
@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (5, 2), (17, 3), (64, 4)])
def test_small_systems_match_dense_solve(orc, preset, n, seed):
    s = W.random_dd(n, 0.3, seed, nonneg_diag=(seed % 2 == 0))
    o = make(orc, s, preset, m=min(10, n + 1))
    x, st = o.solve()
    assert st["status"] == orc.OK, st
    assert st["relres_orig"] < 1e-10
    assert true_relres(s, x) < 1e-10
    xd = np.linalg.solve(s.dense(), s.b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.cond(s.dense()) * np.linalg.norm(xd)


def test_poisson_workload_known_solution_and_paper_claims(orc):
    """b = A 1, so x = 1; int-GMRES needs no more than ~1.25x the FP64 GMRES(m)
    iterations or one extra refinement (Sec. VII-B); counts are multiples of m
    because the residual is checked once per refinement (Sec. VII-A)."""
    s = W.poisson2d(64)
    m = 30
    o = make(orc, s, "paper_noprec", m=m)
    x, st = o.solve()
    assert st["status"] == orc.OK and st["first_ovf"] == orc.NO_EVENT
    assert np.abs(x - 1.0).max() < 1e-7
    assert st["iterations"] == st["refinements"] * m
    _, it64, rc = o.gmres64()
    assert rc == orc.OK and it64 % m == 0
    assert st["iterations"] <= 1.25 * it64 + m
    g = st["hist_gamma"][: st["refinements"]]
    assert np.all(np.diff(g) < 0)  # gamma^(k) decreases (Sec. IV-A)
    ro = st["hist_relres_orig"]
    assert ro[0] == 1.0 and ro[-1] < 1e-10


def test_ilu_and_jacobi_workload_shapes_converge(orc):
    for sysm, preset, m in ((W.random27(12, 12, 8, seed=3), "paper_ilu", 30),
                            (W.convdiff3d(12, seed=2), "jacobi", 50)):
        o = make(orc, sysm, preset, m=m)
        x, st = o.solve()
        assert st["status"] == orc.OK, (preset, st)
        assert true_relres(sysm, x) < 1e-10
        _, it64, _ = o.gmres64()
        assert st["refinements"] <= np.ceil(it64 / m) * 1.25 + 1


def test_skewed_generator_shape_and_solve(orc):
    """The heavy-tailed family: CSR well formed (sorted distinct columns, one
    diagonal per row), strictly diagonally dominant, row lengths heavy-tailed
    (median well below the mean's tail, longest row tens of times the mean),
    the same matrix for the same seed; the oracle solves it to 1e-10."""
    s = W.skewed(4099, seed=11)
    rp, col, val = s.row_ptr, s.col, s.val
    lens = np.diff(rp)
    assert rp[0] == 0 and rp[-1] == len(col) == len(val) and np.all(lens >= 1)
    rows = np.repeat(np.arange(s.n), lens)
    assert np.all((np.diff(col) > 0) | (np.diff(rows) > 0))  # sorted, distinct within a row
    diag = col == rows
    assert np.array_equal(np.bincount(rows[diag], minlength=s.n), np.ones(s.n))
    offsum = np.bincount(rows[~diag], weights=np.abs(val[~diag]), minlength=s.n)
    assert np.all(val[diag] > offsum)
    assert lens.max() > 30 * lens.mean() and np.median(lens) < lens.mean()
    t = W.skewed(4099, seed=11)
    assert np.array_equal(t.col, col) and np.array_equal(t.val, val) and np.array_equal(t.b, s.b)
    o = make(orc, s, "jacobi", m=20)
    x, st = o.solve()
    assert st["status"] == orc.OK and true_relres(s, x) < 1e-10


def test_multiterm_matrix_solve(orc):
    """s = 2 correction matrices (eq. (AA)) with a coarse alpha_a still solves."""
    s = W.convdiff3d(6, seed=9)
    o = make(orc, s, "jacobi", alpha_a=24, s_terms=2, m=20)
    assert o.nterms == 3
    x, st = o.solve()
    assert st["status"] == orc.OK and true_relres(s, x) < 1e-10


def test_overflow_is_reported_with_its_position(orc):
    """The no-preconditioner shifts (beta = 16) with alpha_a = 40 overflow the
    normalisation's numerator shift (|w| 2^(30+16) >= 2^63) in the first step."""
    s = W.poisson2d(16)
    o = make(orc, s, "paper_noprec", alpha_a=40)
    x, st = o.solve()
    assert st["status"] == orc.ERR_OVERFLOW
    j = st["first_ovf"] >> 24
    stage = (st["first_ovf"] >> 16) & 0xFF
    assert j == 1 and stage in (1, 3, 4, 5), hex(st["first_ovf"])
    assert np.all(x == 0)  # the failed refinement is not applied


def test_not_converged_keeps_best_iterate(orc):
    s = W.poisson2d(16)
    o = make(orc, s, "paper_noprec", max_refine=1, tol=1e-14)
    x, st = o.solve()
    assert st["status"] == orc.NOT_CONVERGED and st["refinements"] == 1
    assert st["relres_orig"] < 1.0


def test_resume_from_partial_solution_is_bit_identical(orc):
    """The refinement state is x alone (Fig. 1): stopping after k refinements and
    restarting from that x reproduces the uninterrupted run bit for bit."""
    s = W.convdiff3d(8, seed=4)
    full, st_full = make(orc, s, "jacobi", m=20).solve()
    part, st_part = make(orc, s, "jacobi", m=20, max_refine=2).solve()
    assert st_part["status"] == orc.NOT_CONVERGED
    rest, st_rest = make(orc, s, "jacobi", m=20).solve(x0=part)
    assert st_rest["status"] == orc.OK
    assert st_part["refinements"] + st_rest["refinements"] == st_full["refinements"]
    assert np.array_equal(rest, full)


def test_fp64_comparator_solves(orc):
    s = W.random_dd(50, 0.2, 7)
    for preset in ("paper_noprec", "paper_ilu", "jacobi"):
        o = make(orc, s, preset, m=10)
        x, it, rc = o.gmres64(tol=1e-12)
        assert rc == orc.OK and it % 1 == 0
        assert true_relres(s, x) < 1e-12


# ---- overflow-driven shift retry (a reading: the paper names an auto-tuning
# of the shift for the solver without preconditioner, Sec. VII-D, but gives
# no rule; the rule is documented at orc_shift_retry) ----

ZERO_SHIFTS = dict(b_dot=0, b_axpy=0, b_norm=0, b_rot=0, b_tmp=0)
SHIFT_KEYS = ("b_dot", "b_axpy", "b_norm", "b_div_num", "b_div_den", "b_rot", "b_tmp", "b_cs_num", "b_cs_den")


def code(j, stage, sub=0):
    return (j << 24) | (stage << 16) | sub


def test_shift_retry_rule_by_stage(orc):
    base = orc.policy("paper_noprec", **ZERO_SHIFTS)
    expect = {
        code(1, 3, 0): ("b_dot", 4), code(2, 3, 3): ("b_axpy", 4), code(1, 4): ("b_norm", 4),
        code(1, 5): ("b_div_num", 12), code(1, 6, 1): ("b_rot", 4), code(1, 7): ("b_tmp", 4),
        code(1, 8): ("b_cs_num", 12),
    }
    for c, (key, val) in expect.items():
        changed, p = orc.shift_retry(base, c)
        assert changed and p[key] == val, (hex(c), key, p[key])
        assert all(p[k] == base[k] for k in SHIFT_KEYS if k != key)
    # no shift can prevent an overflow in the SpMV, the preconditioner apply or
    # the rotation of g, or without an event
    for c in (code(1, 1), code(1, 2), code(1, 9), orc.NO_EVENT):
        assert orc.shift_retry(base, c)[0] is False
    # limits: raised shifts stop at df; a division's numerator exponent goes
    # to 0, then its denominator's
    changed, p = orc.shift_retry(dict(base, b_dot=28), code(1, 3, 0))
    assert changed and p["b_dot"] == 30
    assert orc.shift_retry(dict(base, b_dot=30), code(1, 3, 0))[0] is False
    changed, p = orc.shift_retry(dict(base, b_div_num=0, b_div_den=3), code(1, 5))
    assert changed and p["b_div_num"] == 0 and p["b_div_den"] == 0
    assert orc.shift_retry(dict(base, b_div_num=0, b_div_den=0), code(1, 5))[0] is False


def test_shift_retry_repairs_overflow_and_equals_a_solve_with_the_final_shifts(orc):
    """Zero shifts overflow in the first inner product (Q30 x Q30 products of
    the unpreconditioned Poisson matrix). With retries the solve converges,
    every retry happens in the first refinement, so the result must equal, bit
    for bit, a fresh solve that starts from the shifts the retries ended with."""
    s = W.poisson2d(32)
    x0, st0 = make(orc, s, "paper_noprec", **ZERO_SHIFTS).solve()
    assert st0["status"] == orc.ERR_OVERFLOW and (st0["first_ovf"] >> 16) & 0xFF == 3
    o = make(orc, s, "paper_noprec", shift_retry=40, **ZERO_SHIFTS)
    x1, st1 = o.solve()
    assert st1["status"] == orc.OK and st1["relres_orig"] < 1e-10
    assert 0 < st1["shift_retries"] <= 40
    final = {k: o.policy_now()[k] for k in SHIFT_KEYS}
    assert final["b_dot"] > 0 and final["b_norm"] > 0
    x2, st2 = make(orc, s, "paper_noprec", **dict(ZERO_SHIFTS, **final)).solve()
    assert st2["status"] == orc.OK and st2["shift_retries"] == 0
    assert np.array_equal(x1, x2) and st1["refinements"] == st2["refinements"]
    assert np.abs(x1 - 1.0).max() < 1e-8  # Poisson right-hand side = A * ones


def test_shift_retry_limit_and_unretryable_stage(orc):
    s = W.poisson2d(16)
    o = make(orc, s, "paper_noprec", shift_retry=3, **ZERO_SHIFTS)
    x, st = o.solve()
    # three raises of b_dot (0 -> 12) are not enough: still the inner-product overflow
    assert st["status"] == orc.ERR_OVERFLOW and st["shift_retries"] == 3
    assert o.policy_now()["b_dot"] == 12 and (st["first_ovf"] >> 16) & 0xFF == 3
    assert np.all(x == 0)
    # an overflow in the SpMV (alpha_a = 62: entries near 2^62 times Q30
    # vector words) cannot be retried
    o = make(orc, s, "paper_noprec", alpha_a=62, shift_retry=8)
    x, st = o.solve()
    assert st["status"] == orc.ERR_OVERFLOW and st["shift_retries"] == 0
    assert (st["first_ovf"] >> 16) & 0xFF == 1


def test_shift_retry_is_inert_without_overflow(orc):
    s = W.convdiff3d(10, seed=3)
    xa, sa = make(orc, s, "jacobi", m=20).solve()
    xb, sb = make(orc, s, "jacobi", m=20, shift_retry=16).solve()
    assert sb["shift_retries"] == 0 and np.array_equal(xa, xb) and sa["refinements"] == sb["refinements"]


# ---- two-sided scaling, eq. (eq2): a reading (the paper leaves D1 and D2
# open); D1 = D2 = Dhat^(1/2) with Dhat from eq. (eq3), see orc_setup.c ----

def test_two_sided_scaling_keeps_symmetry(orc):
    import scipy.sparse as sp

    s = W.poisson2d(9, 7)
    o = make(orc, s, "paper_noprec", two_sided=1)
    d, a, b = o.scaled()
    A = sp.csr_matrix((a, s.col, s.row_ptr), shape=(s.n, s.n))
    assert (A != A.T).nnz == 0  # bit for bit
    # b = D1^-1 bhat, and A = D1^-1 Ahat D2^-1 with D1 = D2 = diag(sqrt(dhat))
    sq = np.sqrt(d)
    assert np.array_equal(b, s.b / sq)
    rows = np.repeat(np.arange(s.n), np.diff(s.row_ptr))
    assert np.array_equal(a, s.val / (sq[rows] * sq[s.col]))


@pytest.mark.parametrize("preset,gen", [("paper_noprec", lambda: W.poisson2d(20)),
                                        ("jacobi", lambda: W.convdiff3d(8, seed=1)),
                                        ("paper_ilu", lambda: W.random27(5, 4, 3, seed=65))])
def test_two_sided_scaling_solves(orc, preset, gen):
    s = gen()
    x, st = make(orc, s, preset, two_sided=1).solve()
    assert st["status"] == orc.OK and st["relres_orig"] < 1e-10
    xd = np.linalg.solve(s.dense(), s.b)
    assert np.abs(x - xd).max() <= 1e-9 * np.abs(xd).max()


def test_two_sided_equals_row_scaling_when_every_dhat_is_one(orc):
    """Row maxima equal to 2^alpha_a give Dhat = I: both scalings are then the
    identity and the two solves must agree bit for bit (x, refinements,
    residual history)."""
    s = W.poisson2d(10)
    sc = W.System("poisson_2^14", s.n, s.row_ptr, s.col, s.val * 2.0 ** 14, s.b * 2.0 ** 14)
    x1, s1 = make(orc, sc, "paper_noprec").solve()
    x2, s2 = make(orc, sc, "paper_noprec", two_sided=1).solve()
    assert np.array_equal(x1, x2) and s1["refinements"] == s2["refinements"]
    assert np.array_equal(s1["hist_relres_orig"], s2["hist_relres_orig"])
    assert np.array_equal(s1["hist_relres_scaled"], s2["hist_relres_scaled"])


def test_s_schedule_ramp(orc):
    """s(k) of eq. (AA) under the ramp reading (s_rule 1: s(k) = min(S, k - 1)).
    Pins: with S = 0 it is the constant rule bit for bit; refinement k of the
    ramp equals one refinement with the constant rule at s = min(S, k - 1)
    resumed from the ramp's previous iterate (checked for k = 1, 2, 3, so an
    off-by-one in k or in the term count fails); the first call's cycle
    trace uses A_0 alone; and the ramp solves to tolerance."""
    s = W.convdiff3d(9, 8, 7, seed=10)
    kw = dict(m=15, alpha_a=24)

    def solve(x0=None, **p):
        return orc.OracleSystem.from_system(s, orc.policy("jacobi", **kw, **p)).solve(x0)

    x0, st0 = solve(s_terms=0)
    xr0, str0 = solve(s_terms=0, s_rule=1)
    assert np.array_equal(x0, xr0) and st0["refinements"] == str0["refinements"]
    xk = None
    for k in (1, 2, 3):
        x_step, _ = solve(x0=xk, s_terms=min(2, k - 1), max_refine=1)
        x_ramp, st = solve(s_terms=2, s_rule=1, max_refine=k)
        assert st["refinements"] == k
        assert np.array_equal(x_step, x_ramp), k
        xk = x_ramp
    # the integer loop of refinement k follows s(k): k = 1 is A_0 alone
    o_ramp = orc.OracleSystem.from_system(s, orc.policy("jacobi", **kw, s_terms=2, s_rule=1))
    o_one = orc.OracleSystem.from_system(s, orc.policy("jacobi", **kw, s_terms=0))
    o_two = orc.OracleSystem.from_system(s, orc.policy("jacobi", **kw, s_terms=1))
    r, _ = o_one.residual(np.zeros(s.n))
    v1 = o_one.start_vector(r)["v1"]
    assert np.array_equal(o_ramp.cycle(v1, k=1)["V"], o_one.cycle(v1)["V"])
    assert np.array_equal(o_ramp.cycle(v1, k=2)["V"], o_two.cycle(v1)["V"])
    assert not np.array_equal(o_ramp.cycle(v1, k=2)["V"], o_one.cycle(v1)["V"])
    x, st = solve(s_terms=2, s_rule=1)
    assert st["status"] == 0 and st["relres_orig"] < 1e-10
