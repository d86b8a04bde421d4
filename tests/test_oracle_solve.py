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


def test_multiterm_matrix_solve(orc):
    """s = 2 correction matrices (eq. (AA)) with a coarse alpha_a still solves."""
    s = W.convdiff3d(6, seed=9)
    o = make(orc, s, "jacobi", alpha_a=24, s_terms=2, m=20)
    assert o.nterms == 3
    x, st = o.solve()
    assert st["status"] == orc.OK and true_relres(s, x) < 1e-10


def test_overflow_is_reported_with_its_position(orc):
    """The no-preconditioner shifts (beta = 16) with alpha_a = 40 overflow the
    line 11 numerator shift (|w| 2^(30+16) >= 2^63) in the first step."""
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
