"""Pins for the oracle's setup: initial scaling (Sec. III), integer matrices
A_0..A_p (Sec. IV-B) and the integer ILU(0)/Jacobi factors (Sec. VI-A)."""
from fractions import Fraction

import numpy as np
import pytest

from paper_2009_07495_amd import workloads as W


def make(orc, sysm, preset="paper_noprec", **kw):
    return orc.OracleSystem.from_system(sysm, orc.policy(preset, **kw))


def test_scaling_row_max_is_two_to_alpha(orc):
    for sysm, preset in ((W.random_dd(40, 0.2, 1), "paper_noprec"), (W.convdiff3d(6, seed=7), "jacobi"),
                         (W.random27(5, 4, 3, seed=1), "paper_ilu")):
        o = make(orc, sysm, preset)
        d, a, b = o.scaled()
        alpha = orc.PRESETS[preset]["alpha_a"]
        for i in range(sysm.n):
            lo, hi = sysm.row_ptr[i], sysm.row_ptr[i + 1]
            assert np.abs(a[lo:hi]).max() == 2.0 ** alpha  # eq. (eq3): exact
            mu = np.abs(sysm.val[lo:hi]).max()
            assert d[i] == mu / 2.0 ** alpha
        # A = Dhat^-1 Ahat up to one rounding per entry
        rows = np.repeat(np.arange(sysm.n), np.diff(sysm.row_ptr))
        np.testing.assert_allclose(a * d[rows], sysm.val, rtol=2.0 ** -52, atol=0)
        np.testing.assert_allclose(b * d, sysm.b, rtol=2.0 ** -52, atol=0)


def test_poisson_integer_matrix_closed_form(orc):
    """4 / (4 * 2^-16) = 2^16 on the diagonal, -1 / (4 * 2^-16) = -2^14 off it."""
    s = W.poisson2d(16)
    o = make(orc, s, "paper_noprec")
    ab, al = o.terms()
    rows = np.repeat(np.arange(s.n), np.diff(s.row_ptr))
    diag = s.col == rows
    assert np.all(ab[0][diag] == 65536) and np.all(ab[0][~diag] == -16384)
    assert ab.shape[0] == 1 and al[0] == 0


def test_jacobi_factors_closed_form(orc):
    """Diagonal = row max = 2^32 after scaling, so Lbar_ii = Ubar_ii = 2^16."""
    s = W.convdiff3d(8, seed=3)
    o = make(orc, s, "jacobi")
    fac, ld, ud = o.precond()
    assert np.all(ld == 65536) and np.all(ud == 65536) and np.all(fac == 0)


@pytest.mark.parametrize("alpha_a", [8, 16, 32])
def test_multiterm_decomposition_reconstructs_A(orc, alpha_a):
    """eq. (A): A = A_0 + sum_l 2^-alpha_l A_l exactly once enough terms are kept;
    alpha_l strictly increasing; max|A_l| in [2^alpha_a, 2^(alpha_a+1))."""
    s = W.random_dd(30, 0.3, 11)
    o = make(orc, s, "paper_noprec", alpha_a=alpha_a, s_terms=8)
    _, a, _ = o.scaled()
    ab, al = o.terms()
    assert ab.shape[0] >= 2
    assert all(al[l] < al[l + 1] for l in range(1, len(al) - 1))
    for l in range(1, ab.shape[0]):
        mx = int(np.abs(ab[l]).max())
        assert (1 << alpha_a) <= mx < (1 << (alpha_a + 1)), (l, mx)
    for e in range(len(a)):
        tot = Fraction(int(ab[0][e])) + sum(Fraction(int(ab[l][e]), 1 << int(al[l])) for l in range(1, ab.shape[0]))
        assert tot == Fraction(float(a[e])), e
    # truncating the series loses at most 2^-alpha_s per entry (relative to units of A_0)
    o2 = make(orc, s, "paper_noprec", alpha_a=alpha_a, s_terms=1)
    ab2, al2 = o2.terms()
    for e in range(len(a)):
        approx = Fraction(int(ab2[0][e])) + Fraction(int(ab2[1][e]), 1 << int(al2[1]))
        assert abs(Fraction(float(a[e])) - approx) < Fraction(1, 1 << int(al2[1]))


def _lu_dense(orc, sysm, preset):
    o = make(orc, sysm, preset)
    lu = o.ilu_fp()
    n = sysm.n
    L, U = np.eye(n), np.zeros((n, n))
    for i in range(n):
        for e in range(sysm.row_ptr[i], sysm.row_ptr[i + 1]):
            j = sysm.col[e]
            if j < i:
                L[i, j] = lu[e]
            else:
                U[i, j] = lu[e]
    return o, L, U


def test_ilu0_full_pattern_is_dense_lu(orc):
    """ILU(0) on a full pattern is the LU factorisation without pivoting."""
    rng = np.random.default_rng(12)
    n = 24
    a = rng.standard_normal((n, n))
    a += np.diag(np.abs(a).sum(axis=1) + 1.0)
    s = W.from_dense(a, rng.standard_normal(n))
    o, L, U = _lu_dense(orc, s, "paper_ilu")
    _, A, _ = o.scaled()
    Ad = W.from_dense(a, s.b)
    Ad.val = A
    np.testing.assert_allclose(L @ U, Ad.dense(), rtol=1e-12, atol=1e-12 * np.abs(A).max())
    assert np.allclose(np.diag(L), 1.0)


def test_ilu0_tridiagonal_is_thomas(orc):
    """No fill on a tridiagonal pattern: ILU(0) = exact LU (Thomas recurrences)."""
    rng = np.random.default_rng(13)
    n = 50
    dmain = rng.uniform(3, 5, n)
    lo, up = rng.uniform(-1, 1, n - 1), rng.uniform(-1, 1, n - 1)
    a = np.diag(dmain) + np.diag(lo, -1) + np.diag(up, 1)
    s = W.from_dense(a, np.ones(n))
    o, L, U = _lu_dense(orc, s, "paper_ilu")
    d_, A, _ = o.scaled()
    Ad = s.dense() / d_[:, None]
    # Thomas: c'_i pivot recurrence on the scaled matrix
    piv = np.empty(n)
    piv[0] = Ad[0, 0]
    for i in range(1, n):
        piv[i] = Ad[i, i] - Ad[i, i - 1] / piv[i - 1] * Ad[i - 1, i]
    np.testing.assert_allclose(np.diag(U), piv, rtol=1e-13)
    np.testing.assert_allclose(L @ U, Ad, rtol=1e-12, atol=1e-9)


def test_ilu0_matches_A_on_pattern(orc):
    """Defining property of ILU(0): (L U)_ij = a_ij for every (i, j) in the pattern."""
    s = W.random27(6, 5, 4, seed=5)
    o, L, U = _lu_dense(orc, s, "paper_ilu")
    _, A, _ = o.scaled()
    LU = L @ U
    rows = np.repeat(np.arange(s.n), np.diff(s.row_ptr))
    np.testing.assert_allclose(LU[rows, s.col], A, rtol=1e-12, atol=1e-12 * np.abs(A).max())


def test_integer_factors_properties(orc):
    """Eqs. (dl)-(ilu2): Lbar_ii > 0, sgn(Ubar_ii) = sgn(d_i), Lbar Ubar ~ A."""
    s = W.random_dd(40, 0.25, 14, nonneg_diag=False)
    o, L, U = _lu_dense(orc, s, "paper_ilu")
    fac, ld, ud = o.precond()
    d = np.diag(U)
    assert np.all(ld > 0)
    assert np.all(np.sign(ud) == np.sign(d))
    assert np.all(np.abs(ld - np.sqrt(np.abs(d))) < 1) and np.all(np.abs(ud - np.sign(d) * np.sqrt(np.abs(d))) < 1)
    n = s.n
    Lb, Ub = np.diag(ld.astype(float)), np.diag(ud.astype(float))
    for i in range(n):
        for e in range(s.row_ptr[i], s.row_ptr[i + 1]):
            j = s.col[e]
            if j < i:
                Lb[i, j] = fac[e]
            elif j > i:
                Ub[i, j] = fac[e]
    np.testing.assert_allclose(Lb @ Ub, L @ U, rtol=0, atol=2.0 ** -13 * np.abs(L @ U).max())


def test_setup_errors(orc):
    s = W.random_dd(10, 0.3, 15)
    # all-zero row: dhat undefined
    val = s.val.copy()
    val[s.row_ptr[3]:s.row_ptr[4]] = 0.0
    with pytest.raises(orc.OracleError) as e:
        orc.OracleSystem(s.n, s.row_ptr, s.col, val, s.b, orc.policy("paper_noprec"))
    assert e.value.status == orc.ERR_SINGULAR_ROW
    # NaN input
    val = s.val.copy()
    val[0] = np.nan
    with pytest.raises(orc.OracleError) as e:
        orc.OracleSystem(s.n, s.row_ptr, s.col, val, s.b, orc.policy("paper_noprec"))
    assert e.value.status == orc.ERR_ARG
    # unsorted columns
    col = s.col.copy()
    col[s.row_ptr[2]], col[s.row_ptr[2] + 1] = col[s.row_ptr[2] + 1], col[s.row_ptr[2]]
    with pytest.raises(orc.OracleError) as e:
        orc.OracleSystem(s.n, s.row_ptr, col, s.val, s.b, orc.policy("paper_noprec"))
    assert e.value.status == orc.ERR_ARG
    # zero pivot in ILU(0): structurally zero diagonal
    a = np.array([[0.0, 1.0], [1.0, 1.0]])
    z = W.from_dense(a, np.ones(2))
    with pytest.raises(orc.OracleError) as e:
        orc.OracleSystem.from_system(z, orc.policy("paper_ilu"))
    assert e.value.status == orc.ERR_ZERO_PIVOT
    # a bad policy
    with pytest.raises(orc.OracleError) as e:
        orc.OracleSystem.from_system(s, orc.policy("paper_noprec", df=70))
    assert e.value.status == orc.ERR_ARG


def test_presets_match_paper_tables(orc):
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "shift_presets.txt")
    n = 0
    for line in open(path):
        line = line.split("#")[0].split()
        if not line:
            continue
        preset, key, val = line
        assert orc.PRESETS[preset][key] == int(val), (preset, key)
        n += 1
    assert n == 24


# ---- Gauss-Seidel splitting (a reading: the paper reports a Gauss-Seidel
# preconditioner, Sec. VII-D, without its construction; see orc_setup.c) ----

def test_gauss_seidel_factors_reproduce_the_splitting(orc):
    """Lbar Ubar approximates M = D + L_A (diagonal and strict lower part of
    the scaled A) within the truncation of the two casts, with nothing above
    the diagonal; Ubar is diagonal."""
    s = W.convdiff2d(9, 7, seed=5)
    o = orc.OracleSystem.from_system(s, orc.policy("paper_ilu", gauss_seidel=1))
    fac, ld, ud = o.precond()
    _, a, _ = o.scaled()
    n = s.n
    rows = np.repeat(np.arange(n), np.diff(s.row_ptr))
    upper = s.col > rows
    assert np.all(fac[upper] == 0)
    L = np.zeros((n, n))
    L[rows[~upper & (s.col != rows)], s.col[~upper & (s.col != rows)]] = fac[~upper & (s.col != rows)]
    L[np.arange(n), np.arange(n)] = ld
    M = L @ np.diag(ud.astype(float))
    Aful = np.zeros((n, n))
    Aful[rows, s.col] = a
    target = np.tril(Aful)
    # each factor entry is truncated once (error < 1) and Ubar is diagonal
    bound = np.abs(L) + np.abs(ud)[None, :] + 1.0
    assert np.all(np.abs(M - target) <= bound)


def test_gauss_seidel_equals_ilu0_on_a_lower_triangular_matrix(orc):
    """ILU(0) of a lower-triangular matrix eliminates nothing and has U = I,
    which is the Gauss-Seidel splitting: both must give the same solve bit for
    bit. On a general matrix they differ."""
    rng = np.random.default_rng(3)
    n = 40
    A = np.tril(rng.normal(size=(n, n)) * (rng.random((n, n)) < 0.2), -1)
    A += np.diag(np.abs(A).sum(1) * 1.1 + 1.0)
    s = W.from_dense(A, rng.uniform(-1, 1, n))
    x1, s1 = orc.OracleSystem.from_system(s, orc.policy("paper_ilu")).solve()
    x2, s2 = orc.OracleSystem.from_system(s, orc.policy("paper_ilu", gauss_seidel=1)).solve()
    assert s1["status"] == s2["status"] == orc.OK and np.array_equal(x1, x2)
    g = W.convdiff2d(12, 10, seed=6)
    f1 = orc.OracleSystem.from_system(g, orc.policy("paper_ilu")).precond()[0]
    f2 = orc.OracleSystem.from_system(g, orc.policy("paper_ilu", gauss_seidel=1)).precond()[0]
    assert not np.array_equal(f1, f2)


@pytest.mark.parametrize("gen", [lambda: W.convdiff2d(30, 20, seed=3), lambda: W.random27(5, 4, 3, seed=65)])
def test_gauss_seidel_solves(orc, gen):
    s = gen()
    x, st = orc.OracleSystem.from_system(s, orc.policy("paper_ilu", gauss_seidel=1)).solve()
    assert st["status"] == orc.OK and st["relres_orig"] < 1e-10
    xd = np.linalg.solve(s.dense(), s.b)
    assert np.abs(x - xd).max() <= 1e-9 * np.abs(xd).max()
    with pytest.raises(orc.OracleError):  # only as a variant of the ILU(0) preconditioner
        orc.OracleSystem.from_system(s, orc.policy("jacobi", gauss_seidel=1))
