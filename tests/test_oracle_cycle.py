"""Pins for the oracle's integer kernels and one int-GMRES(m) call (Fig. 2).

The paper prints no intermediate values, so the exact bits of a cycle are
"parity unpinned"; these tests pin them through properties a dropped term, a
wrong sign, a wrong index or a swapped operand would break:
  * SpMV = exact integer matrix-vector product (eq. (matvec));
  * integer sweeps satisfy the truncated-division residual property;
  * after the rotations H is upper triangular, |g| is non-increasing (Sec.
    V-D.3, rotation of g), c^2 + s^2 = 1, the basis is normalised with its
    upper bits zero (Sec. V-D.2, inner product);
  * the GMRES residual identity rho |g_{j+1}| = ||Mbar^-1 (b - Abar x_j)||;
  * each rotated column matches one FP64 MGS step on the oracle's own basis;
  * A = c I breaks down at j = 1.
"""
import numpy as np
import pytest

from paper_2009_07495_amd import workloads as W

TWO30 = float(1 << 30)


def make(orc, sysm, preset, **kw):
    return orc.OracleSystem.from_system(sysm, orc.policy(preset, **kw))


def int_dense(sysm, vals):
    a = np.zeros((sysm.n, sysm.n), dtype=object)
    a[:] = 0
    for i in range(sysm.n):
        for e in range(sysm.row_ptr[i], sysm.row_ptr[i + 1]):
            a[i, sysm.col[e]] = int(vals[e])
    return a


def test_spmv_is_exact_integer_product(orc):
    s = W.random_dd(37, 0.2, 21)
    o = make(orc, s, "paper_noprec", s_terms=3)
    ab, al = o.terms()
    rng = np.random.default_rng(1)
    v = rng.integers(-(1 << 30), 1 << 30, s.n)
    vo = np.array([int(t) for t in v], dtype=object)
    z0, first = o.spmv(v, nterms=1)
    assert first == orc.NO_EVENT
    ref0 = int_dense(s, ab[0]).dot(vo)
    assert [int(t) for t in z0] == list(ref0)
    nt = ab.shape[0]
    assert nt >= 2
    z, first = o.spmv(v, nterms=nt)
    ref = ref0.copy()
    for l in range(1, nt):
        ref = ref + int_dense(s, ab[l]).dot(vo) // (1 << int(al[l]))  # floor shift of each term
    assert [int(t) for t in z] == list(ref)


def test_spmv_overflow_flag(orc):
    s = W.poisson2d(8)
    o = make(orc, s, "paper_ilu")  # entries up to 2^32
    v = np.full(s.n, 1 << 31, dtype=np.int64)
    z, first = o.spmv(v, j=7)
    assert first == orc.code(7, 1, 0)  # 2^32 * 2^31 = 2^63 leaves int64
    v = np.full(s.n, 1 << 29, dtype=np.int64)
    assert o.spmv(v)[1] == orc.NO_EVENT


@pytest.mark.parametrize("preset", ["paper_ilu", "jacobi"])
def test_precond_truncated_substitution(orc, preset):
    s = W.random27(5, 4, 4, seed=22) if preset == "paper_ilu" else W.convdiff3d(6, seed=22)
    o = make(orc, s, preset)
    fac, ld, ud = o.precond()
    rng = np.random.default_rng(2)
    z = rng.integers(-(1 << 40), 1 << 40, s.n)
    w, first = o.precond_apply(z)
    assert first == orc.NO_EVENT
    if preset == "jacobi":
        t = [int(np.trunc(a / b)) for a, b in zip(z, ld)]  # |z| < 2^53: exact in double
        t = [int(a / int(b)) if abs(a) < 2 ** 50 else None for a, b in zip(t, ud)]
        assert [int(x) for x in w] == t
        return
    n = s.n
    # forward: y_i = tdiv(z_i - sum_{j<i} L_ij y_j, L_ii); then backward on u
    # property: |num_i - L_ii y_i| < |L_ii| with the sign of num_i (truncation)
    rows = np.repeat(np.arange(n), np.diff(s.row_ptr))
    Lo = {(int(r), int(c)): int(f) for r, c, f in zip(rows, s.col, fac) if c < r}
    Uo = {(int(r), int(c)): int(f) for r, c, f in zip(rows, s.col, fac) if c > r}
    u = [int(t) for t in w]
    # reconstruct y from u: y_i = Ubar_ii u_i + sum_{j>i} U_ij u_j + rem, |rem| < |U_ii|
    y = [None] * n
    for i in range(n):
        num = sum(f * u[c] for (r, c), f in Uo.items() if r == i)
        acc = int(ud[i]) * u[i]
        y[i] = (acc, num)
    # run the forward sweep independently in exact integers and check both
    ye = [0] * n
    for i in range(n):
        num = int(z[i]) - sum(f * ye[c] for (r, c), f in Lo.items() if r == i)
        q = abs(num) // int(ld[i])
        ye[i] = q if num >= 0 else -q
        rem = num - int(ld[i]) * ye[i]
        assert abs(rem) < int(ld[i]) and (rem == 0 or (rem > 0) == (num > 0))
    for i in range(n):
        acc, num = y[i]
        rem = (ye[i] - num) - acc
        assert abs(rem) < abs(int(ud[i])) and (rem == 0 or (rem > 0) == ((ye[i] - num) > 0))


def residual_sequence(tr):
    """|g_{j+1}| right after step j (rotation of g), before step j+1 rotates it:
    G_0 = 2^df, G_{j+1} = floor(-s_j G_j / 2^df); also checks that the stored
    g_j equals floor(c_j G_j / 2^df)."""
    G = [1 << 30]
    for j in range(tr["jstar"]):
        gj = G[-1]
        assert int(tr["g"][j]) == (int(tr["c"][j]) * gj) // (1 << 30)
        G.append((-int(tr["s"][j]) * gj) // (1 << 30))
    assert int(tr["g"][tr["jstar"]]) == G[-1]
    return G


def run_cycle(orc, sysm, preset, m, **kw):
    o = make(orc, sysm, preset, m=m, **kw)
    r, _ = o.residual(np.zeros(sysm.n))
    l1 = o.start_vector(r)
    assert l1["status"] == orc.OK
    tr = o.cycle(l1["v1"])
    return o, l1, tr


CASES = [
    ("poisson", lambda: W.poisson2d(16), "paper_noprec", 20),
    ("ilu", lambda: W.random27(6, 6, 5, seed=23), "paper_ilu", 20),
    ("jacobi", lambda: W.convdiff3d(8, seed=23), "jacobi", 25),
    ("dd", lambda: W.random_dd(64, 0.1, 24), "paper_ilu", 30),
]


@pytest.mark.parametrize("name,gen,preset,m", CASES)
def test_cycle_invariants(orc, name, gen, preset, m):
    s = gen()
    o, l1, tr = run_cycle(orc, s, preset, m)
    assert tr["first_ovf"] == orc.NO_EVENT
    js = tr["jstar"]
    H, g, c, sn, V = tr["H"], tr["g"], tr["c"], tr["s"], tr["V"]
    pol = o.pol
    G = residual_sequence(tr)
    for j in range(js):
        assert H[j + 1, j] == 0  # set to zero after the new rotation
        assert np.all(H[j + 2:, j] == 0)  # upper triangular after the rotations
        assert H[j, j] > 0
        cs = float(c[j]) ** 2 + float(sn[j]) ** 2
        # rotation is orthonormal up to the truncation of t (rotation radius) and
        # of the shifted denominator (new rotation), both relative to t
        tol_cs = 4.0 * ((1 << pol["b_cs_den"]) + (1 << pol["b_tmp"])) / float(H[j, j]) + 2.0 ** -26
        assert abs(cs / 2.0 ** 60 - 1.0) < tol_cs
        assert abs(G[j + 1]) <= abs(G[j]) * (1 + 2.0 ** -12) + 2  # residual non-increasing
    for i in range(js + (tr["breakdown"] == 0)):
        v = V[i].astype(float)
        assert np.abs(V[i]).max() < (1 << 31)  # upper bits zero (Sec. V-D.2)
        assert abs(np.linalg.norm(v) / TWO30 - 1.0) < (2e-3 if preset == "paper_noprec" else 1e-6)


def dense_mbar_inv(o, sysm):
    fac, ld, ud = o.precond()
    n = sysm.n
    if o.pol["precond"] == 0:
        return np.eye(n)
    L, U = np.diag(ld.astype(float)), np.diag(ud.astype(float))
    if o.pol["precond"] == 2:
        for i in range(n):
            for e in range(sysm.row_ptr[i], sysm.row_ptr[i + 1]):
                j = sysm.col[e]
                if j < i:
                    L[i, j] = fac[e]
                elif j > i:
                    U[i, j] = fac[e]
    return np.linalg.inv(L @ U)


@pytest.mark.parametrize("name,gen,preset,m", CASES)
def test_gmres_residual_identity(orc, name, gen, preset, m):
    """rho |g_{j+1}| 2^-df equals the preconditioned residual norm of the
    iterate built from the first j columns (closing least-squares step), up to the fixed-point
    rounding of the basis."""
    s = gen()
    o, l1, tr = run_cycle(orc, s, preset, m)
    ab, _ = o.terms()
    Ab = s.__class__("a", s.n, s.row_ptr, s.col, ab[0].astype(float), s.b).dense()
    Minv = dense_mbar_inv(o, s)
    rho, bk = l1["rho"], l1["bk"]
    rtol = 2e-2 if preset == "paper_noprec" else 1e-5
    G = residual_sequence(tr)
    for j in sorted({1, 2, 5, tr["jstar"] // 2, tr["jstar"]}):
        if j < 1:
            continue
        t = tr["_t"]
        saved = t.jstar
        t.jstar = j
        x = o.cycle_update(tr, rho)
        t.jstar = saved
        res = np.linalg.norm(Minv @ (bk - Ab @ x))
        pred = rho * abs(float(G[j])) / TWO30
        assert abs(res - pred) <= rtol * max(pred, 1e-30) + 1e-6 * rho, (j, res, pred)


@pytest.mark.parametrize("name,gen,preset,m", CASES)
def test_columns_match_fp64_mgs_step(orc, name, gen, preset, m):
    """Column by column: take the oracle's own basis v_1..v_j (exact Q30
    integers), do one FP64 Arnoldi/MGS step for column j, apply the oracle's
    rotations c_i, s_i (i < j) in FP64, and compare with the stored rotated
    column, t = H_jj and (c_j, s_j) = (h_jj, h_j+1,j) / t. A wrong index, a
    dropped term or a sign error in the Arnoldi step or its rotations breaks this at the first column
    where it acts; fixed-point rounding only costs ~2^-30 (or 2^-14 with the
    16-bit shifts)."""
    s = gen()
    o, l1, tr = run_cycle(orc, s, preset, m)
    ab, _ = o.terms()
    Ab = s.__class__("a", s.n, s.row_ptr, s.col, ab[0].astype(float), s.b).dense()
    op = dense_mbar_inv(o, s) @ Ab
    V = tr["V"] / TWO30
    c, sn = tr["c"] / TWO30, tr["s"] / TWO30
    scale = np.abs(tr["H"]).max() / TWO30
    tol = (2e-4 if preset == "paper_noprec" else 1e-7) * scale
    for j in range(tr["jstar"]):
        w = op @ V[j]
        h = np.zeros(j + 2)
        for i in range(j + 1):
            h[i] = w @ V[i]
            w = w - h[i] * V[i]
        h[j + 1] = np.linalg.norm(w)
        for i in range(j):
            a, b = h[i], h[i + 1]
            h[i], h[i + 1] = c[i] * a + sn[i] * b, -sn[i] * a + c[i] * b
        t = np.hypot(h[j], h[j + 1])
        col = tr["H"][: j + 1, j] / TWO30
        np.testing.assert_allclose(col[:j], h[:j], rtol=0, atol=tol, err_msg=f"column {j}")
        assert abs(col[j] - t) <= tol, (j, col[j], t)
        ctol = (2e-4 if preset == "paper_noprec" else 1e-7) * scale / t + 2.0 ** -28
        assert abs(c[j] - h[j] / t) <= ctol and abs(sn[j] - h[j + 1] / t) <= ctol, j


def test_scalar_matrix_breaks_down_at_step_one(orc):
    """A = 3 I, b = -2 e_5 with the Jacobi preset: v1 = 2^30 e_5 exactly, the
    Gram-Schmidt update leaves w = 0, so the normalisation meets a zero
    denominator at j = 1 and the single column gives the exact solution
    x = b / 3."""
    n = 20
    b = np.zeros(n)
    b[5] = -2.0
    s = W.from_dense(3.0 * np.eye(n), b)
    o, l1, tr = run_cycle(orc, s, "jacobi", 10)
    assert np.array_equal(l1["v1"], np.where(np.arange(n) == 5, -(1 << 30), 0))
    assert tr["breakdown"] == 1 and tr["jstar"] == 1 and tr["steps"] == 1
    assert tr["H"][0, 0] == 1 << 30 and tr["c"][0] == 1 << 30 and tr["s"][0] == 0
    x, st = o.solve()
    assert st["status"] == orc.OK and st["refinements"] == 1
    assert np.array_equal(x, b / 3.0)


def test_singular_direction_gives_no_column(orc):
    """A v1 = 0: the norm and the rotation radius both give 0, the new
    rotation has a zero denominator and no column is usable; the refinement
    driver reports the breakdown."""
    a = np.array([[1.0, 1.0], [1.0, 1.0]])
    s = W.from_dense(a, np.array([1.0, -1.0]))
    o, l1, tr = run_cycle(orc, s, "paper_noprec", 5)
    assert tr["breakdown"] == 2 and tr["jstar"] == 0 and tr["steps"] == 1
    x, st = o.solve()
    assert st["status"] == orc.ERR_BREAKDOWN and np.all(x == 0)
    # ILU(0) of the same singular matrix has a zero pivot
    with pytest.raises(orc.OracleError) as e:
        make(orc, s, "paper_ilu")
    assert e.value.status == orc.ERR_ZERO_PIVOT
