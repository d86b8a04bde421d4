"""GPU parity of each kernel family against the oracle, bit for bit.

Every case runs the HIP kernel through the C ABI on the same seeded input as
the oracle and compares the integer (or FP64) outputs element by element,
plus the reported overflow event code. Sizes span several SELL slices and
workgroups with a ragged tail (n not a multiple of 64 or 256)."""
import numpy as np
import pytest

from paper_2009_07495_amd import binding as B
from paper_2009_07495_amd import workloads as W

pytestmark = pytest.mark.gpu

SYSTEMS = [
    ("poisson_37x29", lambda: W.poisson2d(37, 29), "paper_noprec", {}),
    ("dd_300_ragged", lambda: W.random_dd(300, 0.05, 3), "paper_ilu", {}),
    ("cd_10x9x7", lambda: W.convdiff3d(10, 9, 7, seed=4), "jacobi", {}),
    ("r27_9x7x5", lambda: W.random27(9, 7, 5, seed=5), "paper_ilu", {}),
    ("dd_200_multiterm", lambda: W.random_dd(200, 0.04, 6), "paper_noprec", dict(s_terms=3)),
    # Jacobi with diagonals that are not the row maximum and of both signs:
    # cast diagonals that are not powers of two (general division path)
    ("dd_weakdiag_jacobi", lambda: W.random_dd(257, 0.05, 7, dominance=0.1, nonneg_diag=False), "jacobi", {}),
    # heavy-tailed row lengths (rows up to 548 entries), two terms
    ("skewed_4099_multiterm", lambda: W.skewed(4099, seed=11), "jacobi", dict(s_terms=1)),
    # one row as long as the matrix (every column) beside rows of 4 entries
    ("arrow_3000", lambda: W.arrow(3000), "jacobi", {}),
]
# row-to-lane mappings of the SpMV and the residual: SELL-64 (1), chunks split
# evenly by entries (2), then 4, 16 and 64 lanes per row over CSR (every
# mapping must give the same bits)
LANES = [1, 2, 4, 8, 16, 32, 64]


@pytest.fixture(scope="module")
def torch():
    import torch as T

    assert T.cuda.is_available(), "GPU tests need a HIP device"
    return T


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pair(orc, name, **lib_kw):
    for nm, gen, preset, kw in SYSTEMS:
        if nm == name:
            s = gen()
            return s, orc.OracleSystem.from_system(s, orc.policy(preset, **kw)), B.System.from_system(
                s, preset, **kw, **lib_kw)
    raise KeyError(name)


@pytest.mark.parametrize("name", [s[0] for s in SYSTEMS])
@pytest.mark.parametrize("lanes", LANES)
def test_spmv_bit_exact(orc, torch, name, lanes):
    s, o, g = pair(orc, name, spmv_lanes=lanes)
    assert g.stats()["spmv_lanes"] == lanes
    rng = np.random.default_rng(1)
    for trial in range(3):
        v = rng.integers(-(1 << 30), 1 << 30, s.n)
        for nt in sorted({1, o.nterms}):
            zo, ev_o = o.spmv(v, nterms=nt)
            vd = dev(torch, v)
            zd = torch.zeros(s.n, dtype=torch.int64, device="cuda")
            ev_g = g.spmv(vd, zd, nterms=nt)
            assert np.array_equal(zd.cpu().numpy(), zo), (name, nt)
            assert ev_g == ev_o


def test_spmv_overflow_code(orc, torch):
    s = W.poisson2d(20, 13)
    o = orc.OracleSystem.from_system(s, orc.policy("paper_ilu"))
    g = B.System.from_system(s, "paper_ilu")
    v = np.full(s.n, 1 << 31, dtype=np.int64)
    v[::3] = 5
    zo, ev_o = o.spmv(v)
    zd = torch.zeros(s.n, dtype=torch.int64, device="cuda")
    ev_g = g.spmv(dev(torch, v), zd)
    assert ev_o == orc.code(1, 1, 0) and ev_g == ev_o
    assert np.array_equal(zd.cpu().numpy(), zo)  # wrapped values agree too


@pytest.mark.parametrize("name", [s[0] for s in SYSTEMS])
def test_precond_bit_exact(orc, torch, name):
    s, o, g = pair(orc, name)
    rng = np.random.default_rng(2)
    z = rng.integers(-(1 << 45), 1 << 45, s.n)
    wo, ev_o = o.precond_apply(z)
    wd = torch.zeros(s.n, dtype=torch.int64, device="cuda")
    ev_g = g.precond(dev(torch, z), wd)
    assert np.array_equal(wd.cpu().numpy(), wo)
    assert ev_g == ev_o


@pytest.mark.parametrize("name", ["poisson_37x29", "cd_10x9x7"])
def test_dot_norm_axpy_normalize_bit_exact(orc, torch, name):
    s, o, g = pair(orc, name)
    p = o.pol
    rng = np.random.default_rng(3)
    for trial in range(4):
        w = rng.integers(-(1 << 33), 1 << 33, s.n) if p["b_dot"] else rng.integers(-(1 << 26), 1 << 26, s.n)
        v = rng.integers(-(1 << 30), 1 << 30, s.n)
        wd, vd = dev(torch, w), dev(torch, v)
        h_o, ovf = orc.dot(w, v, p["b_dot"])
        h_g, ev = g.dot(wd, vd)
        assert h_g == h_o and (ev != B.NO_EVENT) == ovf
        n_o, ovf = orc.norm(w, p["b_norm"])
        n_g, ev = g.norm(wd)
        assert n_g == n_o and (ev != B.NO_EVENT) == ovf
        w2_o, ovf = orc.axpy(w, v, h_o, p["b_axpy"])
        ev = g.axpy(h_o, wd, vd)
        assert np.array_equal(wd.cpu().numpy(), w2_o) and (ev != B.NO_EVENT) == ovf
        den = n_o >> p["b_div_den"]
        v2_o, ovf = orc.normalize(w2_o, den, p["b_div_num"], p["b_div_den"])
        v2d = torch.zeros(s.n, dtype=torch.int64, device="cuda")
        ev = g.normalize(wd, n_o, v2d)
        assert np.array_equal(v2d.cpu().numpy(), v2_o) and (ev != B.NO_EVENT) == ovf


def test_normalize_zero_denominator_is_breakdown(orc, torch):
    s = W.poisson2d(9, 7)
    g = B.System.from_system(s, "paper_noprec")  # the normalisation divides by asr(h, 14)
    w = dev(torch, np.ones(s.n, dtype=np.int64))
    v = torch.zeros(s.n, dtype=torch.int64, device="cuda")
    with pytest.raises(B.IgmError) as e:
        g.normalize(w, (1 << 14) - 1, v)
    assert e.value.status == B.ERR_BREAKDOWN


def test_reduction_overflow_flags(orc, torch):
    s = W.poisson2d(33, 17)
    g = B.System.from_system(s, "paper_ilu")
    w = np.full(s.n, 1 << 40, dtype=np.int64)
    v = np.full(s.n, 1 << 30, dtype=np.int64)
    h_o, ovf = orc.dot(w, v, 0)
    h_g, ev = g.dot(dev(torch, w), dev(torch, v))
    assert ovf and ev != B.NO_EVENT and h_g == h_o  # wrapped results agree


@pytest.mark.parametrize("name", [s[0] for s in SYSTEMS])
@pytest.mark.parametrize("lanes", LANES)
def test_residual_and_start_vector_bit_exact(orc, torch, name, lanes):
    s, o, g = pair(orc, name, spmv_lanes=lanes)
    rng = np.random.default_rng(4)
    for x in (np.zeros(s.n), rng.standard_normal(s.n)):
        r_o, rh_o = o.residual(x)
        r = torch.zeros(s.n, dtype=torch.float64, device="cuda")
        rh = torch.zeros_like(r)
        g.residual(dev(torch, x), r, rh)
        assert np.array_equal(r.cpu().numpy(), r_o)
        assert np.array_equal(rh.cpu().numpy(), rh_o)
        l1 = o.start_vector(r_o)
        bk, r0 = torch.zeros_like(r), torch.zeros_like(r)
        v1 = torch.zeros(s.n, dtype=torch.int64, device="cuda")
        st, gamma, rho = g.start_vector(r, bk, r0, v1)
        assert st == B.OK and gamma == l1["gamma"] and rho == l1["rho"]
        assert np.array_equal(bk.cpu().numpy(), l1["bk"])
        assert np.array_equal(r0.cpu().numpy(), l1["r0"])
        assert np.array_equal(v1.cpu().numpy(), l1["v1"])


def test_fp_norm_bit_exact(orc, torch):
    s = W.poisson2d(8)
    g = B.System.from_system(s, "paper_noprec")
    rng = np.random.default_rng(5)
    for n in (1, 2, 63, 64, 65, 1000, 4097, 100003):
        for scale in (1e-300, 1e-8, 1.0, 3e7, 1e300):
            x = rng.standard_normal(n) * scale
            x[rng.integers(0, n)] = 0.0
            assert g.fp_norm(dev(torch, x), n) == orc.dnrm(x), (n, scale)
    # more elements than one pass of the capped grid-stride launch, with the
    # largest entry first or last (the maxima land in different copies of
    # the reduction words)
    for pos in (0, -1):
        x = rng.uniform(-1.0, 1.0, 300001)
        x[pos] = -7.5
        assert g.fp_norm(dev(torch, x), x.size) == orc.dnrm(x), pos
    x = np.array([3.0, 4.0])
    assert g.fp_norm(dev(torch, x), 2) == 5.0
    assert g.fp_norm(dev(torch, np.zeros(10)), 10) == 0.0


def _diag_system(n: int, preset: str):
    """An n-row diagonal system: a cheap carrier for the vector kernels at
    sizes that need many workgroups."""
    rp = np.arange(n + 1, dtype=np.int64)
    return B.System(n, rp, np.arange(n, dtype=np.int32), np.full(n, 2.0), np.ones(n), preset)


@pytest.mark.parametrize("n", [1_048_576, 300_001])
@pytest.mark.parametrize("preset", ["paper_noprec", "paper_ilu"])
def test_dot_norm_many_workgroups(orc, torch, n, preset):
    """The standalone inner product and norm (Fig. 2; Table II) over enough
    elements that 73 to 256 workgroups each add an exact partial and the last
    one to take the completion ticket finishes the sum: in-range operands,
    products that overflow, and sums that overflow although no product does.
    Two calls in a row check that the ticket resets."""
    g = _diag_system(n, preset)
    p = g.policy()
    rng = np.random.default_rng(n + p["b_dot"])
    wr = 1 << (33 if p["b_dot"] else 21)  # no overflow in the products, the sums or the squares
    cases = [
        (rng.integers(-wr, wr, n), rng.integers(-(1 << 30), 1 << 30, n)),  # in range
        (np.full(n, 1 << 40, dtype=np.int64), np.full(n, 1 << 30, dtype=np.int64)),  # products overflow
        (np.full(n, (1 << 37) + 12345, dtype=np.int64), np.full(n, (1 << 30) - 7, dtype=np.int64)),
    ]
    w3 = rng.integers(1 << 20, 1 << 22, n)
    w3[-1] = -(1 << 45)  # the last element alone (the ragged tail) decides the sign
    cases.append((w3, rng.integers(1 << 28, 1 << 30, n)))
    for w, v in cases:
        wd, vd = dev(torch, w), dev(torch, v)
        h_o, ovf = orc.dot(w, v, p["b_dot"])
        n_o, novf = orc.norm(w, p["b_norm"])
        for _ in range(2):
            h_g, ev = g.dot(wd, vd)
            assert h_g == h_o and (ev != B.NO_EVENT) == ovf, (n, preset, h_g, h_o, ev, ovf)
            n_g, ev = g.norm(wd)
            assert n_g == n_o and (ev != B.NO_EVENT) == novf, (n, preset, n_g, n_o, ev, novf)
    g.close()


def test_spmv_full_size_every_mapping(orc, torch):
    """The standalone integer SpMV at full size (the 1M-row heavy-tailed
    matrix of the mapping benchmark, 7.7M entries, rows of 1 to 4,093
    entries) with every row-to-lane mapping equals the oracle's product bit
    for bit, with the same overflow event (none)."""
    s = W.skewed(1 << 20, seed=6)
    o = orc.OracleSystem.from_system(s, orc.policy("jacobi"))
    v = np.random.default_rng(2).integers(-(1 << 30), 1 << 30, s.n)
    zo, ev_o = o.spmv(v)
    vd = dev(torch, v)
    for lanes in LANES:
        g = B.System.from_system(s, "jacobi", spmv_lanes=lanes)
        zd = torch.zeros(s.n, dtype=torch.int64, device="cuda")
        ev_g = g.spmv(vd, zd)
        assert ev_g == ev_o and np.array_equal(zd.cpu().numpy(), zo), lanes
        g.close()
