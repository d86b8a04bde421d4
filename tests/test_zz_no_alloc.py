"""The allocation-free inner product and norm (igm_reduce_noalloc, for
callers that cannot allocate device memory) against the existing entry
points igm_dot / igm_norm and the oracle, through the C ABI: two calls in a
row, the second on a smaller input, for both modes, with and without
overflow, on caller-provided device buffers and the caller's stream."""
import numpy as np
import pytest

from paper_2009_07495_amd import binding as B

pytestmark = pytest.mark.gpu


def _diag_system(n: int, preset: str):
    rp = np.arange(n + 1, dtype=np.int64)
    return B.System(n, rp, np.arange(n, dtype=np.int32), np.full(n, 2.0), np.ones(n), preset)


@pytest.mark.parametrize("preset", ["paper_noprec", "paper_ilu"])
def test_noalloc_reduction_equals_igm_dot_and_norm(orc, preset):
    import torch

    assert torch.cuda.is_available()
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(17)
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    for n, big in ((1_048_576 + 37, False), (300_001, True), (4097, False), (1, False)):
        g = _diag_system(n, preset)
        p = g.policy()
        wr = 1 << (33 if p["b_dot"] else 21)
        if big:  # products or sums out of int64
            w = np.full(n, (1 << 37) + 5, dtype=np.int64)
            v = np.full(n, (1 << 30) - 3, dtype=np.int64)
        else:
            w = rng.integers(-wr, wr, n)
            v = rng.integers(-(1 << 30), 1 << 30, n)
        wd = torch.from_numpy(w).cuda()
        vd = torch.from_numpy(v).cuda()
        for mode, b, ref, oref in ((0, p["b_dot"], g.dot(wd, vd), orc.dot(w, v, p["b_dot"])),
                                   (1, p["b_norm"], g.norm(wd), orc.norm(w, p["b_norm"]))):
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                st = B.igm_reduce_noalloc(mode, n, wd, vd, b, p["df"], out, stream)
            assert st == B.OK
            stream.synchronize()
            h, ev = out.cpu().tolist()
            assert (h, ev) == tuple(ref), (n, mode, h, ev, ref)
            assert h == oref[0] and (ev != B.NO_EVENT) == oref[1]
        g.close()


def test_noalloc_rejects_bad_arguments():
    import torch

    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    w = torch.zeros(8, dtype=torch.int64, device="cuda")
    assert B.igm_reduce_noalloc(2, 8, w, w, 0, 30, out) == B.ERR_ARG
    assert B.igm_reduce_noalloc(0, 0, w, w, 0, 30, out) == B.ERR_ARG
    assert B.igm_reduce_noalloc(0, (1 << 48) + 1, w, w, 0, 30, out) == B.ERR_ARG
    assert B.igm_reduce_noalloc(0, 8, w, None, 0, 30, out) == B.ERR_ARG
    assert B.igm_reduce_noalloc(1, 8, w, None, 31, 30, out) == B.ERR_ARG
    assert B.igm_reduce_noalloc(1, 8, w, None, 0, 30, None) == B.ERR_ARG
