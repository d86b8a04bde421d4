"""CPU model of the merge-based partition of the SpMV chunk (the search and
walk of spmv_chunk_merge, written out in Python): for chunks of 256, 512 and
1024 row slots with empty rows, heavy-tailed lengths, one row longer than the
whole chunk's share, and padded chunks, every entry is consumed exactly once,
by the thread walking its row, every partial lands on the right row, no
thread holds a partial past the last row, and every loaded entry index is in
bounds. (The model mirrors the device code; the GPU parity tests check the
kernel's results against the oracle.)"""
import numpy as np
import pytest

BATCH = 4  # entries loaded and multiplied together (kMergeBatch)


def walk_chunk(lens, block):
    nrows = len(lens)
    rp = np.zeros(block + 1, dtype=np.int64)
    rp[1:nrows + 1] = np.cumsum(lens)
    e = int(rp[nrows])
    rp[nrows + 1:] = e  # padded row slots: empty
    total = block + e
    per = (total + block - 1) // block
    row_sum = np.zeros(block, dtype=np.int64)
    seen = np.zeros(e, dtype=np.int64)
    for t in range(block):
        d0, d1 = min(t * per, total), min(t * per + per, total)
        lo, hi = max(0, d0 - e), min(d0, block)
        while lo < hi:  # merge-path search: row end i precedes entry j iff rp[i + 1] <= j
            mid = (lo + hi) >> 1
            if rp[mid + 1] <= d0 - mid - 1:
                lo = mid + 1
            else:
                hi = mid
        i, j, d, acc = lo, d0 - lo, d0, 0
        while d < d1:
            loaded = [j + u for u in range(BATCH) if j + u < e]
            u = 0
            while d < d1 and u < BATCH:
                if i < block and rp[i + 1] <= j:
                    row_sum[i] += acc
                    acc, i = 0, i + 1
                else:
                    assert j in loaded
                    seen[j] += 1
                    acc += j + 1
                    j, u = j + 1, u + 1
                d += 1
        if i < block:
            row_sum[i] += acc
        else:
            assert acc == 0
    want = np.array([sum(range(rp[r] + 1, rp[r + 1] + 1)) for r in range(block)], dtype=np.int64)
    return seen, row_sum, want


def chunks():
    rng = np.random.default_rng(0)
    for block in (256, 512, 1024):
        for trial in range(15):
            nrows = block if trial % 3 == 0 else int(rng.integers(0, block + 1))
            kind = trial % 5
            if kind == 0:
                lens = rng.integers(0, 3, nrows)
            elif kind == 1:
                lens = np.minimum((3 * (1 + rng.pareto(1.5, nrows))).astype(int), 4096)
            elif kind == 2:
                lens = np.zeros(nrows, dtype=int)
            elif kind == 3:
                lens = np.full(nrows, 27)
            else:
                lens = np.zeros(nrows, dtype=int)
                if nrows:
                    lens[rng.integers(nrows)] = 5000
            yield block, list(lens)
    yield 256, []
    yield 256, [10000]
    yield 256, [1] * 255 + [3000]


@pytest.mark.parametrize("block,lens", list(chunks()))
def test_every_entry_once_on_its_row(block, lens):
    seen, row_sum, want = walk_chunk(lens, block)
    assert np.all(seen == 1)
    assert np.array_equal(row_sum, want)
