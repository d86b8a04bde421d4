"""Seeded synthetic linear systems (CSR, FP64) used by tests, smoke and bench.

This module only builds input matrices and right-hand sides. It holds none of
the solver's arithmetic (no scaling, no fixed point, no factorisation), so both
the CPU oracle and the GPU library can be driven from it.

The paper evaluates on SuiteSparse matrices (Sec. VII-A, Table III), which are
not available here; these seeded stencil families stand in for them:

* ``poisson2d(nx, ny)``   5-point Laplacian, a_ii = 4, neighbours -1,
  Dirichlet boundaries eliminated; b = A * ones so the solution is all ones.
* ``convdiff3d(nx, ny, nz, seed)`` / ``convdiff2d(nx, ny, seed)`` 7-point /
  5-point convection-diffusion, nonsymmetric M-matrix: cell diffusivity
  10**U(-1, 1), harmonic-mean face values (boundary faces take the cell
  value), cell Peclet U(0.1, 2.0) per axis, central-difference convection
  with positive velocity; b ~ U[-1, 1].
* ``batch_systems(count, seed)`` many independent 2D/3D convection-diffusion
  systems with log-uniform sizes (batched solver workload).
* ``served_requests(count, seed)`` / ``arrival_times`` a stream of requests
  from the three families above with Poisson arrivals (served solver
  workload).
* ``random27(nx, ny, nz, seed)`` 27-point pattern, off-diagonals N(0, 1),
  diagonal 1.1 * sum |off-diagonals|; b ~ U[-1, 1].
* ``random_dd(n, density, seed)`` small unstructured diagonally dominant
  systems with ragged row lengths (edge-case coverage).

Every generator is a pure function of its arguments (numpy PCG64 seeds).
Columns within each CSR row are strictly increasing.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class System:
    """A linear system A x = b in CSR form (row_ptr int64, col int32, val f64)."""

    name: str
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    b: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        for i in range(self.n):
            lo, hi = self.row_ptr[i], self.row_ptr[i + 1]
            a[i, self.col[lo:hi]] = self.val[lo:hi]
        return a

    def matvec(self, x: np.ndarray) -> np.ndarray:
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        return np.bincount(rows, weights=self.val * x[self.col], minlength=self.n)


def _stencil_pattern(dims, offsets):
    """CSR pattern of a stencil on a box grid with natural ordering.

    ``dims`` = (nx, ny, nz); ``offsets`` = list of (dx, dy, dz). Returns
    (row_ptr, col, slot) where ``slot[e]`` is the offset index of entry e, and
    entries of each row appear in increasing column order.
    """
    nx, ny, nz = dims
    n = nx * ny * nz
    lin = [dz * nx * ny + dy * nx + dx for (dx, dy, dz) in offsets]
    order = np.argsort(lin, kind="stable")
    idx = np.arange(n, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    valid = np.zeros((n, len(offsets)), dtype=bool)
    cols = np.zeros((n, len(offsets)), dtype=np.int64)
    for k, o in enumerate(order):
        dx, dy, dz = offsets[o]
        ok = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny) & (z + dz >= 0) & (z + dz < nz)
        valid[:, k] = ok
        cols[:, k] = idx + lin[o]
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[valid].astype(np.int32)
    slot = np.broadcast_to(np.asarray(order), (n, len(offsets)))[valid]
    return row_ptr, col, slot


def poisson2d(nx: int = 64, ny: int | None = None) -> System:
    ny = nx if ny is None else ny
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0)]
    row_ptr, col, slot = _stencil_pattern((nx, ny, 1), offs)
    val = np.where(slot == 0, 4.0, -1.0)
    sysm = System(f"poisson2d_{nx}x{ny}", nx * ny, row_ptr, col, val, np.zeros(nx * ny))
    sysm.b = sysm.matvec(np.ones(sysm.n))
    return sysm


def _convdiff(dims, rng, name: str) -> System:
    """Convection-diffusion on a 2D (5-point) or 3D (7-point) box grid; the
    coefficient law of the module docstring, draws in the order cell
    diffusivity, Peclet numbers (cell, axis), right-hand side."""
    nd = len(dims)
    n = int(np.prod(dims))
    dcell = 10.0 ** rng.uniform(-1.0, 1.0, size=n)
    pe = rng.uniform(0.1, 2.0, size=(n, nd))
    b = rng.uniform(-1.0, 1.0, size=n)
    strides = [int(np.prod(dims[:a])) for a in range(nd)]
    idx = np.arange(n)
    coord = [(idx // strides[a]) % dims[a] for a in range(nd)]
    offs = [(0, 0, 0)]
    for a in range(nd):
        e = [0, 0, 0]
        e[a] = -1
        offs.append(tuple(e))
        e[a] = 1
        offs.append(tuple(e))
    box = tuple(dims) + (1,) * (3 - nd)
    row_ptr, col, slot = _stencil_pattern(box, offs)
    rows = np.repeat(idx, np.diff(row_ptr))
    # per (cell, axis): face diffusivities toward +e and -e, convection term
    dplus = np.empty((n, nd))
    dminus = np.empty((n, nd))
    for a in range(nd):
        c = coord[a]
        nb_p = np.minimum(idx + strides[a], n - 1)
        nb_m = np.maximum(idx - strides[a], 0)
        hm_p = 2.0 * dcell * dcell[nb_p] / (dcell + dcell[nb_p])
        hm_m = 2.0 * dcell * dcell[nb_m] / (dcell + dcell[nb_m])
        dplus[:, a] = np.where(c < dims[a] - 1, hm_p, dcell)
        dminus[:, a] = np.where(c > 0, hm_m, dcell)
    p = pe * np.minimum(dplus, dminus) / 2.0
    diag = (dplus + dminus).sum(axis=1)
    # slot k in offs: 0 = centre, 2a+1 = -e_a, 2a+2 = +e_a
    val = np.empty(len(col))
    for k in range(2 * nd + 1):
        m = slot == k
        r = rows[m]
        if k == 0:
            val[m] = diag[r]
        else:
            a = (k - 1) // 2
            if k % 2 == 0:  # +e neighbour
                val[m] = -dplus[r, a] + p[r, a]
            else:  # -e neighbour
                val[m] = -dminus[r, a] - p[r, a]
    return System(name, n, row_ptr, col, val, b)


def convdiff3d(nx: int = 64, ny: int | None = None, nz: int | None = None, seed: int = 2) -> System:
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return _convdiff((nx, ny, nz), np.random.default_rng(seed), f"convdiff3d_{nx}x{ny}x{nz}_s{seed}")


def convdiff2d(nx: int = 64, ny: int | None = None, seed: int = 2) -> System:
    ny = nx if ny is None else ny
    return _convdiff((nx, ny), np.random.default_rng(seed), f"convdiff2d_{nx}x{ny}_s{seed}")


def _batch_member(i: int, child, n_lo: int, n_hi: int) -> System:
    rng = np.random.default_rng(child)
    nt = int(round(float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))))
    if rng.random() < 0.5:
        nx = max(1, int(round(np.sqrt(nt))))
        ny = max(1, int(round(nt / nx)))
        return _convdiff((nx, ny), rng, f"b{i}_convdiff2d_{nx}x{ny}")
    nx = max(1, int(round(nt ** (1.0 / 3.0))))
    nz = max(1, int(round(nt / (nx * nx))))
    return _convdiff((nx, nx, nz), rng, f"b{i}_convdiff3d_{nx}x{nx}x{nz}")


def batch_systems(count: int = 512, seed: int = 4, n_lo: int = 1024, n_hi: int = 65536) -> list:
    """Independent systems for the batched solver: sizes log-uniform on
    [n_lo, n_hi], each a 2D 5-point or a 3D 7-point convection-diffusion
    system (probability 1/2 each) with the coefficient law above. System i
    draws everything from child i of SeedSequence(seed): target size, family,
    then its coefficients and right-hand side."""
    return [_batch_member(i, child, n_lo, n_hi)
            for i, child in enumerate(np.random.SeedSequence(seed).spawn(count))]


def batch_system(i: int, seed: int = 4, n_lo: int = 1024, n_hi: int = 65536) -> System:
    """System i of batch_systems(count, seed) for any count > i (children of a
    SeedSequence do not depend on how many are spawned)."""
    return _batch_member(i, np.random.SeedSequence(seed).spawn(i + 1)[i], n_lo, n_hi)


def random27(nx: int = 128, ny: int | None = None, nz: int = 64, seed: int = 3) -> System:
    ny = nx if ny is None else ny
    n = nx * ny * nz
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    row_ptr, col, slot = _stencil_pattern((nx, ny, nz), offs)
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    is_diag = col == rows
    off = rng.standard_normal(int((~is_diag).sum()))
    b = rng.uniform(-1.0, 1.0, size=n)
    val = np.empty(len(col))
    val[~is_diag] = off
    absum = np.bincount(rows[~is_diag], weights=np.abs(off), minlength=n)
    val[is_diag] = 1.1 * absum
    return System(f"random27_{nx}x{ny}x{nz}_s{seed}", n, row_ptr, col, val, b)


def random_dd(n: int, density: float = 0.1, seed: int = 0, dominance: float = 1.5,
              nonneg_diag: bool = True) -> System:
    """Unstructured sparse, strictly diagonally dominant, ragged row lengths."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    np.fill_diagonal(mask, True)
    vals = rng.standard_normal((n, n)) * mask
    np.fill_diagonal(vals, 0.0)
    d = dominance * np.abs(vals).sum(axis=1) + 0.5
    if not nonneg_diag:
        d = d * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    np.fill_diagonal(vals, d)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=row_ptr[1:])
    r, c = np.nonzero(mask)
    b = rng.uniform(-1.0, 1.0, size=n)
    return System(f"random_dd_{n}_s{seed}", n, row_ptr, c.astype(np.int32), vals[r, c].astype(np.float64), b)


def skewed(n: int, mean_len: float = 8.0, shape: float = 1.5, max_len: int = 4096, seed: int = 6) -> System:
    """Unstructured nonsymmetric sparse matrix with heavy-tailed row lengths,
    the kind that one-lane-per-row layouts pad badly: each row holds its
    diagonal and about k off-diagonal entries, k drawn from a Pareto law of the
    given shape with mean mean_len - 1, capped at min(max_len, n - 1);
    off-diagonal columns uniform over the other rows (repeats merged),
    off-diagonal values N(0, 1), diagonal 1.1 times the row's absolute sum (1
    for a row without off-diagonal entries)."""
    rng = np.random.default_rng(seed)
    cap = max(0, min(max_len, n - 1))
    scale = (mean_len - 1.0) * (shape - 1.0) / shape  # Pareto minimum giving that mean
    k = np.minimum(np.floor(scale * (1.0 + rng.pareto(shape, size=n))), cap).astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), k)
    u = rng.integers(0, max(n - 1, 1), size=len(rows), dtype=np.int64)
    cols = u + (u >= rows)  # skip the diagonal
    key = np.unique(rows * n + cols)
    rows, cols = key // n, key % n
    off = rng.standard_normal(len(rows))
    absum = np.bincount(rows, weights=np.abs(off), minlength=n)
    diag = np.where(absum > 0, 1.1 * absum, 1.0)
    r_all = np.concatenate([rows, np.arange(n, dtype=np.int64)])
    c_all = np.concatenate([cols, np.arange(n, dtype=np.int64)])
    v_all = np.concatenate([off, diag])
    order = np.lexsort((c_all, r_all))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r_all, minlength=n), out=row_ptr[1:])
    b = rng.uniform(-1.0, 1.0, size=n)
    return System(f"skewed_{n}_m{mean_len:g}_s{seed}", n, row_ptr, c_all[order].astype(np.int32), v_all[order], b)


def arrow(n: int, seed: int = 7) -> System:
    """Row 0 dense (every column), every other row its diagonal, column 0 and
    its two neighbours: one row as long as the matrix beside rows of 4 or
    fewer entries. Off-diagonal values N(0, 1), diagonal 1.1 times the row's
    absolute sum."""
    rng = np.random.default_rng(seed)
    rows, cols = [np.zeros(n, dtype=np.int64)], [np.arange(n, dtype=np.int64)]
    for d in (0, -1, 1):  # column 0 (d = 0 marks it), left and right neighbours
        r = np.arange(1, n, dtype=np.int64)
        c = np.zeros_like(r) if d == 0 else r + d
        keep = (c >= 0) & (c < n) & (c != r) & ~((d == -1) & (c == 0))
        rows.append(r[keep])
        cols.append(c[keep])
    r_all, c_all = np.concatenate(rows), np.concatenate(cols)
    r_all = np.concatenate([r_all, np.arange(1, n, dtype=np.int64)])  # diagonals of rows 1..n-1
    c_all = np.concatenate([c_all, np.arange(1, n, dtype=np.int64)])
    order = np.lexsort((c_all, r_all))
    r_all, c_all = r_all[order], c_all[order]
    v = rng.standard_normal(len(r_all))
    diag = r_all == c_all
    absum = np.bincount(r_all[~diag], weights=np.abs(v[~diag]), minlength=n)
    v[diag] = 1.1 * absum[r_all[diag]] + 1.0
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r_all, minlength=n), out=row_ptr[1:])
    b = rng.uniform(-1.0, 1.0, size=n)
    return System(f"arrow_{n}_s{seed}", n, row_ptr, c_all.astype(np.int32), v, b)


def served_requests(count: int = 20000, seed: int = 5, n_lo: int = 4096, n_hi: int = 1 << 20):
    """Request stream for the served solver, one (system, preset) at a time:
    sizes log-uniform on [n_lo, n_hi], family uniform over 2D 5-point
    convection-diffusion (jacobi), 3D 7-point convection-diffusion (jacobi)
    and the 27-point random family (paper_ilu). Request i draws everything
    from child i of SeedSequence(seed)."""
    for i, child in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(child)
        nt = int(round(float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))))
        fam = int(rng.integers(3))
        if fam == 0:
            nx = max(1, int(round(np.sqrt(nt))))
            ny = max(1, int(round(nt / nx)))
            yield _convdiff((nx, ny), rng, f"r{i}_convdiff2d_{nx}x{ny}"), "jacobi"
        else:
            nx = max(1, int(round(nt ** (1.0 / 3.0))))
            nz = max(1, int(round(nt / (nx * nx))))
            if fam == 1:
                yield _convdiff((nx, nx, nz), rng, f"r{i}_convdiff3d_{nx}x{nx}x{nz}"), "jacobi"
            else:
                yield random27(nx, nx, nz, seed=int(rng.integers(1 << 31))), "paper_ilu"


def arrival_times(count: int, rate_per_s: float = 2000.0, seed: int = 5) -> np.ndarray:
    """Poisson arrivals: cumulative sums of exponential gaps (seconds)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(count + 1)[count])
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def from_dense(a: np.ndarray, b: np.ndarray, name: str = "dense") -> System:
    n = a.shape[0]
    mask = a != 0.0
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=row_ptr[1:])
    r, c = np.nonzero(mask)
    return System(name, n, row_ptr, c.astype(np.int32), a[r, c].astype(np.float64), np.asarray(b, dtype=np.float64))


# Named workloads: (generator, preset name, restart length m).
WORKLOADS = {
    "poisson2d_64": (lambda: poisson2d(64), "paper_noprec", 30),
    "convdiff3d_64": (lambda: convdiff3d(64, seed=2), "jacobi", 50),
    "random27_1m": (lambda: random27(128, 128, 64, seed=3), "paper_ilu", 30),
    # heavy-tailed row lengths (the SpMV row-to-lane mappings' benchmark matrix)
    "skewed_1m": (lambda: skewed(1 << 20, seed=6), "jacobi", 30),
}
