"""ctypes binding of the igmres C ABI (include/igmres.h).

Argument marshalling only: every step of the solver runs inside
``libigmres.so`` (HIP kernels for gfx950). The functions keep the C names;
``System`` is a small convenience wrapper around one ``igm_system``. Device
buffers are passed as integers or as objects with ``data_ptr()`` (for example
torch CUDA tensors); PyTorch is never imported here.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libigmres.so")

OK, NOT_CONVERGED, PENDING = 0, 1, 2
ERR_ARG, ERR_SINGULAR_ROW, ERR_ZERO_PIVOT, ERR_OVERFLOW = -1, -2, -3, -4
ERR_RANGE, ERR_OOM, ERR_DEVICE, ERR_BREAKDOWN, ERR_UNSUPPORTED = -5, -6, -7, -8, -9
PRE_NONE, PRE_JACOBI, PRE_ILU0 = 0, 1, 2
PRESET = {"paper_noprec": 0, "paper_ilu": 1, "jacobi": 2}
NO_EVENT = (1 << 63) - 1

_POLICY_INT_FIELDS = ("df", "alpha_a", "s_terms", "m", "precond", "b_dot", "b_axpy", "b_norm", "b_div_num",
                      "b_div_den", "b_rot", "b_tmp", "b_cs_num", "b_cs_den", "max_refine")


class Policy(C.Structure):
    _fields_ = ([("struct_size", C.c_int32)] + [(f, C.c_int32) for f in _POLICY_INT_FIELDS]
                + [("gtol", C.c_int64), ("tol", C.c_double), ("grid_blocks", C.c_int32),
                   ("phase_clock", C.c_int32), ("shift_retry", C.c_int32), ("two_sided", C.c_int32),
                   ("gauss_seidel", C.c_int32), ("sweep_rows", C.c_int32), ("sweep_lanes", C.c_int32),
                   ("s_rule", C.c_int32), ("spmv_lanes", C.c_int32), ("reserved_", C.c_int32 * 3)])

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f in _POLICY_INT_FIELDS}
        d.update(gtol=self.gtol, tol=self.tol, grid_blocks=self.grid_blocks, phase_clock=self.phase_clock,
                 shift_retry=self.shift_retry, two_sided=self.two_sided, gauss_seidel=self.gauss_seidel,
                 sweep_rows=self.sweep_rows, sweep_lanes=self.sweep_lanes, s_rule=self.s_rule,
                 spmv_lanes=self.spmv_lanes)
        return d


class Stats(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("status", C.c_int32), ("refinements", C.c_int32),
                ("iterations", C.c_int32), ("first_ovf", C.c_int64), ("relres_orig", C.c_double),
                ("relres_scaled", C.c_double), ("time_solve_ms", C.c_double), ("time_cycle_ms", C.c_double),
                ("time_setup_ms", C.c_double), ("n", C.c_int64), ("nnz", C.c_int64), ("nterms", C.c_int32),
                ("grid_blocks", C.c_int32), ("rows_per_thread", C.c_int32), ("block_threads", C.c_int32),
                ("levels_fwd", C.c_int32), ("levels_bwd", C.c_int32), ("device_bytes", C.c_int64),
                ("last_error_line", C.c_int32), ("shift_retries", C.c_int32), ("time_kernel_ms", C.c_double),
                ("phase_us", C.c_double * 8), ("spmv_lanes", C.c_int32), ("sweep_rows", C.c_int32),
                ("reserved_", C.c_int32 * 2)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if not f.endswith("_")}
        d["phase_us"] = list(self.phase_us)
        return d


class CycleTrace(C.Structure):
    _fields_ = [("m", C.c_int32), ("jstar", C.c_int32), ("breakdown", C.c_int32), ("steps", C.c_int32),
                ("first_ovf", C.c_int64), ("H", C.c_void_p), ("c", C.c_void_p), ("s", C.c_void_p),
                ("g", C.c_void_p), ("V", C.c_void_p)]


class IgmError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        super().__init__(f"{where}: {status_str(status)} ({status})")
        self.status = status


_lib = None

# Objects still open at interpreter exit are closed by an atexit hook, while
# the HIP runtime (and any profiler attached to it) is certainly alive; their
# __del__ does nothing once the interpreter is finalising.
_open = weakref.WeakSet()


@atexit.register
def _close_open_objects():
    for obj in list(_open):
        obj.close()

_SIGS = {
    "igm_policy_preset": [C.c_int32, C.c_void_p],
    "igm_create_system": [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "igm_set_policy": [C.c_void_p, C.c_void_p],
    "igm_set_rhs": [C.c_void_p, C.c_void_p],
    "igm_set_stream": [C.c_void_p, C.c_void_p],
    "igm_solve": [C.c_void_p, C.c_void_p],
    "igm_solve_device": [C.c_void_p, C.c_void_p],
    "igm_get_stats": [C.c_void_p, C.c_void_p],
    "igm_get_policy": [C.c_void_p, C.c_void_p],
    "igm_get_history": [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                        C.c_void_p],
    "igm_int_cycle": [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
    "igm_spmv": [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p],
    "igm_precond": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "igm_dot": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "igm_axpy": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p],
    "igm_norm": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "igm_normalize": [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p],
    "igm_residual": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "igm_fp_norm": [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p],
    "igm_start_vector": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "igm_reduce_noalloc": [C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                           C.c_void_p],
    "igm_destroy": [C.c_void_p],
    "igm_status_str": [C.c_int],
    "igm_batch_create": [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                         C.c_void_p, C.c_void_p],
    "igm_batch_set_stream": [C.c_void_p, C.c_void_p],
    "igm_batch_set_shape": [C.c_void_p, C.c_int32, C.c_int32],
    "igm_batch_autotune": [C.c_void_p, C.c_void_p, C.c_void_p],
    "igm_batch_set_phase_clock": [C.c_void_p, C.c_int32],
    "igm_batch_solve_device": [C.c_void_p, C.c_void_p],
    "igm_batch_solve": [C.c_void_p, C.c_void_p],
    "igm_batch_get_result": [C.c_void_p, C.c_int32, C.c_void_p],
    "igm_batch_get_stats": [C.c_void_p, C.c_void_p],
    "igm_batch_destroy": [C.c_void_p],
    "igm_server_create": [C.c_void_p, C.c_void_p],
    "igm_server_submit": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                          C.c_void_p, C.c_void_p],
    "igm_server_poll": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p],
    "igm_server_wait": [C.c_void_p, C.c_int64, C.c_double, C.c_void_p, C.c_void_p],
    "igm_server_get_stats": [C.c_void_p, C.c_void_p],
    "igm_server_destroy": [C.c_void_p, C.c_double],
}
EXPORTED = tuple(_SIGS)


def lib():
    """Load libigmres.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2009_07495_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.igm_destroy.restype = None
        L.igm_batch_destroy.restype = None
        L.igm_server_destroy.restype = None
        L.igm_status_str.restype = C.c_char_p
        _lib = L
    return _lib


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take a device pointer of {type(x)}")


def _check(st: int, where: str, ok=(OK,)):
    if st not in ok:
        raise IgmError(st, where)
    return st


def status_str(st: int) -> str:
    return lib().igm_status_str(st).decode()


igm_status_str = status_str


def igm_reduce_noalloc(mode: int, n: int, w, v, b: int, df: int, out_dev, stream=None) -> int:
    """Inner product (mode 0) or norm (mode 1) into out_dev[0..1] (device),
    enqueued on `stream` without any allocation; returns the status."""
    handle = getattr(stream, "cuda_stream", stream)
    return lib().igm_reduce_noalloc(int(mode), int(n), _ptr(w), _ptr(v), int(b), int(df), _ptr(out_dev),
                                    C.c_void_p(handle or 0))


def igm_policy_preset(preset) -> Policy:
    p = Policy()
    code = PRESET[preset] if isinstance(preset, str) else int(preset)
    _check(lib().igm_policy_preset(code, C.byref(p)), "igm_policy_preset")
    return p


def make_policy(preset: str = "paper_noprec", **overrides) -> Policy:
    p = igm_policy_preset(preset)
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _policy_struct(pol) -> Policy:
    if isinstance(pol, Policy):
        return pol
    p = igm_policy_preset(0)
    for k, v in dict(pol).items():
        if k == "pad_":
            continue
        setattr(p, k, v)
    return p


def igm_create_system(n, row_ptr, col, val, b, pol):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    vl = np.ascontiguousarray(val, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    h = C.c_void_p()
    ps = _policy_struct(pol)
    st = lib().igm_create_system(int(n), rp.ctypes.data, cl.ctypes.data, vl.ctypes.data, bb.ctypes.data,
                                 C.addressof(ps), C.byref(h))
    return st, h


class System:
    """One igm_system (owned; destroyed with the object)."""

    def __init__(self, n, row_ptr, col, val, b, pol="paper_noprec", **overrides):
        if isinstance(pol, str):
            pol = make_policy(pol, **overrides)
        st, h = igm_create_system(n, row_ptr, col, val, b, pol)
        _check(st, "igm_create_system")
        self.h = h
        self.n = int(n)
        self.pol = _policy_struct(pol)
        _open.add(self)

    @classmethod
    def from_system(cls, sysm, pol="paper_noprec", **overrides):
        return cls(sysm.n, sysm.row_ptr, sysm.col, sysm.val, sysm.b, pol, **overrides)

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.igm_destroy(self.h)
        self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if not _finalizing():  # see _open
            self.close()

    def set_policy(self, pol):
        ps = _policy_struct(pol)
        _check(lib().igm_set_policy(self.h, C.addressof(ps)), "igm_set_policy")
        self.pol = ps

    def set_rhs(self, b):
        bb = np.ascontiguousarray(b, dtype=np.float64)
        _check(lib().igm_set_rhs(self.h, bb.ctypes.data), "igm_set_rhs")

    def set_stream(self, stream):
        handle = getattr(stream, "cuda_stream", stream)
        _check(lib().igm_set_stream(self.h, C.c_void_p(handle or 0)), "igm_set_stream")

    def solve(self, x0=None):
        """Host solve: returns (x, status)."""
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        st = lib().igm_solve(self.h, x.ctypes.data)
        if st == ERR_DEVICE:
            raise IgmError(st, "igm_solve")
        return x, st

    def solve_device(self, x_dev) -> int:
        st = lib().igm_solve_device(self.h, _ptr(x_dev))
        if st == ERR_DEVICE:
            raise IgmError(st, "igm_solve_device")
        return st

    def stats(self) -> dict:
        s = Stats()
        s.struct_size = C.sizeof(Stats)
        _check(lib().igm_get_stats(self.h, C.byref(s)), "igm_get_stats")
        return s.as_dict()

    def policy(self) -> dict:
        """The current policy (shifts adjusted by overflow retries included)."""
        p = Policy()
        p.struct_size = C.sizeof(Policy)
        _check(lib().igm_get_policy(self.h, C.byref(p)), "igm_get_policy")
        return p.as_dict()

    def history(self, cap: int = 4096) -> dict:
        ro, rs, g, rho = (np.zeros(cap) for _ in range(4))
        js = np.zeros(cap, dtype=np.int32)
        cnt = C.c_int32(0)
        _check(lib().igm_get_history(self.h, cap, ro.ctypes.data, rs.ctypes.data, g.ctypes.data, rho.ctypes.data,
                                     js.ctypes.data, C.byref(cnt)), "igm_get_history")
        k = cnt.value
        return dict(relres_orig=ro[:k], relres_scaled=rs[:k], gamma=g[:k], rho=rho[:k], jstar=js[:k])

    def int_cycle(self, v1, with_basis: bool = True, k: int = 1) -> dict:
        """The int-GMRES call of refinement k (lines 3-20 of Fig. 2; the
        matrix Abar^(k) of eq. (AA)) from the integer v1."""
        m = self.pol.m
        v1 = np.ascontiguousarray(v1, dtype=np.int64)
        H = np.zeros((m + 1) * m, dtype=np.int64)
        c, s = np.zeros(m, dtype=np.int64), np.zeros(m, dtype=np.int64)
        g = np.zeros(m + 1, dtype=np.int64)
        V = np.zeros((m + 1) * self.n, dtype=np.int64) if with_basis else None
        t = CycleTrace(m, 0, 0, 0, 0, H.ctypes.data, c.ctypes.data, s.ctypes.data, g.ctypes.data,
                       V.ctypes.data if V is not None else None)
        _check(lib().igm_int_cycle(self.h, v1.ctypes.data, int(k), C.byref(t)), "igm_int_cycle")
        return dict(m=m, jstar=t.jstar, breakdown=t.breakdown, steps=t.steps, first_ovf=t.first_ovf,
                    H=H.reshape(m + 1, m), c=c, s=s, g=g, V=None if V is None else V.reshape(m + 1, self.n))

    # kernel-level entry points (device buffers)
    def spmv(self, v, z, nterms=None) -> int:
        ev = C.c_int64(0)
        nt = self.pol.s_terms + 1 if nterms is None else nterms
        _check(lib().igm_spmv(self.h, nt, _ptr(v), _ptr(z), C.byref(ev)), "igm_spmv")
        return ev.value

    def precond(self, z, w) -> int:
        ev = C.c_int64(0)
        _check(lib().igm_precond(self.h, _ptr(z), _ptr(w), C.byref(ev)), "igm_precond")
        return ev.value

    def dot(self, w, v):
        h, ev = C.c_int64(0), C.c_int64(0)
        _check(lib().igm_dot(self.h, _ptr(w), _ptr(v), C.byref(h), C.byref(ev)), "igm_dot")
        return h.value, ev.value

    def axpy(self, h: int, w, v) -> int:
        ev = C.c_int64(0)
        _check(lib().igm_axpy(self.h, int(h), _ptr(w), _ptr(v), C.byref(ev)), "igm_axpy")
        return ev.value

    def norm(self, w):
        h, ev = C.c_int64(0), C.c_int64(0)
        _check(lib().igm_norm(self.h, _ptr(w), C.byref(h), C.byref(ev)), "igm_norm")
        return h.value, ev.value

    def normalize(self, w, h: int, v) -> int:
        ev = C.c_int64(0)
        _check(lib().igm_normalize(self.h, _ptr(w), int(h), _ptr(v), C.byref(ev)), "igm_normalize")
        return ev.value

    def residual(self, x, r, rhat):
        _check(lib().igm_residual(self.h, _ptr(x), _ptr(r), _ptr(rhat)), "igm_residual")

    def fp_norm(self, x, length=None) -> float:
        out = C.c_double(0)
        ln = self.n if length is None else length
        _check(lib().igm_fp_norm(self.h, _ptr(x), ln, C.byref(out)), "igm_fp_norm")
        return out.value

    def start_vector(self, r, bk, r0, v1):
        g, rho = C.c_double(0), C.c_double(0)
        st = lib().igm_start_vector(self.h, _ptr(r), _ptr(bk), _ptr(r0), _ptr(v1), C.byref(g), C.byref(rho))
        _check(st, "igm_start_vector", ok=(OK, ERR_RANGE))
        return st, g.value, rho.value


class Batch:
    """One igm_batch: many independent systems solved in one persistent launch
    (owned; destroyed with the object). Solutions are laid end to end in
    system order; ``offsets[i]`` is where system i starts."""

    def __init__(self, systems, pol="jacobi", **overrides):
        if isinstance(pol, str):
            pol = make_policy(pol, **overrides)
        self.pol = _policy_struct(pol)
        ns = len(systems)
        self.n = np.array([s.n for s in systems], dtype=np.int64)
        self.nnz = np.array([s.nnz for s in systems], dtype=np.int64)
        self.offsets = np.zeros(ns + 1, dtype=np.int64)
        np.cumsum(self.n, out=self.offsets[1:])
        self.total_n = int(self.offsets[-1])
        rp = np.ascontiguousarray(np.concatenate([np.asarray(s.row_ptr, dtype=np.int64) for s in systems]))
        cl = np.ascontiguousarray(np.concatenate([np.asarray(s.col, dtype=np.int32) for s in systems]))
        vl = np.ascontiguousarray(np.concatenate([np.asarray(s.val, dtype=np.float64) for s in systems]))
        bb = np.ascontiguousarray(np.concatenate([np.asarray(s.b, dtype=np.float64) for s in systems]))
        failed = C.c_int32(-1)
        h = C.c_void_p()
        st = lib().igm_batch_create(ns, self.n.ctypes.data, rp.ctypes.data, cl.ctypes.data, vl.ctypes.data,
                                    bb.ctypes.data, C.addressof(self.pol), C.byref(failed), C.byref(h))
        if st != OK:
            raise IgmError(st, f"igm_batch_create (system {failed.value})")
        self.h = h
        self.nsys = ns
        _open.add(self)

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.igm_batch_destroy(self.h)
        self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if not _finalizing():  # see _open
            self.close()

    def set_stream(self, stream):
        handle = getattr(stream, "cuda_stream", stream)
        _check(lib().igm_batch_set_stream(self.h, C.c_void_p(handle or 0)), "igm_batch_set_stream")

    def set_shape(self, block: int, rows_per_thread: int) -> int:
        return lib().igm_batch_set_shape(self.h, int(block), int(rows_per_thread))

    def set_phase_clock(self, on: bool):
        _check(lib().igm_batch_set_phase_clock(self.h, int(bool(on))), "igm_batch_set_phase_clock")

    def autotune(self):
        b, r = C.c_int32(0), C.c_int32(0)
        _check(lib().igm_batch_autotune(self.h, C.byref(b), C.byref(r)), "igm_batch_autotune")
        return b.value, r.value

    def solve_device(self, x_dev) -> int:
        st = lib().igm_batch_solve_device(self.h, _ptr(x_dev))
        if st == ERR_DEVICE:
            raise IgmError(st, "igm_batch_solve_device")
        return st

    def solve(self, x0=None):
        x = np.zeros(self.total_n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        st = lib().igm_batch_solve(self.h, x.ctypes.data)
        if st == ERR_DEVICE:
            raise IgmError(st, "igm_batch_solve")
        return x, st

    def result(self, i: int) -> dict:
        s = Stats()
        s.struct_size = C.sizeof(Stats)
        _check(lib().igm_batch_get_result(self.h, int(i), C.byref(s)), "igm_batch_get_result")
        return s.as_dict()

    def results(self) -> list:
        return [self.result(i) for i in range(self.nsys)]

    def stats(self) -> dict:
        s = Stats()
        s.struct_size = C.sizeof(Stats)
        _check(lib().igm_batch_get_stats(self.h, C.byref(s)), "igm_batch_get_stats")
        return s.as_dict()


class ServerConfig(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("block", C.c_int32), ("rows_per_thread", C.c_int32),
                ("max_slots", C.c_int32), ("setup_threads", C.c_int32), ("reserve_cus", C.c_int32),
                ("pool_bytes", C.c_int64), ("stage_bytes", C.c_int64), ("host_setup", C.c_int32),
                ("reserved_", C.c_int32 * 5)]


class ServerStats(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("slots_used", C.c_int32), ("submitted", C.c_int64),
                ("completed", C.c_int64), ("prepared_waiting", C.c_int64), ("resident", C.c_int64),
                ("pool_bytes", C.c_int64), ("pool_used", C.c_int64), ("pool_peak", C.c_int64),
                ("workgroups", C.c_int64), ("workgroups_busy", C.c_int64), ("block_threads", C.c_int32),
                ("rows_per_thread", C.c_int32), ("setup_waiting", C.c_int64), ("jobs_published", C.c_int64),
                ("kernel_alive", C.c_int32), ("reserved_", C.c_int32 * 5)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if not f.endswith("_")}


class Server:
    """One igm_server: a persistent kernel that solves submitted requests as
    they arrive (continuous batching). Owned; closing drains it."""

    def __init__(self, block=0, rows_per_thread=0, max_slots=0, setup_threads=0, pool_bytes=0, reserve_cus=0,
                 stage_bytes=0, host_setup=False):
        cfg = ServerConfig(C.sizeof(ServerConfig), block, rows_per_thread, max_slots, setup_threads, reserve_cus,
                           int(pool_bytes), int(stage_bytes), 1 if host_setup else 0)
        h = C.c_void_p()
        _check(lib().igm_server_create(C.byref(cfg), C.byref(h)), "igm_server_create")
        self.h = h
        self._n = {}
        _open.add(self)

    def close(self, timeout_ms: float = 60000.0):
        if getattr(self, "h", None) and _lib is not None:
            _lib.igm_server_destroy(self.h, float(timeout_ms))
        self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if not _finalizing():  # see _open
            self.close(10000.0)

    def submit(self, sysm, pol="jacobi", x0=None, **overrides) -> int:
        if isinstance(pol, str):
            pol = make_policy(pol, **overrides)
        ps = _policy_struct(pol)
        rp = np.ascontiguousarray(sysm.row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(sysm.col, dtype=np.int32)
        vl = np.ascontiguousarray(sysm.val, dtype=np.float64)
        bb = np.ascontiguousarray(sysm.b, dtype=np.float64)
        xx = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        t = C.c_int64(-1)
        _check(lib().igm_server_submit(self.h, int(sysm.n), rp.ctypes.data, cl.ctypes.data, vl.ctypes.data,
                                       bb.ctypes.data, None if xx is None else xx.ctypes.data,
                                       C.addressof(ps), C.byref(t)), "igm_server_submit")
        self._n[t.value] = int(sysm.n)
        return t.value

    def poll(self, ticket: int):
        """(done, x, stats); x and stats are None until done."""
        x = np.zeros(max(self._n.get(ticket, 0), 1))  # unknown tickets: the library reports ERR_ARG
        s = Stats()
        s.struct_size = C.sizeof(Stats)
        done = C.c_int32(0)
        _check(lib().igm_server_poll(self.h, int(ticket), C.byref(done), x.ctypes.data, C.byref(s)),
               "igm_server_poll")
        if not done.value:
            return False, None, None
        n = self._n.pop(ticket)
        return True, x[:n], s.as_dict()

    def wait(self, ticket: int, timeout_ms: float = -1.0):
        """(x, stats) once the request has finished; raises IgmError(PENDING) on timeout."""
        x = np.zeros(max(self._n.get(ticket, 0), 1))  # unknown tickets: the library reports ERR_ARG
        s = Stats()
        s.struct_size = C.sizeof(Stats)
        st = lib().igm_server_wait(self.h, int(ticket), float(timeout_ms), x.ctypes.data, C.byref(s))
        if st != OK:
            raise IgmError(st, f"igm_server_wait (server: {self.stats()})")
        n = self._n.pop(ticket)
        return x[:n], s.as_dict()

    def stats(self) -> dict:
        s = ServerStats()
        s.struct_size = C.sizeof(ServerStats)
        _check(lib().igm_server_get_stats(self.h, C.byref(s)), "igm_server_get_stats")
        return s.as_dict()
