"""ctypes wrapper around the C oracle (``liborc.so``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this module to compute expected results; the GPU library
never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
SOURCES = ["orc_fx.c", "orc_setup.c", "orc_cycle.c", "orc_ir.c", "orc_gmres64.c"]
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra"]

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_SINGULAR_ROW, ERR_ZERO_PIVOT, ERR_OVERFLOW, ERR_RANGE, ERR_BREAKDOWN = -1, -2, -3, -4, -5, -8
PRE_NONE, PRE_JACOBI, PRE_ILU0 = 0, 1, 2
NO_EVENT = (1 << 63) - 1


def code(j: int, stage: int, sub: int = 0) -> int:
    """Overflow event code: step j, stage (1 SpMV .. 9 rotation of g), sub-index."""
    return (j << 24) | (stage << 16) | sub


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liborc.so."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", *CFLAGS, "-o", LIB_PATH + ".tmp", *[os.path.join(HERE, s) for s in SOURCES], "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Policy(C.Structure):
    _fields_ = [(name, C.c_int32) for name in (
        "df", "alpha_a", "s_terms", "m", "precond", "b_dot", "b_axpy", "b_norm", "b_div_num", "b_div_den",
        "b_rot", "b_tmp", "b_cs_num", "b_cs_den", "max_refine", "shift_retry")] + [("gtol", C.c_int64), ("tol", C.c_double),
                                                                            ("two_sided", C.c_int32), ("gauss_seidel", C.c_int32),
                                                                            ("s_rule", C.c_int32)]


# Shift settings of the paper: Table IV (no preconditioner) and Table VI (ILU),
# with d_f = 30, WL = 64, s = 0, alpha_a = 16 / 32 (Sec. VII-B, VII-C).
# "jacobi" is this implementation's extension: the ILU construction on the
# diagonal-only pattern with the Table VI shifts.
_BASE = dict(df=30, s_terms=0, m=30, max_refine=2000, shift_retry=0, gtol=-1, tol=1e-10, two_sided=0,
             gauss_seidel=0, s_rule=0)
PRESETS = {
    "paper_noprec": dict(_BASE, alpha_a=16, precond=PRE_NONE, b_dot=16, b_axpy=16, b_norm=16, b_div_num=16,
                         b_div_den=14, b_rot=16, b_tmp=16, b_cs_num=16, b_cs_den=14),
    "paper_ilu": dict(_BASE, alpha_a=32, precond=PRE_ILU0, b_dot=0, b_axpy=0, b_norm=0, b_div_num=30,
                      b_div_den=0, b_rot=0, b_tmp=0, b_cs_num=30, b_cs_den=0),
    "jacobi": dict(_BASE, alpha_a=32, precond=PRE_JACOBI, b_dot=0, b_axpy=0, b_norm=0, b_div_num=30,
                   b_div_den=0, b_rot=0, b_tmp=0, b_cs_num=30, b_cs_den=0),
}


def shift_retry(pol: dict, code: int):
    """orc_shift_retry on a copy of `pol`: (changed, new policy dict)."""
    p = _policy_struct(pol)
    changed = lib().orc_shift_retry(C.byref(p), code)
    return bool(changed), {name: getattr(p, name) for name, _ in Policy._fields_}


def policy(preset: str = "paper_noprec", **overrides) -> dict:
    p = dict(PRESETS[preset])
    p.update(overrides)
    return p


def _policy_struct(p: dict) -> Policy:
    s = Policy()
    for k, v in p.items():
        setattr(s, k, v)
    return s


class Trace(C.Structure):
    _fields_ = [("m", C.c_int32), ("jstar", C.c_int32), ("breakdown", C.c_int32), ("steps", C.c_int32),
                ("first_ovf", C.c_int64), ("H", C.c_void_p), ("c", C.c_void_p), ("s", C.c_void_p),
                ("g", C.c_void_p), ("V", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("refinements", C.c_int32), ("iterations", C.c_int32),
                ("hist_cap", C.c_int32), ("first_ovf", C.c_int64), ("relres_orig", C.c_double),
                ("relres_scaled", C.c_double), ("hist_relres_orig", C.c_void_p), ("hist_relres_scaled", C.c_void_p),
                ("hist_gamma", C.c_void_p), ("hist_rho", C.c_void_p), ("hist_jstar", C.c_void_p),
                ("shift_retries", C.c_int32), ("pad_", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        i64, i32, dbl, vp = C.c_int64, C.c_int32, C.c_double, C.c_void_p
        pi32 = C.POINTER(C.c_int32)
        sig = {
            "orc_asr": (i64, [i64, i32]),
            "orc_shl": (i64, [i64, i32, pi32]),
            "orc_sc": (i64, [i64, i32, pi32]),
            "orc_tdiv": (i64, [i64, i64, pi32]),
            "orc_isqrt": (i64, [i64]),
            "orc_trunc": (i64, [dbl, pi32]),
            "orc_mul": (i64, [i64, i64, i32, i32, i32, pi32]),
            "orc_div": (i64, [i64, i64, i32, i32, i32, pi32, pi32]),
            "orc_dot": (i64, [i64, vp, vp, i32, i32, pi32]),
            "orc_norm": (i64, [i64, vp, i32, i32, pi32]),
            "orc_axpy": (None, [i64, vp, vp, i64, i32, i32, pi32]),
            "orc_normalize": (None, [i64, vp, i64, i32, i32, i32, vp, pi32]),
            "orc_dnrm": (dbl, [i64, vp]),
            "orc_u128_to_double": (dbl, [C.c_uint64, C.c_uint64]),
            "orc_create": (C.c_int, [i64, vp, vp, vp, vp, C.POINTER(Policy), C.POINTER(vp)]),
            "orc_destroy": (None, [vp]),
            "orc_n": (i64, [vp]),
            "orc_nnz": (i64, [vp]),
            "orc_nterms": (i32, [vp]),
            "orc_get_scaled": (None, [vp, vp, vp, vp]),
            "orc_get_terms": (None, [vp, vp, vp]),
            "orc_get_precond": (None, [vp, vp, vp, vp]),
            "orc_get_ilu_fp": (C.c_int, [vp, vp]),
            "orc_spmv": (None, [vp, i32, vp, vp, i32, C.POINTER(i64)]),
            "orc_precond_apply": (None, [vp, vp, vp, i32, C.POINTER(i64)]),
            "orc_cycle": (C.c_int, [vp, vp, i32, C.POINTER(Trace)]),
            "orc_cycle_update": (None, [vp, C.POINTER(Trace), dbl, vp]),
            "orc_solve": (C.c_int, [vp, vp, C.POINTER(Stats)]),
            "orc_shift_retry": (C.c_int, [C.POINTER(Policy), i64]),
            "orc_get_policy": (None, [vp, C.POINTER(Policy)]),
            "orc_residual": (None, [vp, vp, vp, vp]),
            "orc_start_vector": (C.c_int, [vp, vp, vp, vp, vp, C.POINTER(dbl), C.POINTER(dbl)]),
            "orc_gmres64": (C.c_int, [vp, i32, dbl, i32, vp, C.POINTER(i32)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int64)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---- primitives ----------------------------------------------------------
def asr(x: int, b: int) -> int:
    return lib().orc_asr(x, b)


def shl(x: int, b: int):
    o = C.c_int32(0)
    r = lib().orc_shl(x, b, C.byref(o))
    return r, bool(o.value)


def sc(x: int, e: int):
    o = C.c_int32(0)
    r = lib().orc_sc(x, e, C.byref(o))
    return r, bool(o.value)


def tdiv(a: int, d: int):
    o = C.c_int32(0)
    r = lib().orc_tdiv(a, d, C.byref(o))
    return r, bool(o.value)


def isqrt(x: int) -> int:
    return lib().orc_isqrt(x)


def trunc(y: float):
    o = C.c_int32(0)
    r = lib().orc_trunc(y, C.byref(o))
    return r, bool(o.value)


def mul(t1: int, t2: int, b1: int, b2: int, df: int = 30):
    o = C.c_int32(0)
    r = lib().orc_mul(t1, t2, b1, b2, df, C.byref(o))
    return r, bool(o.value)


def div(t1: int, t2: int, b1: int, b2: int, df: int = 30):
    o, z = C.c_int32(0), C.c_int32(0)
    r = lib().orc_div(t1, t2, b1, b2, df, C.byref(o), C.byref(z))
    return r, bool(o.value), bool(z.value)


def dot(w, v, b: int, df: int = 30):
    w, v = _i64(w), _i64(v)
    o = C.c_int32(0)
    r = lib().orc_dot(len(w), _p(w), _p(v), b, df, C.byref(o))
    return r, bool(o.value)


def norm(w, b: int, df: int = 30):
    w = _i64(w)
    o = C.c_int32(0)
    r = lib().orc_norm(len(w), _p(w), b, df, C.byref(o))
    return r, bool(o.value)


def axpy(w, v, h: int, b: int, df: int = 30):
    w = _i64(w).copy()
    v = _i64(v)
    o = C.c_int32(0)
    lib().orc_axpy(len(w), _p(w), _p(v), h, b, df, C.byref(o))
    return w, bool(o.value)


def normalize(w, den: int, b1: int, b2: int, df: int = 30):
    w = _i64(w)
    v = np.empty_like(w)
    o = C.c_int32(0)
    lib().orc_normalize(len(w), _p(w), den, b1, b2, df, _p(v), C.byref(o))
    return v, bool(o.value)


def dnrm(x) -> float:
    x = _f64(x)
    return lib().orc_dnrm(len(x), _p(x))


def u128_to_double(v: int) -> float:
    return lib().orc_u128_to_double(v & ((1 << 64) - 1), v >> 64)


# ---- system --------------------------------------------------------------
class OracleSystem:
    """One linear system set up by the oracle (scaling, A_l, preconditioner)."""

    def __init__(self, n, row_ptr, col, val, b, pol: dict):
        self.pol = dict(pol)
        self.n = int(n)
        self._keep = (_i64(row_ptr), np.ascontiguousarray(col, dtype=np.int32), _f64(val), _f64(b))
        h = C.c_void_p()
        ps = _policy_struct(self.pol)
        self.status = lib().orc_create(self.n, *[_p(a) for a in self._keep], C.byref(ps), C.byref(h))
        self.h = h
        if self.status != OK:
            self.h = None
            raise OracleError(self.status)
        self.nnz = lib().orc_nnz(self.h)
        self.nterms = lib().orc_nterms(self.h)

    @classmethod
    def from_system(cls, sysm, pol: dict):
        return cls(sysm.n, sysm.row_ptr, sysm.col, sysm.val, sysm.b, pol)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def policy_now(self) -> dict:
        """The system's current policy (shifts adjusted by overflow retries included)."""
        p = Policy()
        lib().orc_get_policy(self.h, C.byref(p))
        return {name: getattr(p, name) for name, _ in Policy._fields_}

    def scaled(self):
        d, a, b = np.empty(self.n), np.empty(self.nnz), np.empty(self.n)
        lib().orc_get_scaled(self.h, _p(d), _p(a), _p(b))
        return d, a, b

    def terms(self):
        ab = np.empty(self.nterms * max(self.nnz, 1), dtype=np.int64)
        al = np.empty(self.nterms, dtype=np.int32)
        lib().orc_get_terms(self.h, _p(ab), _p(al))
        return ab[: self.nterms * self.nnz].reshape(self.nterms, self.nnz), al

    def precond(self):
        fac = np.zeros(self.nnz, dtype=np.int64)
        ld, ud = np.zeros(self.n, dtype=np.int64), np.zeros(self.n, dtype=np.int64)
        lib().orc_get_precond(self.h, _p(fac), _p(ld), _p(ud))
        return fac, ld, ud

    def ilu_fp(self):
        lu = np.empty(self.nnz)
        return lu if lib().orc_get_ilu_fp(self.h, _p(lu)) else None

    def spmv(self, v, nterms=None, j=1):
        v = _i64(v)
        z = np.empty(self.n, dtype=np.int64)
        first = C.c_int64(NO_EVENT)
        nt = self.pol["s_terms"] + 1 if nterms is None else nterms
        lib().orc_spmv(self.h, nt, _p(v), _p(z), j, C.byref(first))
        return z, first.value

    def precond_apply(self, z, j=1):
        z = _i64(z)
        w = np.empty(self.n, dtype=np.int64)
        first = C.c_int64(NO_EVENT)
        lib().orc_precond_apply(self.h, _p(z), _p(w), j, C.byref(first))
        return w, first.value

    def cycle(self, v1, m=None, k: int = 1):
        """The int-GMRES call of refinement k (its matrix per eq. (AA))."""
        m = self.pol["m"] if m is None else m
        v1 = _i64(v1)
        H = np.zeros((m + 1) * m, dtype=np.int64)
        c, s = np.zeros(m, dtype=np.int64), np.zeros(m, dtype=np.int64)
        g = np.zeros(m + 1, dtype=np.int64)
        V = np.zeros(self.n * (m + 1), dtype=np.int64)
        t = Trace(m, 0, 0, 0, 0, _p(H).value, _p(c).value, _p(s).value, _p(g).value, _p(V).value)
        rc = lib().orc_cycle(self.h, _p(v1), int(k), C.byref(t))
        if rc != OK:
            raise OracleError(rc)
        out = dict(m=m, jstar=t.jstar, breakdown=t.breakdown, steps=t.steps, first_ovf=t.first_ovf,
                   H=H.reshape(m + 1, m), c=c, s=s, g=g, V=V.reshape(m + 1, self.n))
        out["_t"] = t
        out["_keep"] = (H, c, s, g, V)
        return out

    def cycle_update(self, tr: dict, rho: float):
        x = np.empty(self.n)
        lib().orc_cycle_update(self.h, C.byref(tr["_t"]), rho, _p(x))
        return x

    def residual(self, x):
        x = _f64(x)
        r, rh = np.empty(self.n), np.empty(self.n)
        lib().orc_residual(self.h, _p(x), _p(r), _p(rh))
        return r, rh

    def start_vector(self, r):
        r = _f64(r)
        bk, r0 = np.empty(self.n), np.empty(self.n)
        v1 = np.empty(self.n, dtype=np.int64)
        g, rho = C.c_double(0), C.c_double(0)
        rc = lib().orc_start_vector(self.h, _p(r), _p(bk), _p(r0), _p(v1), C.byref(g), C.byref(rho))
        return dict(status=rc, bk=bk, r0=r0, v1=v1, gamma=g.value, rho=rho.value)

    def solve(self, x0=None, hist_cap: int | None = None):
        x = np.zeros(self.n) if x0 is None else _f64(x0).copy()
        cap = (self.pol["max_refine"] + 1) if hist_cap is None else hist_cap
        cap = max(cap, 1)
        h_ro, h_rs, h_g, h_rho = (np.full(cap, np.nan) for _ in range(4))
        h_j = np.full(cap, -1, dtype=np.int32)
        st = Stats(0, 0, 0, cap, 0, 0.0, 0.0, _p(h_ro).value, _p(h_rs).value, _p(h_g).value, _p(h_rho).value,
                   _p(h_j).value)
        rc = lib().orc_solve(self.h, _p(x), C.byref(st))
        k = st.refinements
        stats = dict(status=rc, refinements=st.refinements, iterations=st.iterations, first_ovf=st.first_ovf,
                     shift_retries=st.shift_retries,
                     relres_orig=st.relres_orig, relres_scaled=st.relres_scaled,
                     hist_relres_orig=h_ro[: min(k + 1, cap)], hist_relres_scaled=h_rs[: min(k + 1, cap)],
                     hist_gamma=h_g[: min(k + 1, cap)], hist_rho=h_rho[: min(k + 1, cap)],
                     hist_jstar=h_j[: min(k, cap)])
        return x, stats

    def gmres64(self, m=None, tol=None, max_restart=2000):
        m = self.pol["m"] if m is None else m
        tol = self.pol["tol"] if tol is None else tol
        x = np.zeros(self.n)
        it = C.c_int32(0)
        rc = lib().orc_gmres64(self.h, m, tol, max_restart, _p(x), C.byref(it))
        return x, it.value, rc


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status
