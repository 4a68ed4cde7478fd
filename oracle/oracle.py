"""ctypes wrapper around the C oracle plus the dense double reference.

Test infrastructure only (see the package docstring).
"""

from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

from fps_inputs.generators import CSR

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB lets the mutation tests point the wrapper at a deliberately broken build
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()


class _Csr(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("nnz", C.c_int64),
        ("row_ptr", C.POINTER(C.c_int64)),
        ("col", C.POINTER(C.c_int32)),
        ("val", C.POINTER(C.c_double)),
    ]


class _Stats(C.Structure):
    _fields_ = [
        ("kind", C.c_int32),
        ("index", C.c_int32),
        ("products", C.c_int64),
        ("nnz_struct", C.c_int64),
        ("nnz_kept", C.c_int64),
        ("n_dropped", C.c_int64),
        ("n_zero", C.c_int64),
        ("dropped_1norm", C.c_double),
        ("dropped_max", C.c_double),
        ("kept_min", C.c_double),
    ]


class _Alg1(C.Structure):
    _fields_ = [
        ("eps_g", C.c_double),
        ("threshold", C.c_double),
        ("dropped", C.c_double),
        ("iters", C.c_int32),
        ("pad", C.c_int32),
    ]


STAGE_KINDS = {0: "power", 1: "block", 2: "gstep", 3: "horner"}


def lib_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                from . import build as _b

                _b.build()
            lib = C.CDLL(_LIB_PATH)
            P = C.POINTER
            lib.orc_spgemm.argtypes = [P(_Csr), P(_Csr), P(_Csr), C.c_double, P(_Csr), P(_Stats), C.c_int]
            lib.orc_spgemm.restype = C.c_int
            lib.orc_axpy.argtypes = [C.c_int64, C.c_int, P(C.c_double), P(P(_Csr)), P(_Csr), P(_Stats), C.c_int]
            lib.orc_axpy.restype = C.c_int
            lib.orc_schedule.argtypes = [C.c_int, C.c_int] + [P(C.c_int)] * 7
            lib.orc_schedule.restype = C.c_int
            lib.orc_filtered_ps.argtypes = [P(_Csr), P(C.c_double), C.c_int, C.c_int, C.c_double, P(_Csr),
                                            P(_Stats), C.c_int, P(C.c_int), C.c_int]
            lib.orc_filtered_ps.restype = C.c_int
            lib.orc_dense_horner_ld.argtypes = [C.c_int64, P(C.c_double), P(C.c_double), C.c_int,
                                                P(C.c_longdouble)]
            lib.orc_dense_horner_ld.restype = C.c_int
            lib.orc_csr_free.argtypes = [P(_Csr)]
            lib.orc_csr_free.restype = None
            lib.orc_alg1_filter.argtypes = [P(_Csr), C.c_double, C.c_double, C.c_int, P(_Alg1)]
            lib.orc_alg1_filter.restype = C.c_int
            lib.orc_fnt_thresholds.argtypes = [P(C.c_double), C.c_int, C.c_int, C.c_double, P(C.c_double),
                                               P(C.c_double), P(C.c_double)]
            lib.orc_fnt_thresholds.restype = C.c_int
            lib.orc_filtered_ps_adaptive.argtypes = [P(_Csr), P(C.c_double), C.c_int, C.c_int, C.c_double,
                                                     C.c_double, P(C.c_double), P(_Csr), P(_Stats), C.c_int,
                                                     P(C.c_int), P(_Alg1), C.c_int, P(C.c_int), C.c_int]
            lib.orc_filtered_ps_adaptive.restype = C.c_int
            lib.orc_normest1_power.argtypes = [P(_Csr), C.c_int, P(C.c_double), P(C.c_int64), P(C.c_int)]
            lib.orc_normest1_power.restype = C.c_int
            lib.orc_power_norm_bounds.argtypes = [P(_Csr), C.c_int, C.c_int, P(C.c_double)]
            lib.orc_power_norm_bounds.restype = C.c_int
            lib.orc_series_degree.argtypes = [P(C.c_double), C.c_int, P(C.c_double), C.c_double, P(C.c_int),
                                              P(C.c_int), P(C.c_double)]
            lib.orc_series_degree.restype = C.c_int
            _lib = lib
    return _lib


def _view(m, keep):
    rp = np.ascontiguousarray(m.row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(m.col, dtype=np.int32)
    vl = np.ascontiguousarray(m.val, dtype=np.float64)
    keep.extend([rp, cl, vl])
    s = _Csr()
    s.n = int(m.n)
    s.nnz = int(rp[-1])
    s.row_ptr = rp.ctypes.data_as(C.POINTER(C.c_int64))
    s.col = cl.ctypes.data_as(C.POINTER(C.c_int32))
    s.val = vl.ctypes.data_as(C.POINTER(C.c_double))
    return s


def _take(out: _Csr) -> CSR:
    lib = _load()
    n = int(out.n)
    nnz = int(out.nnz)
    rp = np.ctypeslib.as_array(out.row_ptr, shape=(n + 1,)).copy()
    cl = np.ctypeslib.as_array(out.col, shape=(max(nnz, 1),))[:nnz].copy()
    vl = np.ctypeslib.as_array(out.val, shape=(max(nnz, 1),))[:nnz].copy()
    lib.orc_csr_free(C.byref(out))
    return CSR(n, rp, cl, vl)


def _stats_dict(s: _Stats) -> dict:
    d = {f: getattr(s, f) for f, _ in _Stats._fields_}
    d["kind_name"] = STAGE_KINDS.get(d["kind"], "?")
    return d


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def schedule(m: int, s: int) -> dict:
    """N, q, b, g of eq. 6 with q = s given; J = highest power formed; start =
    first filtered Horner step; n_spgemm = number of sparse products."""
    lib = _load()
    vals = [C.c_int() for _ in range(7)]
    _check(lib.orc_schedule(m, s, *[C.byref(v) for v in vals]), "schedule")
    keys = ["N", "q", "b", "g", "J", "start", "n_spgemm"]
    return {k: v.value for k, v in zip(keys, vals)}


def spgemm(A, B, E=None, tau: float = 0.0, nthreads: int = 0):
    """D_tau(E + A (x) B) with Gustavson rows, k-ascending fma accumulation."""
    lib = _load()
    keep = []
    a, b = _view(A, keep), _view(B, keep)
    e = _view(E, keep) if E is not None else None
    out, st = _Csr(), _Stats()
    _check(lib.orc_spgemm(C.byref(a), C.byref(b), C.byref(e) if e is not None else None, float(tau),
                          C.byref(out), C.byref(st), int(nthreads)), "spgemm")
    return _take(out), _stats_dict(st)


def axpy(n: int, coefs, mats, nthreads: int = 0):
    """sum_t coefs[t] * mats[t] in the given order (None = identity); exact zeros dropped."""
    lib = _load()
    keep = []
    views = [None if m is None else _view(m, keep) for m in mats]
    arr = (C.POINTER(_Csr) * max(len(mats), 1))()
    for i, v in enumerate(views):
        arr[i] = C.pointer(v) if v is not None else C.POINTER(_Csr)()
    cf = np.ascontiguousarray(coefs, dtype=np.float64)
    out, st = _Csr(), _Stats()
    _check(lib.orc_axpy(int(n), len(mats), cf.ctypes.data_as(C.POINTER(C.c_double)), arr, C.byref(out),
                        C.byref(st), int(nthreads)), "axpy")
    return _take(out), _stats_dict(st)


def filtered_ps(Z, coeffs, m: int, s: int, tau: float, nthreads: int = 0):
    """Filtered PS evaluation with a fixed tau.  Returns (F, per-stage stats)."""
    lib = _load()
    keep = []
    z = _view(Z, keep)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    if c.size < m + 1:
        raise ValueError("need m+1 coefficients")
    max_stats = 4 * (m + 4) + 8
    stats = (_Stats * max_stats)()
    ns = C.c_int()
    out = _Csr()
    _check(lib.orc_filtered_ps(C.byref(z), c.ctypes.data_as(C.POINTER(C.c_double)), int(m), int(s),
                               float(tau), C.byref(out), stats, max_stats, C.byref(ns), int(nthreads)),
           "filtered_ps")
    return _take(out), [_stats_dict(stats[i]) for i in range(min(ns.value, max_stats))]


def unfiltered_ps(Z, coeffs, m: int, s: int, nthreads: int = 0):
    """PS scheme (eqs. 2-4) with nothing filtered (tau = 0; exact zeros dropped)."""
    return filtered_ps(Z, coeffs, m, s, 0.0, nthreads)


def dense_horner(Zd: np.ndarray, coeffs, m: int | None = None) -> np.ndarray:
    """P_m(Z) = sum c_k Z^k by the Qin/Horner scheme: Y = c_m I, Y = Y Z + c_k I."""
    c = np.asarray(coeffs, dtype=np.float64)
    if m is None:
        m = c.size - 1
    n = Zd.shape[0]
    Y = c[m] * np.eye(n)
    for k in range(m - 1, -1, -1):
        Y = Y @ Zd
        Y[np.diag_indices(n)] += c[k]
    return Y


def dense_horner_ld(Zd: np.ndarray, coeffs, m: int | None = None) -> np.ndarray:
    """Same definition evaluated in long double (x87 extended) in C."""
    lib = _load()
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    if m is None:
        m = c.size - 1
    Zc = np.ascontiguousarray(Zd, dtype=np.float64)
    n = Zc.shape[0]
    Y = np.zeros((n, n), dtype=np.longdouble)
    _check(lib.orc_dense_horner_ld(n, Zc.ctypes.data_as(C.POINTER(C.c_double)),
                                   c.ctypes.data_as(C.POINTER(C.c_double)), int(m),
                                   Y.ctypes.data_as(C.POINTER(C.c_longdouble))), "dense_horner_ld")
    return Y


def norm1(M) -> float:
    """Max column absolute sum of a dense array or CSR."""
    if isinstance(M, np.ndarray):
        return float(np.max(np.sum(np.abs(M), axis=0))) if M.size else 0.0
    cs = np.zeros(M.n)
    np.add.at(cs, M.col, np.abs(M.val))
    return float(cs.max()) if M.n else 0.0


def fro_norm(M) -> float:
    if isinstance(M, np.ndarray):
        return float(np.sqrt(np.sum(np.abs(M) ** 2)))
    return float(np.sqrt(np.sum(M.val ** 2)))


# ---------------------------------------------------------------------------
# Adaptive filter (Algorithm 1) and the eq. 28 thresholds
# ---------------------------------------------------------------------------

def _alg1_dict(a: _Alg1) -> dict:
    return {"eps_g": a.eps_g, "threshold": a.threshold, "dropped": a.dropped, "iters": a.iters}


def alg1_filter(M, eps_g: float, e_r: float, max_iter: int = 200):
    """Algorithm 1 on a copy of M: returns (filtered matrix, record)."""
    lib = _load()
    rp = np.array(M.row_ptr, dtype=np.int64)
    cl = np.array(M.col, dtype=np.int32)
    vl = np.array(M.val, dtype=np.float64)
    s = _Csr()
    s.n, s.nnz = int(M.n), int(rp[-1])
    s.row_ptr = rp.ctypes.data_as(C.POINTER(C.c_int64))
    s.col = cl.ctypes.data_as(C.POINTER(C.c_int32))
    s.val = vl.ctypes.data_as(C.POINTER(C.c_double))
    st = _Alg1()
    _check(lib.orc_alg1_filter(C.byref(s), float(eps_g), float(e_r), int(max_iter), C.byref(st)), "alg1_filter")
    nnz = int(s.nnz)
    return CSR(int(M.n), rp.copy(), cl[:nnz].copy(), vl[:nnz].copy()), _alg1_dict(st)


def fnt_thresholds(coeffs, m: int, s: int, eps: float, z):
    """zeta_k (k = 0..q, entries < 2 unused) and sigma_j (j = 0..b-1) of eq. 28."""
    lib = _load()
    sc = schedule(m, s)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    zz = np.ascontiguousarray(z, dtype=np.float64)
    if zz.size < sc["q"] * (sc["b"] - 1) + 1 or zz.size < sc["q"] + 1:
        raise ValueError("need z[t] for t = 0..max(q, q(b-1))")
    zeta = np.zeros(sc["q"] + 1)
    sigma = np.zeros(sc["b"] + 1)
    _check(lib.orc_fnt_thresholds(c.ctypes.data_as(C.POINTER(C.c_double)), int(m), int(s), float(eps),
                                  zz.ctypes.data_as(C.POINTER(C.c_double)),
                                  zeta.ctypes.data_as(C.POINTER(C.c_double)),
                                  sigma.ctypes.data_as(C.POINTER(C.c_double))), "fnt_thresholds")
    return zeta, sigma[: sc["b"]]


def filtered_ps_adaptive(Z, coeffs, m: int, s: int, eps: float, e_r: float, z, nthreads: int = 0):
    """Filtered PS with Algorithm 1 and the eq. 28 thresholds.  Returns
    (F, stage records, Algorithm 1 records of the filtered stages)."""
    lib = _load()
    keep = []
    zv = _view(Z, keep)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    zz = np.ascontiguousarray(z, dtype=np.float64)
    max_stats = 4 * (m + 4) + 8
    stats = (_Stats * max_stats)()
    a1 = (_Alg1 * max_stats)()
    ns, na = C.c_int(), C.c_int()
    out = _Csr()
    _check(lib.orc_filtered_ps_adaptive(C.byref(zv), c.ctypes.data_as(C.POINTER(C.c_double)), int(m), int(s),
                                        float(eps), float(e_r), zz.ctypes.data_as(C.POINTER(C.c_double)),
                                        C.byref(out), stats, max_stats, C.byref(ns), a1, max_stats, C.byref(na),
                                        int(nthreads)), "filtered_ps_adaptive")
    return (_take(out), [_stats_dict(stats[i]) for i in range(min(ns.value, max_stats))],
            [_alg1_dict(a1[i]) for i in range(min(na.value, max_stats))])


# ---- series mode (Section 3.2, Algorithm 2 steps 1-3) ------------------------

def normest1_power(Z, p: int) -> dict:
    """Estimate of ||Z^p||_1 (Higham-Tisseur estimator, one column, itmax 5):
    {"est", "ind" (unit vector attaining it, -1: the start vector), "iters"}."""
    lib = _load()
    keep = []
    zv = _view(Z, keep)
    est, ind, it = C.c_double(), C.c_int64(), C.c_int()
    _check(lib.orc_normest1_power(C.byref(zv), int(p), C.byref(est), C.byref(ind), C.byref(it)), "normest1_power")
    return {"est": est.value, "ind": ind.value, "iters": it.value}


def power_norm_bounds(Z, tmax: int, K: int = 10) -> np.ndarray:
    """z[0..tmax] of eq. 37 (estimates up to K, Lemma 1 beyond)."""
    lib = _load()
    keep = []
    zv = _view(Z, keep)
    z = np.zeros(tmax + 1)
    _check(lib.orc_power_norm_bounds(C.byref(zv), int(K), int(tmax), z.ctypes.data_as(C.POINTER(C.c_double))),
           "power_norm_bounds")
    return z


def series_degree(a, z, eps_tol: float) -> dict:
    """N of eq. 34, q of Algorithm 2 step 3 and the tail T_N, for the series
    given by its coefficients a[0..L-1] and the bounds z[0..L-1]."""
    lib = _load()
    aa = np.ascontiguousarray(a, dtype=np.float64)
    zz = np.ascontiguousarray(z, dtype=np.float64)
    if zz.size < aa.size:
        raise ValueError("need z[i] for every coefficient")
    N, q, tail = C.c_int(), C.c_int(), C.c_double()
    _check(lib.orc_series_degree(aa.ctypes.data_as(C.POINTER(C.c_double)), int(aa.size),
                                 zz.ctypes.data_as(C.POINTER(C.c_double)), float(eps_tol), C.byref(N), C.byref(q),
                                 C.byref(tail)), "series_degree")
    return {"N": N.value, "q": q.value, "tail": tail.value}


def series(Z, a, eps_tol: float, e_r: float, K: int = 10, nthreads: int = 0):
    """Algorithm 2 for a power series: z by eq. 37, N by eq. 34, q by step 3,
    then the filtered PS of P_N with Algorithm 1 and the thresholds of eq. 36
    (those of eq. 28 with the budget eps_tol - T_N).  Returns
    (F, info, stage records, Algorithm 1 records)."""
    L = len(a)
    z = power_norm_bounds(Z, L - 1, K)
    d = series_degree(a, z, eps_tol)
    N, q = d["N"], d["q"]
    budget = eps_tol - d["tail"]
    F, stats, a1 = filtered_ps_adaptive(Z, np.asarray(a[:N], dtype=np.float64), N - 1, q, budget, e_r, z,
                                        nthreads)
    info = dict(d, z=z, budget=budget, m=N - 1, s=q)
    return F, info, stats, a1
