"""ctypes binding of libfps (include/fps.h), names as in the C ABI.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libfps.so.  PyTorch supplies device memory (CUDA/HIP tensors) and
stream handles.  If the library is not built, importing this module raises
ImportError: there is no fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfps.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "fps.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2208_05683_amd.build` "
        "(hipcc, gfx950); there is no non-HIP implementation")

# torch first: it loads its own HIP runtime, whose soname (libamdhip64.so.7)
# then satisfies libfps.so's dependency, so the process holds one HIP runtime.
# Loading libfps.so first would pull in the system runtime as well, and the
# library's calls would then run on a second runtime that finds no device.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)


def _header_constants():
    out = {}
    with open(HEADER) as f:
        for line in f:
            m = re.match(r"#define\s+(FPS_\w+)\s+(0x[0-9a-fA-F]+|\d+)(ull)?\b", line)
            if m:
                out[m.group(1)] = int(m.group(2), 0)
    return out


_consts = _header_constants()
globals().update(_consts)

FPS_MAX_STAGES = _consts["FPS_MAX_STAGES"]


class fps_csr_view(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("nnz", C.c_int64),
        ("row_ptr", C.c_void_p),
        ("col", C.c_void_p),
        ("val", C.c_void_p),
    ]


class fps_stats(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("q", C.c_int32), ("b", C.c_int32), ("g", C.c_int32), ("J", C.c_int32),
        ("start", C.c_int32), ("n_spgemm", C.c_int32), ("n_stages", C.c_int32),
        ("evals", C.c_int64), ("nnz_out", C.c_int64), ("products", C.c_int64),
        ("products_skipped", C.c_int64), ("rows_skipped", C.c_int64), ("rows_global", C.c_int64),
        ("rows_wide", C.c_int64), ("resizes", C.c_int64), ("bytes_algorithmic", C.c_double), ("numeric_ms", C.c_double),
        ("numeric_launches", C.c_int32),
        ("kind", C.c_int32 * FPS_MAX_STAGES), ("index", C.c_int32 * FPS_MAX_STAGES),
        ("stage_products", C.c_int64 * FPS_MAX_STAGES), ("stage_nnz", C.c_int64 * FPS_MAX_STAGES),
        ("stage_ms", C.c_double * FPS_MAX_STAGES),
        ("stage_eps_g", C.c_double * FPS_MAX_STAGES),
        ("stage_threshold", C.c_double * FPS_MAX_STAGES),
        ("stage_dropped", C.c_double * FPS_MAX_STAGES),
        ("stage_alg1_iters", C.c_int32 * FPS_MAX_STAGES),
        ("stage_n_dropped", C.c_int64 * FPS_MAX_STAGES),
        ("stage_dropped_max", C.c_double * FPS_MAX_STAGES),
        ("stage_alg1_mode", C.c_int32 * FPS_MAX_STAGES),
        ("stage_rows_skipped", C.c_int64 * FPS_MAX_STAGES),
        ("stage_bytes", C.c_double * FPS_MAX_STAGES),
        ("stage_dense", C.c_int32 * FPS_MAX_STAGES),
        ("dense_ld", C.c_int64),
        ("stage_small", C.c_int32 * FPS_MAX_STAGES),
        ("stage_max_ns", C.c_int64 * FPS_MAX_STAGES),
        ("stage_max_words", C.c_int64 * FPS_MAX_STAGES),
    ]


class fps_filter_opts(C.Structure):
    _fields_ = [
        ("filter", C.c_int32),
        ("max_alg1_iters", C.c_int32),
        ("tau", C.c_double),
        ("eps", C.c_double),
        ("e_r", C.c_double),
        ("znorm", C.POINTER(C.c_double)),
        ("alg1_device_iters", C.c_int32),
        ("reserved", C.c_int32),
    ]


class fps_series_opts(C.Structure):
    _fields_ = [
        ("eps_tol", C.c_double),
        ("e_r", C.c_double),
        ("K", C.c_int32),
        ("max_alg1_iters", C.c_int32),
        ("alg1_device_iters", C.c_int32),
        ("reserved", C.c_int32),
    ]


class fps_batch_item(C.Structure):
    _fields_ = [
        ("Z", fps_csr_view),
        ("coeffs", C.POINTER(C.c_double)),
        ("m", C.c_int32),
        ("s", C.c_int32),
        ("tau", C.c_double),
    ]


class fps_batch_stats(C.Structure):
    _fields_ = [
        ("count", C.c_int32), ("groups", C.c_int32), ("graph", C.c_int32), ("reserved", C.c_int32),
        ("evals", C.c_int64), ("graph_launches", C.c_int64), ("resizes", C.c_int64), ("rows", C.c_int64),
        ("nnz_out", C.c_int64), ("products", C.c_int64), ("bytes_algorithmic", C.c_double),
    ]


class fps_server_opts(C.Structure):
    _fields_ = [("slots", C.c_int32), ("max_queue", C.c_int32), ("hbm_budget", C.c_int64), ("flags", C.c_uint64),
                ("fake_backend", C.c_int32), ("no_grow", C.c_int32)]


class fps_server_request(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("attempts", C.c_int32), ("s", C.c_int32),
                ("n", C.c_int64), ("reserve", C.c_int64), ("held", C.c_int64), ("peak", C.c_int64),
                ("t_submit_ns", C.c_int64), ("t_start_ns", C.c_int64), ("t_done_ns", C.c_int64)]


class fps_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64), ("retries", C.c_int64),
                ("refused", C.c_int64), ("running", C.c_int32), ("queued", C.c_int32), ("slots", C.c_int32),
                ("peak_running", C.c_int32), ("reserved", C.c_int64), ("peak_reserved", C.c_int64),
                ("budget", C.c_int64), ("grows", C.c_int64)]


_P = C.POINTER
_vp = C.c_void_p
_SIGS = {
    "fps_abi_version": (C.c_int32, []),
    "fps_status_string": (C.c_char_p, [C.c_int32]),
    "fps_last_error": (C.c_char_p, []),
    "fps_schedule": (C.c_int32, [C.c_int32, C.c_int32] + [_P(C.c_int32)] * 7),
    "fps_plan_create": (C.c_int32, [_P(_vp), _P(fps_csr_view), _P(C.c_double), C.c_int32, C.c_int32,
                                    C.c_double, C.c_uint64, _vp]),
    "fps_plan_create_ex": (C.c_int32, [_P(_vp), _P(fps_csr_view), _P(C.c_double), C.c_int32, C.c_int32,
                                       _P(fps_filter_opts), C.c_uint64, _vp]),
    "fps_eval": (C.c_int32, [_vp, _vp]),
    "fps_result_nnz": (C.c_int32, [_vp, _P(C.c_int64)]),
    "fps_result_copy": (C.c_int32, [_vp, _vp, _vp, _vp, _vp]),
    "fps_get_stats": (C.c_int32, [_vp, _P(fps_stats)]),
    "fps_plan_destroy": (None, [_vp]),
    "fps_spgemm": (C.c_int32, [_P(_vp), _P(fps_csr_view), _P(fps_csr_view), _P(fps_csr_view), C.c_double, _vp]),
    "fps_axpy": (C.c_int32, [_P(_vp), C.c_int64, C.c_int32, _P(C.c_double), _P(fps_csr_view), _vp]),
    "fps_matrix_nnz": (C.c_int32, [_vp, _P(C.c_int64)]),
    "fps_matrix_copy": (C.c_int32, [_vp, _vp, _vp, _vp, _vp]),
    "fps_matrix_destroy": (None, [_vp]),
    "fps_normest1": (C.c_int32, [_P(fps_csr_view), C.c_int32, _P(C.c_double), _P(C.c_int64), _P(C.c_int32),
                                 C.c_uint64, _vp]),
    "fps_normest1_noalloc": (C.c_int32, [_P(fps_csr_view), C.c_int32, _P(C.c_double), _P(C.c_int64),
                                         _P(C.c_int32), C.c_uint64, _vp]),
    "fps_power_norm_bounds": (C.c_int32, [_P(fps_csr_view), C.c_int32, C.c_int32, _P(C.c_double), C.c_uint64, _vp]),
    "fps_batch_create": (C.c_int32, [_P(_vp), _P(fps_batch_item), C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                     _vp]),
    "fps_batch_eval": (C.c_int32, [_vp, _vp]),
    "fps_batch_result_nnz": (C.c_int32, [_vp, C.c_int32, _P(C.c_int64)]),
    "fps_batch_result_copy": (C.c_int32, [_vp, C.c_int32, _vp, _vp, _vp, _vp]),
    "fps_batch_get_stats": (C.c_int32, [_vp, _P(fps_batch_stats)]),
    "fps_batch_item_info": (C.c_int32, [_vp, C.c_int32, _P(C.c_int32), _P(C.c_int32), _P(C.c_int64)]),
    "fps_batch_destroy": (None, [_vp]),
    "fps_server_create": (C.c_int32, [_P(_vp), _P(fps_server_opts)]),
    "fps_server_submit": (C.c_int32, [_vp, _P(fps_csr_view), _P(C.c_double), C.c_int32, C.c_int32, C.c_double,
                                      C.c_int64, _P(C.c_int64)]),
    "fps_server_wait": (C.c_int32, [_vp, C.c_int64, C.c_int64, _P(C.c_int32)]),
    "fps_server_result_nnz": (C.c_int32, [_vp, C.c_int64, _P(C.c_int64)]),
    "fps_server_result_copy": (C.c_int32, [_vp, C.c_int64, _vp, _vp, _vp, _vp]),
    "fps_server_release": (C.c_int32, [_vp, C.c_int64]),
    "fps_server_request_info": (C.c_int32, [_vp, C.c_int64, _P(fps_server_request)]),
    "fps_server_get_stats": (C.c_int32, [_vp, _P(fps_server_stats)]),
    "fps_server_destroy": (None, [_vp]),
    "fps_plan_create_series": (C.c_int32, [_P(_vp), _P(fps_csr_view), _P(C.c_double), C.c_int32,
                                           _P(fps_series_opts), C.c_uint64, _vp]),
    "fps_plan_series_info": (C.c_int32, [_vp, _P(C.c_int32), _P(C.c_int32), _P(C.c_double), _P(C.c_double),
                                         _P(C.c_double)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class FpsError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.fps_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.fps_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def _check(st: int, where: str):
    if st != 0:
        raise FpsError(st, where)


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def csr_view(row_ptr, col, val) -> fps_csr_view:
    """fps_csr_view of device tensors (int64 row_ptr, int32 col, float64 val)."""
    import torch

    for t, dt, nm in ((row_ptr, torch.int64, "row_ptr"), (col, torch.int32, "col"), (val, torch.float64, "val")):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise TypeError(f"{nm} must be a contiguous {dt} device tensor")
    v = fps_csr_view()
    v.n = row_ptr.numel() - 1
    v.nnz = col.numel()
    v.row_ptr = row_ptr.data_ptr()
    v.col = col.data_ptr() if col.numel() else None
    v.val = val.data_ptr() if val.numel() else None
    return v


# ---- functions with the C ABI's names ------------------------------------------

def fps_abi_version() -> int:
    return _lib.fps_abi_version()


def fps_schedule(m: int, s: int) -> dict:
    vals = [C.c_int32() for _ in range(7)]
    _check(_lib.fps_schedule(m, s, *[C.byref(v) for v in vals]), "fps_schedule")
    return dict(zip(["N", "q", "b", "g", "J", "start", "n_spgemm"], [v.value for v in vals]))


def fps_plan_create(Z: fps_csr_view, coeffs, m: int, s: int, tau: float, flags: int = 0, stream=None):
    arr = (C.c_double * (m + 1))(*[float(x) for x in coeffs[: m + 1]])
    h = C.c_void_p()
    _check(_lib.fps_plan_create(C.byref(h), C.byref(Z), arr, m, s, float(tau), C.c_uint64(flags),
                                _stream_handle(stream)), "fps_plan_create")
    return h


def fps_plan_create_ex(Z: fps_csr_view, coeffs, m: int, s: int, filter: int = 0, tau: float = 0.0,
                       eps: float = 0.0, e_r: float = 0.0, znorm=None, max_alg1_iters: int = 0, flags: int = 0,
                       stream=None, alg1_device_iters: int = 0):
    arr = (C.c_double * (m + 1))(*[float(x) for x in coeffs[: m + 1]])
    o = fps_filter_opts()
    o.filter = int(filter)
    o.max_alg1_iters = int(max_alg1_iters)
    o.tau = float(tau)
    o.eps = float(eps)
    o.e_r = float(e_r)
    o.alg1_device_iters = int(alg1_device_iters)
    zarr = None
    if znorm is not None:
        zarr = (C.c_double * len(znorm))(*[float(x) for x in znorm])
        o.znorm = C.cast(zarr, C.POINTER(C.c_double))
    h = C.c_void_p()
    _check(_lib.fps_plan_create_ex(C.byref(h), C.byref(Z), arr, m, s, C.byref(o), C.c_uint64(flags),
                                   _stream_handle(stream)), "fps_plan_create_ex")
    return h


def fps_eval(plan, stream=None):
    _check(_lib.fps_eval(plan, _stream_handle(stream)), "fps_eval")


def fps_result_nnz(plan) -> int:
    v = C.c_int64()
    _check(_lib.fps_result_nnz(plan, C.byref(v)), "fps_result_nnz")
    return v.value


def fps_result_copy(plan, row_ptr, col, val, stream=None):
    _check(_lib.fps_result_copy(plan, row_ptr.data_ptr(), col.data_ptr() if col.numel() else None,
                                val.data_ptr() if val.numel() else None, _stream_handle(stream)),
           "fps_result_copy")


def fps_get_stats(plan) -> dict:
    st = fps_stats()
    _check(_lib.fps_get_stats(plan, C.byref(st)), "fps_get_stats")
    d = {}
    for name, _ in fps_stats._fields_:
        v = getattr(st, name)
        if isinstance(v, C.Array):
            v = list(v)[: st.n_stages]
        d[name] = v
    return d


def fps_plan_destroy(plan):
    _lib.fps_plan_destroy(plan)


def fps_spgemm(A: fps_csr_view, B: fps_csr_view, E: fps_csr_view | None, tau: float, stream=None):
    h = C.c_void_p()
    _check(_lib.fps_spgemm(C.byref(h), C.byref(A), C.byref(B), C.byref(E) if E is not None else None, float(tau),
                           _stream_handle(stream)), "fps_spgemm")
    return h


def fps_axpy(n: int, coefs, terms, stream=None):
    """terms: list of fps_csr_view or None (identity)."""
    k = len(coefs)
    arr = (C.c_double * k)(*[float(x) for x in coefs])
    views = (fps_csr_view * k)()
    for i, t in enumerate(terms):
        if t is None:
            views[i].n = n
            views[i].nnz = 0
            views[i].row_ptr = None
        else:
            views[i] = t
    h = C.c_void_p()
    _check(_lib.fps_axpy(C.byref(h), n, k, arr, views, _stream_handle(stream)), "fps_axpy")
    return h


def fps_matrix_nnz(m) -> int:
    v = C.c_int64()
    _check(_lib.fps_matrix_nnz(m, C.byref(v)), "fps_matrix_nnz")
    return v.value


def fps_matrix_copy(m, row_ptr, col, val, stream=None):
    _check(_lib.fps_matrix_copy(m, row_ptr.data_ptr(), col.data_ptr() if col.numel() else None,
                                val.data_ptr() if val.numel() else None, _stream_handle(stream)),
           "fps_matrix_copy")


def fps_matrix_destroy(m):
    _lib.fps_matrix_destroy(m)


def fps_normest1(Z: fps_csr_view, p: int, flags: int = 0, stream=None) -> dict:
    est, ind, it = C.c_double(), C.c_int64(), C.c_int32()
    _check(_lib.fps_normest1(C.byref(Z), int(p), C.byref(est), C.byref(ind), C.byref(it), C.c_uint64(flags),
                             _stream_handle(stream)), "fps_normest1")
    return {"est": est.value, "ind": ind.value, "iters": it.value}


def fps_normest1_noalloc(Z: fps_csr_view, p: int, flags: int = 0, stream=None) -> dict:
    est, ind, it = C.c_double(), C.c_int64(), C.c_int32()
    _check(_lib.fps_normest1_noalloc(C.byref(Z), int(p), C.byref(est), C.byref(ind), C.byref(it),
                                     C.c_uint64(flags), _stream_handle(stream)), "fps_normest1_noalloc")
    return {"est": est.value, "ind": ind.value, "iters": it.value}


def fps_power_norm_bounds(Z: fps_csr_view, K: int, tmax: int, flags: int = 0, stream=None):
    z = (C.c_double * (tmax + 1))()
    _check(_lib.fps_power_norm_bounds(C.byref(Z), int(K), int(tmax), z, C.c_uint64(flags), _stream_handle(stream)),
           "fps_power_norm_bounds")
    return list(z)


def fps_plan_create_series(Z: fps_csr_view, a, eps_tol: float, e_r: float = 0.1, K: int = 0,
                           max_alg1_iters: int = 0, flags: int = 0, stream=None, alg1_device_iters: int = 0):
    arr = (C.c_double * len(a))(*[float(x) for x in a])
    o = fps_series_opts()
    o.eps_tol, o.e_r, o.K, o.max_alg1_iters = float(eps_tol), float(e_r), int(K), int(max_alg1_iters)
    o.alg1_device_iters = int(alg1_device_iters)
    h = C.c_void_p()
    _check(_lib.fps_plan_create_series(C.byref(h), C.byref(Z), arr, len(a), C.byref(o), C.c_uint64(flags),
                                       _stream_handle(stream)), "fps_plan_create_series")
    return h


def fps_plan_series_info(plan, L: int) -> dict:
    N, q, tail, budget = C.c_int32(), C.c_int32(), C.c_double(), C.c_double()
    z = (C.c_double * L)()
    _check(_lib.fps_plan_series_info(plan, C.byref(N), C.byref(q), C.byref(tail), C.byref(budget), z),
           "fps_plan_series_info")
    return {"N": N.value, "q": q.value, "tail": tail.value, "budget": budget.value, "z": list(z)}


def exported_symbols():
    """Names of the functions declared in include/fps.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fps_\w+)\s*\(", text)))


def library():
    return _lib


# ---- autotuner and batch ---------------------------------------------------

def fps_batch_create(items, s_lo: int = 0, s_hi: int = 0, flags: int = 0, stream=None):
    """items: list of (fps_csr_view, coeffs, m, s, tau)."""
    arr = (fps_batch_item * len(items))()
    keep = []
    for k, (Z, coeffs, m, s, tau) in enumerate(items):
        c = (C.c_double * (m + 1))(*[float(x) for x in coeffs[: m + 1]])
        keep.append(c)
        arr[k].Z = Z
        arr[k].coeffs = C.cast(c, C.POINTER(C.c_double))
        arr[k].m = int(m)
        arr[k].s = int(s)
        arr[k].tau = float(tau)
    h = C.c_void_p()
    _check(_lib.fps_batch_create(C.byref(h), arr, len(items), int(s_lo), int(s_hi), C.c_uint64(flags),
                                 _stream_handle(stream)), "fps_batch_create")
    return h


def fps_batch_eval(b, stream=None):
    _check(_lib.fps_batch_eval(b, _stream_handle(stream)), "fps_batch_eval")


def fps_batch_result_nnz(b, i: int) -> int:
    v = C.c_int64()
    _check(_lib.fps_batch_result_nnz(b, int(i), C.byref(v)), "fps_batch_result_nnz")
    return v.value


def fps_batch_result_copy(b, i: int, row_ptr, col, val, stream=None):
    _check(_lib.fps_batch_result_copy(b, int(i), row_ptr.data_ptr(), col.data_ptr() if col.numel() else None,
                                      val.data_ptr() if val.numel() else None, _stream_handle(stream)),
           "fps_batch_result_copy")


def fps_batch_get_stats(b) -> dict:
    st = fps_batch_stats()
    _check(_lib.fps_batch_get_stats(b, C.byref(st)), "fps_batch_get_stats")
    return {name: getattr(st, name) for name, _ in fps_batch_stats._fields_}


def fps_batch_item_info(b, i: int, candidates: int = 0) -> dict:
    """candidates: s_hi - s_lo + 1 of a tuned batch (0: no product counts)."""
    s, g = C.c_int32(), C.c_int32()
    prod = (C.c_int64 * max(candidates, 1))()
    _check(_lib.fps_batch_item_info(b, int(i), C.byref(s), C.byref(g), prod if candidates else None),
           "fps_batch_item_info")
    return {"s": s.value, "group": g.value, "products": list(prod)[:candidates]}


def fps_batch_destroy(b):
    _lib.fps_batch_destroy(b)


# ---- server -------------------------------------------------------------------

def fps_server_create(slots: int, hbm_budget: int, max_queue: int = 0, flags: int = 0, fake_backend: bool = False,
                      no_grow: bool = False):
    o = fps_server_opts(int(slots), int(max_queue), int(hbm_budget), int(flags), 1 if fake_backend else 0,
                        1 if no_grow else 0)
    h = C.c_void_p()
    _check(_lib.fps_server_create(C.byref(h), C.byref(o)), "fps_server_create")
    return h


def fps_server_submit(sv, Z: fps_csr_view, coeffs, m: int, s: int, tau: float, reserve_hint: int = 0) -> int:
    arr = (C.c_double * (m + 1))(*[float(x) for x in coeffs[: m + 1]])
    t = C.c_int64()
    _check(_lib.fps_server_submit(sv, C.byref(Z), arr, int(m), int(s), float(tau), int(reserve_hint), C.byref(t)),
           "fps_server_submit")
    return t.value


def fps_server_wait(sv, ticket: int, timeout_ms: int = -1) -> int:
    st = C.c_int32()
    _check(_lib.fps_server_wait(sv, int(ticket), int(timeout_ms), C.byref(st)), "fps_server_wait")
    return st.value


def fps_server_result_nnz(sv, ticket: int) -> int:
    v = C.c_int64()
    _check(_lib.fps_server_result_nnz(sv, int(ticket), C.byref(v)), "fps_server_result_nnz")
    return v.value


def fps_server_result_copy(sv, ticket: int, row_ptr, col, val, stream=None):
    _check(_lib.fps_server_result_copy(sv, int(ticket), row_ptr.data_ptr(), col.data_ptr() if col.numel() else None,
                                       val.data_ptr() if val.numel() else None, _stream_handle(stream)),
           "fps_server_result_copy")


def fps_server_release(sv, ticket: int):
    _check(_lib.fps_server_release(sv, int(ticket)), "fps_server_release")


def fps_server_request_info(sv, ticket: int) -> dict:
    r = fps_server_request()
    _check(_lib.fps_server_request_info(sv, int(ticket), C.byref(r)), "fps_server_request_info")
    return {name: getattr(r, name) for name, _ in fps_server_request._fields_}


def fps_server_get_stats(sv) -> dict:
    st = fps_server_stats()
    _check(_lib.fps_server_get_stats(sv, C.byref(st)), "fps_server_get_stats")
    return {name: getattr(st, name) for name, _ in fps_server_stats._fields_}


def fps_server_destroy(sv):
    _lib.fps_server_destroy(sv)
