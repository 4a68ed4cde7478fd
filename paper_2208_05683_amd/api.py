"""Torch-facing convenience layer over the C ABI (argument marshalling only).

    Zd = api.to_device(row_ptr, col, val)          # device tensors
    plan = api.Plan(Zd, coeffs, m=30, s=6, tau=1e-12)
    plan.eval()
    row_ptr, col, val = plan.result()              # canonical CSR of F on the device
"""

from __future__ import annotations

import numpy as np
import torch

from . import binding as B


def to_device(row_ptr, col, val, device="cuda"):
    """Host arrays (numpy or torch) of a canonical CSR -> contiguous device tensors."""
    rp = torch.as_tensor(np.asarray(row_ptr, dtype=np.int64)).to(device)
    cl = torch.as_tensor(np.asarray(col, dtype=np.int32)).to(device)
    vl = torch.as_tensor(np.asarray(val, dtype=np.float64)).to(device)
    return rp.contiguous(), cl.contiguous(), vl.contiguous()


def _alloc_csr(n, nnz, device):
    return (torch.empty(n + 1, dtype=torch.int64, device=device),
            torch.empty(nnz, dtype=torch.int32, device=device),
            torch.empty(nnz, dtype=torch.float64, device=device))


class Plan:
    """A plan for F(Z) = sum_k c_k Z^k by filtered PS (fps_plan_create)."""

    def __init__(self, Z, coeffs, m: int, s: int, tau: float = 0.0, flags: int = 0, stream=None,
                 adaptive: bool = False, eps: float = 0.0, e_r: float = 0.1, znorm=None, max_alg1_iters: int = 0,
                 alg1_device_iters: int = 0):
        """Fixed filter (drop |x| < tau) by default; adaptive=True runs
        Algorithm 1 with the eq. 28 thresholds for budget eps (znorm[t] >=
        ||Z^t||_1 required)."""
        self.Z = tuple(Z)  # keep the borrowed device arrays alive
        self.n = self.Z[0].numel() - 1
        self.device = self.Z[0].device
        self.view = B.csr_view(*self.Z)
        self.handle = None
        if adaptive:
            self.handle = B.fps_plan_create_ex(self.view, list(coeffs), m, s, filter=B.FPS_FILTER_ADAPTIVE,
                                               eps=eps, e_r=e_r, znorm=list(znorm) if znorm is not None else None,
                                               max_alg1_iters=max_alg1_iters, flags=flags, stream=stream,
                                               alg1_device_iters=alg1_device_iters)
        else:
            self.handle = B.fps_plan_create(self.view, list(coeffs), m, s, tau, flags, stream)

    @classmethod
    def series(cls, Z, a, eps_tol: float, e_r: float = 0.1, K: int = 10, max_alg1_iters: int = 0, flags: int = 0,
               stream=None, alg1_device_iters: int = 0):
        """Series mode (Algorithm 2): the plan picks N, q and the eq. 36
        thresholds from the norm estimates of eq. 37 so that
        ||f(Z) - F||_1 <= eps_tol; a holds the first coefficients of f."""
        self = cls.__new__(cls)
        self.Z = tuple(Z)
        self.n = self.Z[0].numel() - 1
        self.device = self.Z[0].device
        self.view = B.csr_view(*self.Z)
        self.handle = None
        self.L = len(a)
        self.handle = B.fps_plan_create_series(self.view, list(a), eps_tol, e_r, K, max_alg1_iters, flags, stream,
                                               alg1_device_iters)
        return self

    def series_info(self) -> dict:
        return B.fps_plan_series_info(self.handle, self.L)

    def eval(self, stream=None):
        B.fps_eval(self.handle, stream)

    def nnz(self) -> int:
        return B.fps_result_nnz(self.handle)

    def result(self, stream=None):
        nnz = self.nnz()
        out = _alloc_csr(self.n, nnz, self.device)
        B.fps_result_copy(self.handle, *out, stream=stream)
        torch.cuda.current_stream(self.device).synchronize() if stream is None else stream.synchronize()
        return out

    def stats(self) -> dict:
        return B.fps_get_stats(self.handle)

    def close(self):
        if self.handle is not None:
            B.fps_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _take_matrix(h, n, device):
    try:
        nnz = B.fps_matrix_nnz(h)
        out = _alloc_csr(n, nnz, device)
        B.fps_matrix_copy(h, *out)
        torch.cuda.synchronize(device)
        return out
    finally:
        B.fps_matrix_destroy(h)


def spgemm(A, Bm, E=None, tau: float = 0.0):
    """D_tau(E + A (x) B) for canonical device CSR triples."""
    n = A[0].numel() - 1
    h = B.fps_spgemm(B.csr_view(*A), B.csr_view(*Bm), B.csr_view(*E) if E is not None else None, tau)
    return _take_matrix(h, n, A[0].device)


def axpy(n: int, coefs, terms, device="cuda"):
    """sum_t coefs[t] * terms[t] (None = identity) for canonical device CSR triples."""
    views = [None if t is None else B.csr_view(*t) for t in terms]
    h = B.fps_axpy(n, coefs, views)
    return _take_matrix(h, n, device)


def normest1(Z, p: int) -> dict:
    """Estimate of ||Z^p||_1 (device CSR triple); see fps_normest1."""
    return B.fps_normest1(B.csr_view(*Z), p)


def power_norm_bounds(Z, tmax: int, K: int = 10) -> list:
    """z[0..tmax] of eq. 37 (device CSR triple)."""
    return B.fps_power_norm_bounds(B.csr_view(*Z), K, tmax)


def schedule(m: int, s: int) -> dict:
    return B.fps_schedule(m, s)


class Batch:
    """Many filtered PS evaluations in one launch sequence (see fps_batch_create).

    items: list of dicts with Zd (device CSR triple), coeffs, m, tau and
    optionally s (0 or absent: autotuned in [s_lo, s_hi])."""

    def __init__(self, items, s_lo: int = 0, s_hi: int = 0, flags: int = 0, stream=None):
        self.n = [int(it["Zd"][0].numel() - 1) for it in items]
        self.device = items[0]["Zd"][0].device
        spec = [(B.csr_view(*it["Zd"]), it["coeffs"], int(it["m"]), int(it.get("s", 0)), float(it["tau"]))
                for it in items]
        self.handle = B.fps_batch_create(spec, s_lo, s_hi, flags, stream)

    def eval(self, stream=None):
        B.fps_batch_eval(self.handle, stream)

    def nnz(self, i: int) -> int:
        return B.fps_batch_result_nnz(self.handle, i)

    def result(self, i: int, stream=None):
        out = _alloc_csr(self.n[i], self.nnz(i), self.device)
        B.fps_batch_result_copy(self.handle, i, *out, stream=stream)
        torch.cuda.current_stream(self.device).synchronize() if stream is None else stream.synchronize()
        return out

    def item_info(self, i: int, candidates: int = 0) -> dict:
        return B.fps_batch_item_info(self.handle, i, candidates)

    def stats(self) -> dict:
        return B.fps_batch_get_stats(self.handle)

    def close(self):
        if self.handle is not None:
            B.fps_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass



class Server:
    """Continuous admission of evaluations by device-memory footprint (see
    fps_server_create).  submit() returns a ticket; wait(), result() and
    release() act on it."""

    def __init__(self, slots: int, hbm_budget: int, max_queue: int = 0, flags: int = 0, fake_backend: bool = False,
                 no_grow: bool = False):
        self.handle = B.fps_server_create(slots, hbm_budget, max_queue, flags, fake_backend, no_grow)
        self._n = {}
        self._dev = {}

    def submit(self, Zd, coeffs, m: int, tau: float, s: int = 0, reserve_hint: int = 0) -> int:
        t = B.fps_server_submit(self.handle, B.csr_view(*Zd), coeffs, m, s, tau, reserve_hint)
        self._n[t] = int(Zd[0].numel() - 1)
        self._dev[t] = Zd[0].device
        return t

    def wait(self, ticket: int, timeout_ms: int = -1) -> int:
        return B.fps_server_wait(self.handle, ticket, timeout_ms)

    def result(self, ticket: int, stream=None):
        nnz = B.fps_server_result_nnz(self.handle, ticket)
        out = _alloc_csr(self._n[ticket], nnz, self._dev[ticket])
        B.fps_server_result_copy(self.handle, ticket, *out, stream=stream)
        torch.cuda.current_stream(self._dev[ticket]).synchronize() if stream is None else stream.synchronize()
        return out

    def info(self, ticket: int) -> dict:
        return B.fps_server_request_info(self.handle, ticket)

    def release(self, ticket: int):
        B.fps_server_release(self.handle, ticket)
        self._n.pop(ticket, None)
        self._dev.pop(ticket, None)

    def stats(self) -> dict:
        return B.fps_server_get_stats(self.handle)

    def close(self):
        if self.handle is not None:
            B.fps_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
