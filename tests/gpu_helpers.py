"""Helpers shared by the GPU tests: upload inputs, run the HIP path, fetch
results, compare with the oracle element by element."""

from __future__ import annotations

import numpy as np

from fps_inputs.generators import CSR


def upload(M: CSR):
    from paper_2208_05683_amd import api

    return api.to_device(M.row_ptr, M.col, M.val)


def download(t) -> CSR:
    rp, cl, vl = (x.cpu().numpy() for x in t)
    return CSR(len(rp) - 1, rp.astype(np.int64), cl.astype(np.int32), vl.astype(np.float64))


def gpu_filtered_ps(Z: CSR, coeffs, m, s, tau, flags=0, evals=1):
    from paper_2208_05683_amd import api

    plan = api.Plan(upload(Z), coeffs, m, s, tau, flags)
    try:
        outs = []
        for _ in range(evals):
            plan.eval()
            outs.append(download(plan.result()))
        return outs if evals > 1 else outs[0], plan.stats()
    finally:
        plan.close()


def assert_same_csr(got: CSR, want: CSR, what=""):
    """Bit-for-bit equality of two canonical CSR matrices."""
    assert got.n == want.n, what
    np.testing.assert_array_equal(got.row_ptr, want.row_ptr, err_msg=f"{what}: row pointers differ")
    np.testing.assert_array_equal(got.col, want.col, err_msg=f"{what}: columns differ")
    same = got.val.view(np.uint64) == want.val.view(np.uint64)
    if not np.all(same):
        i = int(np.argmin(same))
        raise AssertionError(f"{what}: {int((~same).sum())} values differ, first at {i}: "
                             f"{got.val[i]!r} vs {want.val[i]!r}")


def rel_fro_csr(got: CSR, want: CSR) -> float:
    g = got.to_scipy()
    w = want.to_scipy()
    d = (g - w)
    num = float(np.sqrt((d.multiply(d)).sum()))
    den = float(np.sqrt((w.multiply(w)).sum()))
    return num / den if den else num


def check_canonical(M: CSR, tau_filtered: float | None = None):
    assert M.row_ptr[0] == 0 and M.row_ptr[-1] == M.col.size == M.val.size
    d = np.diff(M.row_ptr)
    assert np.all(d >= 0)
    rows = np.repeat(np.arange(M.n), d)
    if M.col.size:
        assert M.col.min() >= 0 and M.col.max() < M.n
        same_row = rows[1:] == rows[:-1]
        assert np.all(M.col[1:][same_row] > M.col[:-1][same_row])
    assert np.all(M.val != 0)
    if tau_filtered:
        assert np.all(np.abs(M.val) >= tau_filtered)
