"""The 3D configuration: at its full size (50^3 grid plus random long-range
links, n = 125,000) on the GPU, stage by stage: its Horner steps are beyond
any CPU oracle (about 1e14 multiply-adds each), but its filtered powers are
not.  P_2 = D(Z Z) and P_3 = D(Z P_2) are compared with the oracle element by
element, and P_4 = D(Z P_3) on 1000 sampled rows, which the oracle computes
from its own P_3 (rows of P_4 hold about 5,400 entries: the device-memory
kernel at full scale).  End to end (every Horner step and F) it is compared
bit for bit on 12^3 and 14^3 grids, with the oracle run inside the test, and
on a 20^3 grid (n = 8000) against a stored digest of the oracle's result."""

import numpy as np
import pytest

import oracle as O
from fps_inputs import generators as G

from gpu_helpers import assert_same_csr, check_canonical, download

pytestmark = pytest.mark.gpu


def _rows_only(M, rows):
    """M with every row outside `rows` emptied (same dimension)."""
    cnt = np.zeros(M.n, np.int64)
    cnt[rows] = np.diff(M.row_ptr)[rows]
    rp = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    sel = np.concatenate([np.arange(M.row_ptr[r], M.row_ptr[r + 1]) for r in rows]).astype(np.int64)
    return G.CSR(M.n, rp, M.col[sel].copy(), M.val[sel].copy())


def _device_rows(t, rows):
    """Rows `rows` of a device CSR triple, as a host CSR of the same dimension."""
    import torch

    rp = t[0].cpu().numpy()
    lens = rp[rows + 1] - rp[rows]
    idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows]).astype(np.int64)
    it = torch.from_numpy(idx).to(t[1].device)
    col = t[1].index_select(0, it).cpu().numpy().astype(np.int32)
    val = t[2].index_select(0, it).cpu().numpy().astype(np.float64)
    cnt = np.zeros(len(rp) - 1, np.int64)
    cnt[rows] = lens
    return G.CSR(len(rp) - 1, np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64), col, val)


def test_lap3d_full_size_powers():
    from paper_2208_05683_amd import api

    cfg = G.config3()
    Z, tau = cfg["Z"], cfg["tau"]
    assert Z.n == 125000
    # oracle: P_2, P_3 in full, P_4 on the sampled rows from its own P_3
    P2, _ = O.spgemm(Z, Z, None, tau)
    P3, _ = O.spgemm(Z, P2, None, tau)
    rows = np.sort(np.random.default_rng(7).choice(Z.n, 1000, replace=False))
    P4s, _ = O.spgemm(_rows_only(Z, rows), P3, None, tau)

    Zd = api.to_device(Z.row_ptr, Z.col, Z.val)
    g2 = api.spgemm(Zd, Zd, None, tau)
    got2 = download(g2)
    check_canonical(got2)
    assert_same_csr(got2, P2, "P_2 at 50^3")
    g3 = api.spgemm(Zd, g2, None, tau)
    del g2
    got3 = download(g3)
    assert_same_csr(got3, P3, "P_3 at 50^3")
    del got3
    g4 = api.spgemm(Zd, g3, None, tau)
    del g3
    got4 = _device_rows(g4, rows)
    assert_same_csr(got4, P4s, "P_4 at 50^3, sampled rows")
    assert np.diff(P4s.row_ptr)[rows].mean() > 448  # beyond both shared-memory tiers


# ---------------------------------------------------------------------------
# the 3D workload end to end on smaller grids (its rows fill in to dense)
# ---------------------------------------------------------------------------

def _sparse_path_flags():
    """Flags that keep every stage on the ordered sparse path (the bitwise one)."""
    from paper_2208_05683_amd import binding as B

    return getattr(B, "FPS_FLAG_NO_DENSE", 0)


@pytest.mark.parametrize("side", [12, 14])
def test_lap3d_end_to_end_bitwise(side):
    # every Horner step and F, against the oracle computed here
    from gpu_helpers import gpu_filtered_ps

    cfg = G.config3(side=side)
    Z, c, m, s, tau = cfg["Z"], cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"]
    want, st = O.filtered_ps(Z, c, m, s, tau)
    outs, gst = gpu_filtered_ps(Z, c, m, s, tau, flags=_sparse_path_flags(), evals=2)
    for i, got in enumerate(outs):
        check_canonical(got)
        assert_same_csr(got, want, f"3d {side}^3 eval {i}")
    assert want.nnz > 0.9 * Z.n * Z.n  # F is dense
    assert gst["rows_global"] > 0


def test_lap3d_side20_against_stored_digest():
    # n = 8000: the oracle takes minutes, so its result is stored as a digest
    # written by tests/golden/make_lap3d_digest.py (which calls only the oracle)
    import hashlib
    import json
    import os

    from gpu_helpers import gpu_filtered_ps

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lap3d_side20_cos_m24_s5.json")
    with open(path) as f:
        ref = json.load(f)
    cfg = G.config3(side=20)
    Z, c, m, s, tau = cfg["Z"], cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"]
    assert Z.n == ref["n"] == 8000
    got, gst = gpu_filtered_ps(Z, c, m, s, tau, flags=_sparse_path_flags())
    check_canonical(got)
    assert got.nnz == ref["nnz"]
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(got.row_ptr, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(got.col, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(got.val, dtype="<f8").tobytes())
    assert h.hexdigest() == ref["sha256"]
