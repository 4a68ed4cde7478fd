"""The 3D configuration at its full size (50^3 grid plus random long-range
links, n = 125,000) on the GPU, stage by stage: its Horner steps are beyond
any CPU oracle (about 1e14 multiply-adds each), but its filtered powers are
not.  P_2 = D(Z Z) and P_3 = D(Z P_2) are compared with the oracle element by
element, and P_4 = D(Z P_3) on 1000 sampled rows, which the oracle computes
from its own P_3 (rows of P_4 hold about 5,400 entries: the device-memory
kernel at full scale)."""

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
