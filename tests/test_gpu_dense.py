"""The dense paths.  FPS_FLAG_DENSE: products whose work has gone dense run
as FP64 matrix-core products with the block added and the filter applied in
their write-out.  The sums run in the matrix cores' order, so results are
compared with the oracle within the relative Frobenius tolerance 1e-10 (not
bit for bit), and the eq. 23 bound must still hold; repeated evaluations of
one plan are bit-identical to each other.  FPS_FLAG_DENSE_EXACT: products
whose work has gone dense run as sparse rows times dense rows or as a dense
product on the vector units with each entry's sum in k order, each entry
the sparse path's fma chain with exact zeros added, so results are compared
with the oracle bit for bit."""

import numpy as np
import pytest

import oracle as O
from oracle.bound import filtering_bound, power_norms, rounding_slack
from fps_inputs import generators as G

from gpu_helpers import check_canonical, download, rel_fro_csr, upload

pytestmark = pytest.mark.gpu

REL_TOL = 1e-10


def _dense_plan_evals(Z, c, m, s, tau, evals=2):
    from paper_2208_05683_amd import api, binding as B

    plan = api.Plan(upload(Z), c, m, s, tau, B.FPS_FLAG_DENSE)
    try:
        outs = []
        for _ in range(evals):
            plan.eval()
            outs.append(download(plan.result()))
        return outs, plan.stats()
    finally:
        plan.close()


@pytest.mark.parametrize("side", [10, 12, 14])
def test_lap3d_dense_path_within_tolerance(side):
    cfg = G.config3(side=side)
    Z, c, m, s, tau = cfg["Z"], cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"]
    want, st = O.filtered_ps(Z, c, m, s, tau)
    outs, gst = _dense_plan_evals(Z, c, m, s, tau)
    assert any(gst["stage_dense"]), gst["stage_dense"]
    for got in outs:
        check_canonical(got, tau)
        assert rel_fro_csr(got, want) <= REL_TOL
    # the evaluations of one plan agree bit for bit (a fixed order of sums)
    assert np.array_equal(outs[0].val.view(np.uint64), outs[1].val.view(np.uint64))
    assert np.array_equal(outs[0].col, outs[1].col)


def test_lap3d_dense_path_within_eq23_bound():
    # the filtered result (dense path) against the unfiltered polynomial, in
    # the 1-norm: within the bound of eq. 23 from the oracle's dropped norms
    cfg = G.config3(side=8)
    Z, c, m, s, tau = cfg["Z"], cfg["coeffs"], cfg["m"], cfg["s"], 1e-9
    want, st = O.filtered_ps(Z, c, m, s, tau)
    F0, _ = O.unfiltered_ps(Z, c, m, s)
    (got,), gst = _dense_plan_evals(Z, c, m, s, tau, evals=1)
    assert any(gst["stage_dense"])
    sc = O.schedule(m, s)
    z = power_norms(Z, max(sc["q"], sc["q"] * (sc["b"] - 1)))
    bd = filtering_bound(c, m, s, st, z)["bound"]
    err = O.norm1(got.to_dense() - F0.to_dense())
    assert err <= bd * (1 + 1e-3) + rounding_slack(c, m, float(z[1])) + 2 * Z.n * tau, (err, bd)


@pytest.mark.parametrize("bw", [12, 15])
def test_banded_unfiltered_dense_vs_oracle(bw):
    # tau = 0 (the unfiltered scheme): only rounding separates the two orders
    Z = G.banded_sweep_matrix(bw, 1000, seed=1000 * bw)
    Z = G.CSR(Z.n, Z.row_ptr, Z.col, Z.val / (4.0 * bw))
    c = G.exp_coeffs(30)
    want, _ = O.filtered_ps(Z, c, 30, 6, 0.0)
    (got,), gst = _dense_plan_evals(Z, c, 30, 6, 0.0, evals=1)
    assert any(gst["stage_dense"])
    assert rel_fro_csr(got, want) <= 1e-13


@pytest.mark.parametrize("bw,fn", [(12, "exp"), (13, "cos"), (15, "exp")])
def test_banded_series_mode_dense_within_tolerance(bw, fn):
    # the paper's second test set in series mode (Algorithm 2, eps_tol 1e-14)
    from paper_2208_05683_amd import api, binding as B

    Z = G.banded_sweep_matrix(bw, 1000, seed=1000 * bw + 1)
    a = G.exp_coeffs(199) if fn == "exp" else G.cos_coeffs(199)
    want, info, st, a1 = O.series(Z, a, 1e-14, 0.1)
    plan = api.Plan.series(upload(Z), a, 1e-14, 0.1, flags=B.FPS_FLAG_DENSE)
    try:
        for _ in range(2):
            plan.eval()
            got = download(plan.result())
            gst = plan.stats()
            check_canonical(got)
            assert any(gst["stage_dense"])
            assert rel_fro_csr(got, want) <= REL_TOL
    finally:
        plan.close()


# ---------------------------------------------------------------------------
# the exact dense paths (FPS_FLAG_DENSE_EXACT): bit for bit
# ---------------------------------------------------------------------------

def _rows_plan_evals(Z, c, m, s, tau, evals=2):
    from paper_2208_05683_amd import api, binding as B

    plan = api.Plan(upload(Z), c, m, s, tau, B.FPS_FLAG_DENSE_EXACT)
    try:
        outs = []
        for _ in range(evals):
            plan.eval()
            outs.append(download(plan.result()))
        return outs, plan.stats()
    finally:
        plan.close()


@pytest.mark.parametrize("side", [12, 14])
def test_lap3d_dense_rows_bitwise(side):
    # the powers whose rows have filled in run as Z times dense rows of
    # P_j, the last Horner steps as ordered dense products: every entry is
    # the sparse path's fma chain (plus exact zeros)
    from gpu_helpers import assert_same_csr

    cfg = G.config3(side=side)
    Z, c, m, s, tau = cfg["Z"], cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"]
    want, _ = O.filtered_ps(Z, c, m, s, tau)
    outs, gst = _rows_plan_evals(Z, c, m, s, tau)
    assert 2 in gst["stage_dense"] and 1 not in gst["stage_dense"], gst["stage_dense"]
    for i, got in enumerate(outs):
        check_canonical(got, tau)
        assert_same_csr(got, want, f"3d {side}^3 dense rows, evaluation {i}")


def test_dense_rows_horner_with_block_bitwise():
    # q = 2: P_2 stays sparse while S fills in, so the Horner steps (with
    # their fused coefficient blocks) run as P_2 times dense rows of S
    from gpu_helpers import assert_same_csr

    cfg = G.config3(side=12)
    Z, c, m, s, tau = cfg["Z"], G.cos_coeffs(12), 12, 2, 1e-12
    want, _ = O.filtered_ps(Z, c, m, s, tau)
    outs, gst = _rows_plan_evals(Z, c, m, s, tau)
    horner = [d for d, k in zip(gst["stage_dense"], gst["kind"]) if k == 3]
    assert 2 in horner or 3 in horner, (gst["stage_dense"], gst["kind"])
    for i, got in enumerate(outs):
        check_canonical(got, tau)
        assert_same_csr(got, want, f"q = 2 dense rows, evaluation {i}")


@pytest.mark.parametrize("bw", [11, 15])
def test_banded_series_mode_exact_dense_bitwise(bw):
    # n = 1000 (ld = 1024: the smallest block tiles, 32 x 32) on the exact
    # dense paths in series mode: the oracle's result bit for bit
    from paper_2208_05683_amd import api, binding as B
    from gpu_helpers import assert_same_csr

    Z = G.banded_sweep_matrix(bw, 1000, seed=1000 * bw + 2)
    a = G.exp_coeffs(199)
    want, info, st, a1 = O.series(Z, a, 1e-14, 0.1)
    plan = api.Plan.series(upload(Z), a, 1e-14, 0.1, flags=B.FPS_FLAG_DENSE_EXACT)
    try:
        for e in range(2):
            plan.eval()
            got = download(plan.result())
            gst = plan.stats()
            assert 3 in gst["stage_dense"], gst["stage_dense"]
            if e > 0:  # Algorithm 1's first sums taken by the dense write-out
                modes = [m for m, d in zip(gst["stage_alg1_mode"], gst["stage_dense"]) if d]
                assert modes and all(m == 1 for m in modes), (gst["stage_alg1_mode"], gst["stage_dense"])
            check_canonical(got)
            assert_same_csr(got, want, f"banded b = {bw}, exact dense paths, evaluation {e}")
    finally:
        plan.close()


def test_lap3d_side20_dense_rows_against_stored_digest():
    # n = 8000 on the exact dense paths: the oracle's digest, bit for bit
    import hashlib
    import json
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lap3d_side20_cos_m24_s5.json")
    with open(path) as f:
        ref = json.load(f)
    cfg = G.config3(side=20)
    Z, c, m, s, tau = cfg["Z"], cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"]
    (got,), gst = _rows_plan_evals(Z, c, m, s, tau, evals=1)
    # the fifth power as dense rows, the last two Horner steps ordered on the vector units
    assert 2 in gst["stage_dense"] and 3 in gst["stage_dense"], gst["stage_dense"]
    assert got.nnz == ref["nnz"]
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(got.row_ptr, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(got.col, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(got.val, dtype="<f8").tobytes())
    assert h.hexdigest() == ref["sha256"]
