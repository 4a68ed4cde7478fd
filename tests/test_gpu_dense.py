"""The dense path (FPS_FLAG_DENSE): products whose work has gone dense run
as FP64 matrix-core products with the block added and the filter applied in
their write-out.  The sums run in the matrix cores' order, so results are
compared with the oracle within the relative Frobenius tolerance 1e-10 (not
bit for bit), and the eq. 23 bound must still hold; repeated evaluations of
one plan are bit-identical to each other."""

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
