"""The small-row tier (four rows per wavefront, 16 lanes per row): after the
sizing evaluation, a stage of more than 8192 rows whose rows all fit it runs
there.  Its results
must equal the oracle's and those of the same plan kept on 64-lane
wavefronts (FPS_FLAG_NO_SMALL) bit for bit, in every evaluation, for each
kind of stage it takes: powers, coefficient sums (with the identity term and
with more than 16 terms), Horner steps with a fused block (with and without
main terms), term rows longer than 32 entries, left-operand rows of more than
16 entries, with drop statistics, and under Algorithm 1."""

import numpy as np
import pytest

import oracle as O
from fps_inputs import generators as G

from gpu_helpers import assert_same_csr, check_canonical, gpu_filtered_ps

pytestmark = pytest.mark.gpu


def _small_stages(gst):
    return [i for i, v in enumerate(gst["stage_small"]) if v]


def _run_both(Z, c, m, s, tau, flags=0, evals=3):
    from paper_2208_05683_amd import binding as B

    got, gst = gpu_filtered_ps(Z, c, m, s, tau, flags=flags, evals=evals)
    ref, rst = gpu_filtered_ps(Z, c, m, s, tau, flags=flags | B.FPS_FLAG_NO_SMALL, evals=2)
    assert not _small_stages(rst)
    assert gst["resizes"] == 0
    return got, gst, ref, rst


CASES = {
    # 1D Laplacian: every stage small, Horner steps with block and main terms
    "lap1d": lambda: (G.laplacian_1d(10000, 1.0), G.exp_coeffs(24), 24, 4, 1e-12),
    # 2D Laplacian: powers and the g-step small, late Horner steps not
    "lap2d_100": lambda: (G.laplacian_2d(100, 2.0), G.exp_coeffs(30), 30, 6, 1e-12),
    # s = 18: the g-step sums 19 terms (two chunks of terms, the identity first)
    "lap1d_s18": lambda: (G.laplacian_1d(9000, 1.0), G.cos_coeffs(36), 36, 18, 1e-13),
    # left-operand rows of 21 entries (more than one chunk of terms)
    "banded_b10": lambda: (G.random_banded(9000, 10, 0.9, 1.2, seed=5), G.exp_coeffs(12), 12, 3, 1e-10),
    # term rows of 41 entries (beyond the two loaded per lane)
    "banded_b20": lambda: (G.random_banded(9000, 20, 1.0, 1.0, seed=9), G.exp_coeffs(8), 8, 2, 1e-9),
    # sparse band (40% of the band stored): uneven row lengths and windows
    "banded_sparse": lambda: (G.random_banded(9000, 6, 0.4, 1.3, seed=21), G.cos_coeffs(16), 16, 4, 1e-11),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_small_tier_bitwise(name):
    Z, c, m, s, tau = CASES[name]()
    want, _ = O.filtered_ps(Z, c, m, s, tau)
    got, gst, ref, _ = _run_both(Z, c, m, s, tau)
    assert _small_stages(gst), (name, gst["stage_small"])
    for e, g in enumerate(got):
        check_canonical(g)
        assert_same_csr(g, want, f"{name} eval {e}")
    assert_same_csr(ref[-1], want, f"{name} on 64-lane wavefronts")


def test_small_tier_headline_stages():
    """The 2D Laplacian workload at full size (n = 40000): the five powers and
    the g-step run in the small tier from the second evaluation on."""
    cfg = G.config2()
    Z, c, m, s, tau = cfg["Z"], cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"]
    want, st = O.filtered_ps(Z, c, m, s, tau)
    got, gst, ref, _ = _run_both(Z, c, m, s, tau)
    kinds = {0: "power", 1: "block", 2: "gstep", 3: "horner"}
    small = [(kinds.get(gst["kind"][i]), gst["index"][i]) for i in _small_stages(gst)]
    assert sum(1 for k, _ in small if k == "power") == 5, small
    assert any(k == "gstep" for k, _ in small), small
    for e, g in enumerate(got):
        assert_same_csr(g, want, f"lap2d 200x200 eval {e}")
    assert_same_csr(ref[-1], want, "lap2d 200x200 on 64-lane wavefronts")


def test_small_tier_drop_statistics():
    from paper_2208_05683_amd import binding as B

    Z, c, m, s, tau = G.random_banded(9000, 4, 0.6, 1.5, seed=33), G.exp_coeffs(20), 20, 4, 1e-9
    want, st = O.filtered_ps(Z, c, m, s, tau)
    got, gst, ref, rst = _run_both(Z, c, m, s, tau, flags=B.FPS_FLAG_DROP_STATS)
    assert _small_stages(gst)
    for e, g in enumerate(got):
        assert_same_csr(g, want, f"drop stats eval {e}")
    for key in ("stage_n_dropped", "stage_dropped_max", "stage_dropped", "stage_nnz", "stage_products"):
        assert gst[key] == rst[key], key
    assert sum(gst["stage_n_dropped"]) > 0


def test_small_tier_adaptive():
    """Algorithm 1 with its sums (and drops) taken in the small tier's write-out."""
    from paper_2208_05683_amd import api
    from gpu_helpers import download, upload

    Z, c, m, s, eps = G.laplacian_2d(100, 2.0), G.exp_coeffs(30), 30, 6, 1e-10
    sc = O.schedule(m, s)
    tmax = max(sc["q"], sc["q"] * (sc["b"] - 1))
    # the bounds ||Z^t||_1 <= ||Z||_1^t (the thresholds of eq. 28 from upper bounds)
    cs = np.zeros(Z.n)
    np.add.at(cs, Z.col, np.abs(Z.val))
    z = cs.max() ** np.arange(tmax + 1)
    want, _, a1 = O.filtered_ps_adaptive(Z, c, m, s, eps, 0.1, z)
    plan = api.Plan(upload(Z), c, m, s, adaptive=True, eps=eps, e_r=0.1, znorm=z)
    try:
        for e in range(3):
            plan.eval()
            assert_same_csr(download(plan.result()), want, f"adaptive eval {e}")
        gst = plan.stats()
        assert gst["resizes"] == 0
        assert _small_stages(gst)
        prod = [i for i, k in enumerate(gst["kind"]) if k in (0, 3)]
        assert [gst["stage_threshold"][i] for i in prod] == [x["threshold"] for x in a1]
        assert [gst["stage_alg1_iters"][i] for i in prod] == [x["iters"] for x in a1]
    finally:
        plan.close()


def test_small_tier_operand_change():
    """The operand's values scaled in place by 1.5 after the plan has learned
    its tiers: the stages in the small-row tier stay there and keep giving the
    oracle's bits (the stage whose rows were all proven empty stays so: its
    coefficient block is too small for any scaling to matter), while the last
    Horner step outgrows its learned row stride, so an evaluation is repeated
    with sizing; every evaluation gives the oracle's result for the operand it
    saw, and so does the first operand again afterwards."""
    import torch
    from paper_2208_05683_amd import api
    from gpu_helpers import download, upload

    c, m, s, tau = G.exp_coeffs(30), 30, 6, 1e-12
    Z1 = G.laplacian_2d(100, 2.0)
    Z2 = G.laplacian_2d(100, 2.0)
    Z2.val[:] = Z2.val * 1.5
    want1, _ = O.filtered_ps(Z1, c, m, s, tau)
    want2, _ = O.filtered_ps(Z2, c, m, s, tau)
    Zd = upload(Z1)
    plan = api.Plan(Zd, c, m, s, tau)
    try:
        for k in range(2):
            plan.eval()
            assert_same_csr(download(plan.result()), want1, f"first operand, evaluation {k}")
        g1 = plan.stats()
        skipped = [i for i, v in enumerate(g1["stage_rows_skipped"]) if v == Z1.n]
        assert skipped and all(g1["stage_small"][i] for i in skipped), (g1["stage_rows_skipped"], g1["stage_small"])
        Zd[2].copy_(torch.from_numpy(Z2.val).to(Zd[2].device))
        for k in range(3):
            plan.eval()
            got = download(plan.result())
            check_canonical(got)
            assert_same_csr(got, want2, f"scaled operand, evaluation {k}")
        g2 = plan.stats()
        assert g2["resizes"] >= 1, g2["resizes"]
        assert g2["stage_small"] == g1["stage_small"], (g1["stage_small"], g2["stage_small"])
        assert max(g2["stage_max_ns"]) > max(g1["stage_max_ns"])
        Zd[2].copy_(torch.from_numpy(Z1.val).to(Zd[2].device))
        plan.eval()
        assert_same_csr(download(plan.result()), want1, "first operand again")
    finally:
        plan.close()


def test_small_tier_takes_a_stage_with_a_few_long_rows():
    """A block-diagonal operand: 11,400 rows of a band of half-width 4 and
    600 rows (5%, under one in 16) of a band of half-width 14, whose fourth
    power's rows (113 entries) outgrow the small-row tier while the fixed
    stride (128) stays within four times the mean row bound (35).  The stage
    still runs in the tier and sends those rows on to the wide tier; every
    evaluation equals the oracle and the 64-lane plan bit for bit."""
    import scipy.sparse as sp

    a = G.random_banded(11400, 4, 0.8, None, seed=41).to_scipy()
    b = G.random_banded(600, 14, 1.0, None, seed=42).to_scipy()
    M = sp.block_diag([a, b], format="csr")
    M = M / abs(M).sum(axis=0).max()
    Z = G._from_scipy(sp.csr_matrix(M))
    c, m, s, tau = G.exp_coeffs(16), 16, 4, 1e-12
    want, _ = O.filtered_ps(Z, c, m, s, tau)
    got, gst, ref, rst = _run_both(Z, c, m, s, tau)
    mixed = [i for i in _small_stages(gst) if gst["stage_max_ns"][i] > 96]
    assert mixed, (gst["stage_small"], gst["stage_max_ns"])
    assert gst["rows_wide"] > 0
    for e, g in enumerate(got):
        check_canonical(g)
        assert_same_csr(g, want, f"mixed rows eval {e}")
    assert_same_csr(ref[-1], want, "mixed rows on 64-lane wavefronts")
