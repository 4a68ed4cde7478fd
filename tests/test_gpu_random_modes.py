"""Seeded random cases across the three filter modes (fixed threshold,
Algorithm 1 with the eq. 28 thresholds, series mode), matrix families and
sizes, each evaluated three times on one plan (the first evaluation sizes the
plan, later ones reuse fixed row strides, the learned shared-memory tiers and
the learned Algorithm 1 iteration counts); every evaluation must give the
oracle's result bit for bit."""

import numpy as np
import pytest

import oracle as O
from fps_inputs import generators as G

from gpu_helpers import assert_same_csr, check_canonical, download, upload

pytestmark = pytest.mark.gpu


def _matrix(rng):
    kind = int(rng.integers(0, 4))
    if kind == 0:
        n = int(rng.integers(50, 600))
        return f"random n={n}", G.random_sparse(n, float(rng.uniform(0.005, 0.05)), int(rng.integers(1 << 30)),
                                                scale=float(rng.uniform(0.3, 1.5)))
    if kind == 1:
        n, w = int(rng.integers(200, 1500)), int(rng.integers(1, 40))
        return f"banded n={n} w={w}", G.random_banded(n, w, 0.6, float(rng.uniform(0.5, 2.0)),
                                                      seed=int(rng.integers(1 << 30)))
    if kind == 2:
        side = int(rng.integers(8, 50))
        return f"lap2d {side}", G.laplacian_2d(side, float(rng.uniform(0.5, 2.5)))
    side = int(rng.integers(4, 9))
    return f"lap3d {side}", G.laplacian_3d_perturbed(side, seed=int(rng.integers(1 << 30)))


@pytest.mark.parametrize("seed", range(24))
def test_random_modes_repeated(seed):
    from paper_2208_05683_amd import api

    rng = np.random.default_rng(9100 + seed)
    name, Z = _matrix(rng)
    mode = ["fixed", "adaptive", "series"][seed % 3]
    what = f"seed {seed} {mode} {name}"
    if mode == "series":
        a = G.exp_coeffs(80) if rng.random() < 0.5 else G.cos_coeffs(80)
        eps_tol = float(10.0 ** rng.uniform(-13, -6))
        want, _, _, _ = O.series(Z, a, eps_tol, 0.1)
        plan = api.Plan.series(upload(Z), a, eps_tol, 0.1)
    else:
        m = int(rng.integers(2, 25))
        s = int(rng.integers(1, 8))
        c = G.exp_coeffs(m) if rng.random() < 0.5 else G.random_series_coeffs(m, rng)
        if mode == "fixed":
            tau = float(10.0 ** rng.uniform(-14, -4))
            want, _ = O.filtered_ps(Z, c, m, s, tau)
            plan = api.Plan(upload(Z), c, m, s, tau)
        else:
            eps = float(10.0 ** rng.uniform(-13, -5))
            sc = O.schedule(m, s)
            z = O.power_norm_bounds(Z, max(sc["q"], sc["q"] * (sc["b"] - 1)))
            want, _, _ = O.filtered_ps_adaptive(Z, c, m, s, eps, 0.1, z)
            plan = api.Plan(upload(Z), c, m, s, adaptive=True, eps=eps, e_r=0.1, znorm=list(z))
    try:
        for k in range(3):
            plan.eval()
            got = download(plan.result())
            check_canonical(got)
            assert_same_csr(got, want, f"{what}, evaluation {k}")
            if k == 0:
                resizes0 = plan.stats()["resizes"]
        # on a fixed operand no later evaluation is repeated (a speculative
        # Algorithm 1 drop that always missed would double the cost silently)
        assert plan.stats()["resizes"] == resizes0, what
    finally:
        plan.close()
