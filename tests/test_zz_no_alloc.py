"""The estimator entry point for callers that cannot allocate
(fps_normest1_noalloc), called through the C ABI: its estimate, index and
iteration count must equal fps_normest1's bit for bit, on two calls in a row
(the second on a smaller matrix, so that it reads the shared static workspace
left by the first), and sizes beyond its limits are refused."""

import numpy as np
import pytest

from fps_inputs import generators as G

from gpu_helpers import upload

pytestmark = pytest.mark.gpu


def _both(B, Zd, p):
    v = B.csr_view(*Zd)
    a = B.fps_normest1(v, p)
    b = B.fps_normest1_noalloc(v, p)
    return a, b


def test_noalloc_estimator_matches_allocating_one():
    from paper_2208_05683_amd import binding as B

    big = G.laplacian_2d(200, 2.0)                                   # n = 40000, the 2D workload
    small = G.random_sparse(700, 0.01, seed=3, scale=0.8)            # n = 700, signed entries
    for name, Z, ps in (("lap2d 200", big, (1, 4, 7)), ("random 700", small, (0, 1, 3, 10))):
        Zd = upload(Z)
        for p in ps:
            a, b = _both(B, Zd, p)
            assert np.float64(a["est"]).view(np.uint64) == np.float64(b["est"]).view(np.uint64), (name, p, a, b)
            assert (a["ind"], a["iters"]) == (b["ind"], b["iters"]), (name, p, a, b)
            assert b["est"] > 0.0


def test_noalloc_estimator_largest_accepted_and_refused_sizes():
    from paper_2208_05683_amd import binding as B

    # n at the limit: a 1D Laplacian with FPS_NOALLOC_MAX_N rows
    Z = G.laplacian_1d(B.FPS_NOALLOC_MAX_N, 1.0)
    Zd = upload(Z)
    a, b = _both(B, Zd, 2)
    assert a == b
    # one row more is refused before any device work
    Z2 = G.laplacian_1d(B.FPS_NOALLOC_MAX_N + 1, 1.0)
    with pytest.raises(B.FpsError) as e:
        B.fps_normest1_noalloc(B.csr_view(*upload(Z2)), 1)
    assert e.value.status == B.FPS_ERR_CAPACITY
    # and a smaller call afterwards still agrees
    Z3 = G.laplacian_2d(30, 2.0)
    a, b = _both(B, upload(Z3), 3)
    assert a == b
