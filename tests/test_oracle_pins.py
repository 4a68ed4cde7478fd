"""Pins for the CPU oracle: closed forms, brute force, the paper's operation
count and error bound, invariants and an independent second implementation.

Each test ties the oracle to something other than itself, so that a plausible
mistake in it (a dropped term, a wrong coefficient index, a transposed
operand, a filter applied at the wrong stage) fails at least one of them.
"""

import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from oracle.bound import filtering_bound, power_norms, rounding_slack
from fps_inputs import generators as G


def check_canonical(M):
    rp, cl, vl = M.row_ptr, M.col, M.val
    assert rp[0] == 0 and rp[-1] == cl.size == vl.size
    assert np.all(np.diff(rp) >= 0)
    for r in range(M.n):
        c = cl[rp[r]:rp[r + 1]]
        assert np.all(np.diff(c) > 0), f"row {r} not sorted/unique"
    if cl.size:
        assert cl.min() >= 0 and cl.max() < M.n
    assert np.all(vl != 0.0)
    assert np.all(np.isfinite(vl))


def rel_fro(X, Y):
    return float(np.linalg.norm(X - Y) / np.linalg.norm(Y))


# ---------------------------------------------------------------------------
# P8: schedule and number of sparse products (eqs. 5-6)
# ---------------------------------------------------------------------------

def test_schedule_counts_match_eq5():
    for m in range(0, 41):
        N = m + 1
        for s in range(1, 13):
            sc = O.schedule(m, s)
            q, b = s, -(-N // s)
            g = 1 if N - q * (b - 1) == 1 else 0
            assert (sc["q"], sc["b"], sc["g"]) == (q, b, g)
            if b >= 2:
                assert sc["n_spgemm"] == q + b - 2 - g  # eq. 5
            else:
                assert sc["n_spgemm"] == max(m - 1, 0)


def test_paper_q_choice_gives_eq5_minimum():
    # with q = floor(sqrt(N-1)) (eq. 6) and N > 2 the count is mt(N) of eq. 5
    for N in range(3, 60):
        q = math.isqrt(N - 1)
        b = -(-N // q)
        g = 1 if N - q * (b - 1) == 1 else 0
        assert O.schedule(N - 1, q)["n_spgemm"] == q + b - 2 - g


@pytest.mark.parametrize("m,s", [(16, 4), (30, 6), (24, 5), (7, 1), (9, 3), (3, 8)])
def test_stage_log_matches_schedule(m, s):
    Z = G.random_banded(60, 2, 0.6, 1.0, seed=1)
    _, st = O.filtered_ps(Z, G.exp_coeffs(m), m, s, 1e-12)
    n_products = sum(1 for x in st if x["kind"] in (0, 3))
    assert n_products == O.schedule(m, s)["n_spgemm"]


# ---------------------------------------------------------------------------
# P1: nilpotent shift matrices, exact closed form (bitwise)
# ---------------------------------------------------------------------------

def shift_expected(n, v, c, m, s, tau):
    """F for Z = v*J (J the upper shift) with v a power of two.

    Every product then has a single term, so no rounding happens.  The filtered
    power P_j = v^j J^j (eq. 11) is dropped whole once |v^j| < tau (j >= 2),
    and every later power with it.  Block i enters the Horner recurrence at
    step b-1-i (eq. 14) with the value c_k v^j on the k-th superdiagonal; with
    g = 1 the last coefficient rides with block b-2 as its j = q term.  Each
    later step multiplies by P_q (or annihilates if P_q was dropped); steps
    start..b-1 are filtered and drop the entry once its magnitude is below tau."""
    sc = O.schedule(m, s)
    q, b, g, start = sc["q"], sc["b"], sc["g"], sc["start"]
    J = sc["J"]
    alive = [True] * (J + 2)
    for j in range(2, J + 1):
        alive[j] = alive[j - 1] and abs(v ** j) >= tau and j < n
    E = np.zeros((n, n))
    for k in range(0, min(m, n - 1) + 1):
        if c[k] == 0.0:
            continue
        if b >= 2 and g == 1 and k == m:
            i, j = b - 2, q
        else:
            i, j = divmod(k, q)
        if j >= 1 and not alive[j]:
            continue
        val, e = c[k] * v ** j, j
        dropped = False
        if b >= 2:
            entry = b - 1 - i
            for t in range(entry, b):
                if t > entry:
                    if not alive[q]:
                        dropped = True
                        break
                    val, e = val * v ** q, e + q
                if e >= n:
                    dropped = True
                    break
                if t >= start and abs(val) < tau:
                    dropped = True
                    break
        if not dropped:
            assert val == c[k] * v ** k
            E[np.arange(n - k), np.arange(k, n)] = val
    return E


@pytest.mark.parametrize("n,v,m,s,tau", [
    (12, 1.0, 16, 4, 1e-14),    # b=5, g=1
    (12, 0.5, 16, 4, 1e-9),     # values shrink through the steps
    (20, 2.0, 9, 3, 1e-3),      # values grow: the first filtered step decides
    (9, 1.0, 5, 8, 1e-2),       # b=1: nothing is filtered at all
    (9, 1.0, 4, 3, 1e-2),       # b=2, g=1: the only Horner step is the shortcut
    (9, 0.5, 6, 3, 5e-3),       # b=3, g=1
    (30, 0.5, 24, 5, 1e-10),    # b=5, g=0 (config-3 shape)
    (7, 1.0, 12, 1, 1e-4),      # s=1: plain filtered Horner
    (40, 1.0, 30, 6, 1e-12),    # config-2 shape
    (12, 0.0625, 16, 4, 1e-4),  # P_4 itself drops, so every Horner product vanishes
    (16, 0.125, 14, 5, 1e-5),   # P_5 drops (q = 5): only the coefficient sums survive
    (16, 0.25, 11, 3, 2e-3),    # P_3 survives narrowly, later values drop
    (12, 0.0625, 5, 8, 1e-4),   # b=1: a dropped power is the only filter applied
    (12, 0.0625, 4, 4, 1e-4),   # b=2, g=1: P_q drops before the unfiltered shortcut
])
def test_shift_matrix_closed_form(n, v, m, s, tau):
    Z = G.shift_matrix(n, 1, v)
    c = G.exp_coeffs(m)
    F, _ = O.filtered_ps(Z, c, m, s, tau)
    check_canonical(F)
    np.testing.assert_array_equal(F.to_dense(), shift_expected(n, v, c, m, s, tau))


def test_shift_matrix_transpose_is_lower():
    # the transpose of the problem must give the transposed (lower) answer
    n, m, s = 10, 8, 3
    Z = G.shift_matrix(n, 1, 1.0)
    Zt = G.from_dense(Z.to_dense().T)
    c = G.exp_coeffs(m)
    F, _ = O.filtered_ps(Z, c, m, s, 0.0)
    Ft, _ = O.filtered_ps(Zt, c, m, s, 0.0)
    np.testing.assert_array_equal(Ft.to_dense(), F.to_dense().T)
    assert np.allclose(np.tril(F.to_dense(), -1), 0)


# ---------------------------------------------------------------------------
# P2: strictly upper triangular Z with m >= n-1 terminates exactly
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_nilpotent_series_terminates(seed):
    n = 12
    Z = G.random_sparse(n, 0.5, seed, scale=0.7, strictly_upper=True)
    Zd = Z.to_dense()
    m = 20  # >= n-1, so exp(Z) = P_m(Z) exactly
    c = G.exp_coeffs(m)
    F, _ = O.unfiltered_ps(Z, c, m, 4)
    # exp of a nilpotent matrix by its finite Taylor sum in long double
    E = np.eye(n, dtype=np.longdouble)
    T = np.eye(n, dtype=np.longdouble)
    for k in range(1, n):
        T = T @ Zd.astype(np.longdouble) / k
        E = E + T
    assert float(np.max(np.abs(F.to_dense() - E.astype(np.float64)))) <= 1e-14 * float(np.max(np.abs(E)))


# ---------------------------------------------------------------------------
# P3: diagonal Z reduces to scalar series
# ---------------------------------------------------------------------------

def test_diagonal_exp_and_cos_closed_form():
    rng = np.random.default_rng(7)
    lam = rng.uniform(-1.0, 1.0, 50)
    Z = G.diagonal(lam)
    m = 22
    F, _ = O.filtered_ps(Z, G.exp_coeffs(m), m, 5, 1e-300)
    d = F.to_dense()
    assert np.allclose(d, np.diag(np.diag(d)), atol=0)
    # truncation |lam|^(m+1) e^|lam| / (m+1)! < 1e-22, so only rounding remains
    np.testing.assert_allclose(np.diag(d), np.exp(lam), rtol=4e-16 * (m + 1), atol=0)
    F, _ = O.filtered_ps(Z, G.cos_coeffs(m), m, 5, 1e-300)
    np.testing.assert_allclose(np.diag(F.to_dense()), np.cos(lam), rtol=4e-16 * (m + 1), atol=1e-16)


def test_diagonal_exact_rationals():
    # lam = 1/2, 1/4, 1/8 and s = 1 (plain Horner): compare with the exact
    # rational polynomial value; the computed value is within (m+1) ulps
    lam = [0.5, 0.25, -0.125]
    Z = G.diagonal(lam)
    m = 10
    c = G.exp_coeffs(m)
    for s in (1, 3, 4, 11):
        F, _ = O.unfiltered_ps(Z, c, m, s)
        got = np.diag(F.to_dense())
        for i, x in enumerate(lam):
            exact = sum(Fraction(c[k]) * Fraction(x) ** k for k in range(m + 1))
            assert abs(Fraction(float(got[i])) - exact) <= Fraction(2 * (m + 1)) * Fraction(2.0 ** -52) * abs(exact)


# ---------------------------------------------------------------------------
# P4: special cases
# ---------------------------------------------------------------------------

def test_zero_matrix_gives_c0_identity():
    n = 5
    Z = G.empty_matrix(n)
    for m, s in [(0, 3), (5, 2), (16, 4), (30, 6)]:
        c = G.exp_coeffs(m)
        F, _ = O.filtered_ps(Z, c, m, s, 1e-12)
        np.testing.assert_array_equal(F.to_dense(), np.eye(n))


def test_zero_matrix_small_c0_filtered_only_if_a_filtered_step_runs():
    n = 4
    Z = G.empty_matrix(n)
    c = np.array([1e-20, 1.0, 1.0, 1.0, 1.0])
    # m=4, s=2: b=3, g=1, one filtered step (i=2) -> c_0 I dropped
    F, _ = O.filtered_ps(Z, c, 4, 2, 1e-12)
    assert F.nnz == 0
    # m=4, s=8: b=1, nothing filtered -> c_0 I kept
    F, _ = O.filtered_ps(Z, c, 4, 8, 1e-12)
    np.testing.assert_array_equal(F.to_dense(), 1e-20 * np.eye(n))


def test_scalar_n1_equals_polynomial():
    Z = G.diagonal([0.75])
    m = 14
    c = G.exp_coeffs(m)
    for s in range(1, 16):
        F, _ = O.unfiltered_ps(Z, c, m, s)
        assert abs(F.val[0] - sum(c[k] * 0.75 ** k for k in range(m + 1))) <= 1e-15


def test_s1_is_plain_horner_count():
    Z = G.random_banded(30, 2, 0.6, 1.0, seed=3)
    m = 9
    _, st = O.filtered_ps(Z, G.exp_coeffs(m), m, 1, 1e-14)
    assert sum(1 for x in st if x["kind"] in (0, 3)) == m - 1


# ---------------------------------------------------------------------------
# P5 / P6: unfiltered PS against Horner (double) and long-double brute force
# ---------------------------------------------------------------------------

def test_config1_unfiltered_matches_dense_horner():
    cfg = G.config1()
    F, _ = O.unfiltered_ps(cfg["Z"], cfg["coeffs"], cfg["m"], cfg["s"])
    Y = O.dense_horner(cfg["Z"].to_dense(), cfg["coeffs"])
    assert rel_fro(F.to_dense(), Y) <= 1e-14


@pytest.mark.parametrize("seed", range(6))
def test_small_random_nonsymmetric_against_long_double(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 40))
    Z = G.random_sparse(n, 0.2, seed, scale=0.4)
    m = int(rng.integers(3, 25))
    s = int(rng.integers(1, 7))
    c = G.exp_coeffs(m) if seed % 2 == 0 else G.random_series_coeffs(m, rng)
    Yld = O.dense_horner_ld(Z.to_dense(), c)
    Y = Yld.astype(np.float64)
    F, _ = O.unfiltered_ps(Z, c, m, s)
    assert rel_fro(F.to_dense(), Y) <= 1e-14
    # and the result is not symmetric, so a transposed operand would show
    if np.linalg.norm(Y - Y.T) > 1e-3 * np.linalg.norm(Y):
        assert rel_fro(F.to_dense().T, Y) > 1e-6


# ---------------------------------------------------------------------------
# P7: the paper's a-posteriori filtering bound (eq. 23)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["c1", "lap2d_side20", "band_big_tau", "rand_small", "cos3d"])
def test_filtering_error_within_eq23_bound(case):
    if case == "c1":
        cfg = G.config1()
        Z, c, m, s, tau = cfg["Z"], cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"]
    elif case == "lap2d_side20":
        Z, c, m, s, tau = G.laplacian_2d(20, 2.0), G.exp_coeffs(30), 30, 6, 1e-8
    elif case == "band_big_tau":
        Z, c, m, s, tau = G.random_banded(300, 3, 0.6, 1.5, seed=11), G.exp_coeffs(20), 20, 4, 1e-6
    elif case == "rand_small":
        Z, c, m, s, tau = G.random_sparse(40, 0.1, 5, 0.5), G.exp_coeffs(18), 18, 3, 1e-5
    else:
        Z, c, m, s, tau = G.laplacian_3d_perturbed(6, seed=3), G.cos_coeffs(24), 24, 5, 1e-7
    F, st = O.filtered_ps(Z, c, m, s, tau)
    if Z.n <= 64:
        P = O.dense_horner_ld(Z.to_dense(), c).astype(np.float64)
    else:
        P = O.dense_horner(Z.to_dense(), c)
    err = O.norm1(F.to_dense() - P)
    z = power_norms(Z, s * (-(-(m + 1) // s)))
    bd = filtering_bound(c, m, s, st, z)
    slack = rounding_slack(c, m, O.norm1(Z))
    assert sum(x["n_dropped"] for x in st) > 0, "case must exercise the filter"
    assert err > 0
    assert err <= bd["bound"] * (1 + 1e-3) + slack, (err, bd["bound"], slack)


# ---------------------------------------------------------------------------
# P9: invariants
# ---------------------------------------------------------------------------

def test_invariants_and_structure_subset():
    Z = G.laplacian_2d(30, 2.0)
    m, s, tau = 30, 6, 1e-10
    c = G.exp_coeffs(m)
    F, st = O.filtered_ps(Z, c, m, s, tau)
    F0, _ = O.unfiltered_ps(Z, c, m, s)
    check_canonical(F)
    check_canonical(F0)
    for x in st:
        if x["kind"] in (0, 3):  # filtered stages
            assert x["dropped_max"] < tau
            assert x["kept_min"] >= tau or x["nnz_kept"] == 0
        else:  # coefficient sums drop exact zeros only
            assert x["n_dropped"] == 0
    assert np.all(np.abs(F.val) >= tau)
    # filtering only removes structure (Section 4: PSSCF results are sparser)
    s_f = set(zip(np.repeat(np.arange(F.n), np.diff(F.row_ptr)), F.col))
    s_0 = set(zip(np.repeat(np.arange(F0.n), np.diff(F0.row_ptr)), F0.col))
    assert s_f <= s_0
    assert F.nnz < F0.nnz


def test_tie_at_tau_is_kept():
    # Z = diag(0.5): P_2 = 0.25 exactly; tau = 0.25 keeps it, tau = nextafter drops it
    Z = G.diagonal([0.5])
    A, _ = O.spgemm(Z, Z, None, 0.25)
    assert A.nnz == 1 and A.val[0] == 0.25
    B, _ = O.spgemm(Z, Z, None, np.nextafter(0.25, 1.0))
    assert B.nnz == 0


def test_exact_cancellation_dropped_even_without_filter():
    Z = G.from_dense(np.array([[1.0, 1.0], [1.0, -1.0]]))
    # Z^2 = 2 I: off-diagonals cancel exactly and must not be stored
    P, st = O.spgemm(Z, Z, None, 0.0)
    np.testing.assert_array_equal(P.to_dense(), 2 * np.eye(2))
    assert st["n_zero"] == 2


# ---------------------------------------------------------------------------
# P10: regrouping invariance (eq. 2 is an exact regrouping)
# ---------------------------------------------------------------------------

def test_unfiltered_result_independent_of_s():
    Z = G.random_banded(200, 3, 0.6, 1.2, seed=9)
    m = 20
    c = G.exp_coeffs(m)
    ref, _ = O.unfiltered_ps(Z, c, m, 1)
    R = ref.to_dense()
    for s in range(2, 10):
        F, _ = O.unfiltered_ps(Z, c, m, s)
        assert rel_fro(F.to_dense(), R) <= 1e-14


# ---------------------------------------------------------------------------
# P12: an independent second implementation (scipy sparse products)
# ---------------------------------------------------------------------------

def _scipy_filtered_ps(Z, c, m, s, tau):
    n = Z.n
    A = Z.to_scipy().tocsr()
    N = m + 1
    q, b = s, -(-N // s)
    g = N - q * (b - 1) == 1

    def filt(M):
        M = M.tocsr()
        M.data[np.abs(M.data) < tau] = 0.0
        M.eliminate_zeros()
        return M

    J = q if b >= 2 else m
    P = [sp.identity(n, format="csr"), A]
    for _ in range(2, J + 1):
        P.append(filt(A @ P[-1]))

    def block(i, jmax):
        out = sp.csr_matrix((n, n))
        for j in range(0, jmax + 1):
            if i * q + j <= m:
                out = out + c[i * q + j] * P[j]
        return out

    if b == 1:
        return block(0, q - 1)
    if g:
        S = block(b - 2, q)
        start = 2
    else:
        S = block(b - 1, q - 1)
        start = 1
    for i in range(start, b):
        S = filt(block(b - 1 - i, q - 1) + P[q] @ S)
    return S


@pytest.mark.parametrize("case", ["c1", "band", "lap2d", "rand"])
def test_against_scipy_implementation(case):
    if case == "c1":
        cfg = G.config1()
        Z, c, m, s, tau = cfg["Z"], cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"]
    elif case == "band":
        Z, c, m, s, tau = G.random_banded(500, 4, 0.6, 1.7, seed=2), G.exp_coeffs(20), 20, 5, 1e-12
    elif case == "lap2d":
        Z, c, m, s, tau = G.laplacian_2d(40, 2.0), G.cos_coeffs(30), 30, 6, 1e-12
    else:
        Z, c, m, s, tau = G.random_sparse(80, 0.05, 4, 0.8), G.exp_coeffs(15), 15, 4, 0.0
    F, _ = O.filtered_ps(Z, c, m, s, tau)
    R = _scipy_filtered_ps(Z, c, m, s, tau).toarray()
    assert rel_fro(F.to_dense(), R) <= (1e-14 if tau == 0 else 1e-10)


# ---------------------------------------------------------------------------
# Adaptive filter (Algorithm 1) and the eq. 28 thresholds
# ---------------------------------------------------------------------------

def _exact_col_norm1(M, mask):
    """max over columns of the exactly rounded sum of |x| over masked entries."""
    rows_cols = {}
    for r in range(M.n):
        for p in range(M.row_ptr[r], M.row_ptr[r + 1]):
            if mask[p]:
                rows_cols.setdefault(int(M.col[p]), []).append(abs(float(M.val[p])))
    return max((math.fsum(v) for v in rows_cols.values()), default=0.0)


def _dropped_mask(before, after):
    kept = set()
    for r in range(after.n):
        for p in range(after.row_ptr[r], after.row_ptr[r + 1]):
            kept.add((r, int(after.col[p])))
    mask = np.zeros(before.nnz, dtype=bool)
    for r in range(before.n):
        for p in range(before.row_ptr[r], before.row_ptr[r + 1]):
            mask[p] = (r, int(before.col[p])) not in kept
    return mask


@pytest.mark.parametrize("seed", range(6))
def test_alg1_postconditions(seed):
    rng = np.random.default_rng(40 + seed)
    n = int(rng.integers(5, 60))
    d = np.where(rng.random((n, n)) < 0.3, 10.0 ** rng.uniform(-16, -9, (n, n)), 0.0)
    d *= np.where(rng.random((n, n)) < 0.5, -1.0, 1.0)
    M = G.from_dense(d)
    eps_g = float(10.0 ** rng.uniform(-13, -10))
    e_r = 0.1
    F, st = O.alg1_filter(M, eps_g, e_r)
    check_canonical(F)
    drop = _dropped_mask(M, F)
    t = st["threshold"]
    assert 0 < t <= eps_g
    # exactly the entries with |x| <= t are dropped
    np.testing.assert_array_equal(drop, np.abs(M.val) <= t)
    # the dropped norm satisfies Algorithm 1's postcondition, and the reported
    # (integer-summed) norm bounds the exact one from above
    exact = _exact_col_norm1(M, drop)
    assert exact <= eps_g * (1 + e_r)
    assert exact <= st["dropped"] * (1 + 1e-12) + 1e-300
    assert st["dropped"] <= eps_g * (1 + e_r)
    # the loop did not stop earlier
    if st["iters"] > 1:
        with pytest.raises(RuntimeError):
            O.alg1_filter(M, eps_g, e_r, max_iter=st["iters"] - 1)


def test_alg1_closed_forms():
    eps = 1e-10
    # one column with 10 entries of 0.5 eps: the first candidate set has norm
    # 5 eps > 1.1 eps, the next threshold eps / 5 protects every entry
    d = np.zeros((12, 12))
    d[:10, 3] = 0.5 * eps
    d[11, 11] = 1.0
    F, st = O.alg1_filter(G.from_dense(d), eps, 0.1)
    assert st["iters"] == 2 and st["dropped"] == 0.0 and F.nnz == 11
    assert abs(st["threshold"] - eps / 5) <= 1e-15 * eps
    # geometric column eps 2^-i: norm < eps, all dropped in one iteration
    d = np.zeros((25, 25))
    d[:20, 0] = eps * 2.0 ** -np.arange(1, 21)
    d[24, 24] = 1.0
    F, st = O.alg1_filter(G.from_dense(d), eps, 0.1)
    assert st["iters"] == 1 and F.nnz == 1
    # a diagonal candidate matrix has norm max|x| <= eps: one iteration
    F, st = O.alg1_filter(G.diagonal([0.3 * eps, 0.9 * eps, 2 * eps]), eps, 0.0)
    assert st["iters"] == 1 and F.nnz == 1 and F.val[0] == 2 * eps
    # ties: |x| == eps_f is a candidate (Algorithm 1 protects |x| > eps_f only)
    F, st = O.alg1_filter(G.diagonal([eps, 1.0]), eps, 0.0)
    assert F.nnz == 1
    # ... also in the candidate norm: a column {eps, 0.2 eps} has norm 1.2 eps >
    # 1.1 eps at eps_f = eps, so the next threshold eps/1.2 keeps the tie entry
    d = np.zeros((3, 3))
    d[0, 1], d[1, 1], d[2, 2] = eps, 0.2 * eps, 1.0
    F, st = O.alg1_filter(G.from_dense(d), eps, 0.1)
    assert st["iters"] == 2 and F.nnz == 2 and eps in F.val


@pytest.mark.parametrize("m,s", [(16, 4), (30, 6), (24, 5), (9, 3), (20, 4), (7, 8)])
def test_fnt_thresholds_share_eps_equally(m, s):
    # eq. 28: each filtered stage gets the same share eps / M of the eq. 27
    # budget, so the eq. 23 bound evaluated at the thresholds equals eps
    Z = G.random_banded(80, 2, 0.6, 1.3, seed=7)
    c = G.exp_coeffs(m) if m != 24 else G.cos_coeffs(24)
    sc = O.schedule(m, s)
    z = power_norms(Z, max(sc["q"], sc["q"] * (sc["b"] - 1)))
    eps = 1e-11
    zeta, sigma = O.fnt_thresholds(c, m, s, eps, z)
    stats = [{"kind": 0, "index": k, "dropped_1norm": zeta[k]} for k in range(2, sc["J"] + 1)]
    stats += [{"kind": 3, "index": j, "dropped_1norm": sigma[j]} for j in range(sc["start"], sc["b"])]
    bd = filtering_bound(c, m, s, stats, z)
    assert abs(bd["bound"] - eps) <= 1e-12 * eps, (bd["bound"], eps)


@pytest.mark.parametrize("case", ["c1", "lap2d", "band", "rand", "cos3d"])
def test_adaptive_error_within_eps(case):
    # the paper's guarantee (eq. 27): with the eq. 28 thresholds the filtering
    # error is at most eps (1 + e_r) to first order
    if case == "c1":
        Z, c, m, s = G.laplacian_1d(400, 1.0), G.exp_coeffs(16), 16, 4
    elif case == "lap2d":
        Z, c, m, s = G.laplacian_2d(25, 2.0), G.exp_coeffs(30), 30, 6
    elif case == "band":
        Z, c, m, s = G.random_banded(300, 3, 0.6, 1.5, seed=5), G.exp_coeffs(20), 20, 4
    elif case == "rand":
        Z, c, m, s = G.random_sparse(50, 0.08, 3, 0.4), G.exp_coeffs(18), 18, 3
    else:
        Z, c, m, s = G.laplacian_3d_perturbed(6, seed=3), G.cos_coeffs(24), 24, 5
    sc = O.schedule(m, s)
    z = power_norms(Z, max(sc["q"], sc["q"] * (sc["b"] - 1)))
    for eps in (1e-12, 1e-8):
        e_r = 0.1
        F, st, a1 = O.filtered_ps_adaptive(Z, c, m, s, eps, e_r, z)
        check_canonical(F)
        assert len(a1) == sc["n_spgemm"]
        for a in a1:
            assert a["dropped"] <= a["eps_g"] * (1 + e_r)
        if Z.n <= 64:
            P = O.dense_horner_ld(Z.to_dense(), c).astype(np.float64)
        else:
            P = O.dense_horner(Z.to_dense(), c)
        err = O.norm1(F.to_dense() - P)
        assert err <= eps * (1 + e_r) * (1 + 1e-3) + rounding_slack(c, m, O.norm1(Z)), (case, eps, err)
        # every filtered stage ran Algorithm 1 with its eq. 28 threshold
        zeta, sigma = O.fnt_thresholds(c, m, s, eps, z)
        want = [zeta[k] for k in range(2, sc["J"] + 1)] + [sigma[j] for j in range(sc["start"], sc["b"])]
        np.testing.assert_array_equal([a["eps_g"] for a in a1], want)
        if case in ("lap2d", "band") and eps == 1e-8:
            # and the Horner steps do filter: the result is much sparser
            F0, _ = O.unfiltered_ps(Z, c, m, s)
            assert F.nnz < 0.8 * F0.nnz
            assert any(a["dropped"] > 0 for a in a1[sc["J"] - 1:])
    # a tiny budget drops (almost) nothing beyond exact zeros
    F, _, _ = O.filtered_ps_adaptive(Z, c, m, s, 1e-300, 0.1, z)
    F0, _ = O.unfiltered_ps(Z, c, m, s)
    assert F.nnz == F0.nnz


# ---------------------------------------------------------------------------
# Series mode (Section 3.2, Algorithm 2 steps 1-3): the 1-norm estimator on
# Z^p, the bounds of eq. 37 (Lemma 1) and the degree N of eq. 34
# ---------------------------------------------------------------------------

def _nonneg_random(n, density, seed):
    rng = np.random.default_rng(seed)
    d = (rng.random((n, n)) < density) * rng.random((n, n))
    np.fill_diagonal(d, 0.0)
    d[np.arange(n - 1), np.arange(1, n)] += 0.25  # a path so that powers stay nonzero
    return G.from_dense(d)


def _exact_power_norm1(Zd, p):
    """||Z^p||_1 in exact rational arithmetic (tiny matrices only)."""
    n = Zd.shape[0]
    A = [[Fraction(float(Zd[i, j])) for j in range(n)] for i in range(n)]
    P = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for _ in range(p):
        P = [[sum((P[i][k] * A[k][j] for k in range(n) if A[k][j] != 0), Fraction(0)) for j in range(n)]
             for i in range(n)]
    return max(sum(abs(P[i][j]) for i in range(n)) for j in range(n))


@pytest.mark.parametrize("seed", range(4))
def test_normest1_exact_for_nonnegative_matrices(seed):
    # For a nonnegative A the estimator's first sign vector is all ones, so
    # A^T s is the vector of column sums and the second iterate is the column
    # of largest sum: the estimate is ||A||_1 itself.
    n = 9 + seed
    Z = _nonneg_random(n, 0.3, seed)
    Zd = Z.to_dense()
    for p in (1, 2, 3, 5):
        r = O.normest1_power(Z, p)
        exact = float(_exact_power_norm1(Zd, p))
        assert abs(r["est"] - exact) <= 1e-14 * exact, (p, r, exact)
        assert r["ind"] >= 0


@pytest.mark.parametrize("seed", range(6))
def test_normest1_is_an_attained_lower_bound(seed):
    # est <= ||A||_1 always; est is the 1-norm of A v for the returned unit
    # vector v = e_ind (or of the start vector ones/n); the iteration never
    # returns less than its first iterate
    Z = G.random_sparse(40, 0.12, seed + 11, 0.5)
    Zd = Z.to_dense()
    for p in (1, 2, 4):
        A = np.linalg.matrix_power(Zd, p)
        r = O.normest1_power(Z, p)
        colsums = np.abs(A).sum(0)
        first = np.abs(A @ np.full(Z.n, 1.0 / Z.n)).sum()
        assert r["est"] <= colsums.max() * (1 + 1e-12)
        assert r["est"] >= first * (1 - 1e-12)
        attained = colsums[r["ind"]] if r["ind"] >= 0 else first
        assert abs(r["est"] - attained) <= 1e-12 * max(attained, 1e-300), (p, r, attained)
        assert 1 <= r["iters"] <= 6


def test_normest1_closed_forms():
    # diagonal: ||D^p||_1 = max |d|^p; shift J: ||J^p||_1 = 1 for p < n, 0 after
    d = np.array([0.5, -1.25, 0.75, -0.3, 1.0])
    Z = G.diagonal(d)
    for p in range(1, 6):
        assert O.normest1_power(Z, p)["est"] == 1.25 ** p
    J = G.shift_matrix(6)
    for p in range(1, 9):
        assert O.normest1_power(J, p)["est"] == (1.0 if p < 6 else 0.0)
    assert O.normest1_power(G.diagonal([-3.0]), 3)["est"] == 27.0


@pytest.mark.parametrize("seed", range(3))
def test_power_norm_bounds_eq37_and_lemma1(seed):
    # z[0] = 1, z[i] the estimates up to K = 10; beyond K, Lemma 1 gives
    # ||Z^i|| <= alpha^i with alpha = max_{k=5..10} ||Z^k||^(1/k), so with the
    # exact norms of a nonnegative matrix every z[i] bounds ||Z^i||_1
    n = 10
    Z = _nonneg_random(n, 0.35, 20 + seed)
    Zd = Z.to_dense()
    z = O.power_norm_bounds(Z, 20)
    assert z[0] == 1.0
    for i in range(1, 11):
        assert z[i] == O.normest1_power(Z, i)["est"]
    for i in range(11, 21):
        exact = float(_exact_power_norm1(Zd, i))
        assert z[i] >= exact * (1 - 1e-12), (i, z[i], exact)
    # a 2-cycle with weights 4 and 1/4: ||Z^k||_1 is 4 for odd k and 1 for even
    # k, so only the maximum over k = 5..10 (alpha = 4^(1/5)) bounds the odd powers
    C2 = G.from_dense(np.array([[0.0, 4.0], [0.25, 0.0]]))
    zc = O.power_norm_bounds(C2, 21)
    for i in range(1, 22):
        assert zc[i] >= (4.0 if i % 2 else 1.0) * (1 - 1e-12), (i, zc[i])
    # diagonal closed form: every ||D^k||^(1/k) = max |d|, so z[i] = max|d|^i
    zd = O.power_norm_bounds(G.diagonal([0.25, -1.5, 1.0]), 16)
    for i in range(17):
        assert abs(zd[i] - 1.5 ** i) <= 1e-14 * 1.5 ** i


@pytest.mark.parametrize("eps", [1e-4, 3e-7, 1e-10, 2e-13, 1e-15])
def test_series_degree_eq34_in_exact_arithmetic(eps):
    # N = min m with sum_{i>=m} |a_i| z_i <= eps/2 (eq. 34), recomputed with
    # exact rationals from the same double inputs; q = floor(sqrt(N - 1))
    L = 60
    a = G.exp_coeffs(L - 1)
    z = np.array([1.5 ** i for i in range(L)])
    T = [Fraction(0)] * (L + 1)
    for m in range(L - 1, -1, -1):
        T[m] = T[m + 1] + Fraction(float(a[m])) * Fraction(float(z[m]))
    half = Fraction(eps) / 2
    N = next(m for m in range(1, L + 1) if T[m] <= half)
    # stay away from inputs whose decision rounding could flip
    assert abs(T[N] - half) > half * Fraction(1, 10 ** 9) and abs(T[N - 1] - half) > half * Fraction(1, 10 ** 9)
    d = O.series_degree(a, z, eps)
    assert d["N"] == N
    assert d["q"] == max(1, math.isqrt(N - 1))
    assert abs(Fraction(d["tail"]) - T[N]) <= T[N] * Fraction(1, 10 ** 13)
    with pytest.raises(RuntimeError):
        O.series_degree(a[:N], z[:N], eps)  # too few coefficients: the tail is not below eps/2


@pytest.mark.parametrize("case", ["exp_lap2d", "exp_band", "cos_lap1d", "exp_rand"])
def test_series_mode_error_within_tol(case):
    # Algorithm 2: ||f(Z) - F|| <= eps_tol, with f computed by scipy's dense
    # expm / cosm; the truncation tail and the filtering budget of eq. 36
    # add up to eps_tol
    import scipy.linalg as sl

    if case == "exp_lap2d":
        Z, a, f = G.laplacian_2d(10, 2.0), G.exp_coeffs(60), sl.expm
    elif case == "exp_band":
        Z, a, f = G.random_banded(120, 3, 0.6, 1.5, seed=9), G.exp_coeffs(60), sl.expm
    elif case == "cos_lap1d":
        Z, a, f = G.laplacian_1d(150, 2.5), G.cos_coeffs(70), sl.cosm
    else:
        Z, a, f = G.random_sparse(60, 0.1, 4, 0.5), G.exp_coeffs(60), sl.expm
    ref = f(Z.to_dense())
    for eps_tol in (1e-6, 1e-11):
        e_r = 0.1
        F, info, st, a1 = O.series(Z, a, eps_tol, e_r)
        check_canonical(F)
        sc = O.schedule(info["m"], info["s"])
        assert info["m"] == info["N"] - 1 and info["s"] == info["q"]
        assert info["budget"] + info["tail"] == pytest.approx(eps_tol, rel=1e-15)
        assert info["tail"] <= 0.5 * eps_tol
        assert len(a1) == sc["n_spgemm"]
        # the thresholds of eq. 36 share the budget eps_tol - T_N equally
        zeta, sigma = O.fnt_thresholds(a[: info["N"]], info["m"], info["s"], info["budget"], info["z"])
        stats = [{"kind": 0, "index": k, "dropped_1norm": zeta[k]} for k in range(2, sc["J"] + 1)]
        stats += [{"kind": 3, "index": j, "dropped_1norm": sigma[j]} for j in range(sc["start"], sc["b"])]
        bd = filtering_bound(a[: info["N"]], info["m"], info["s"], stats, info["z"])
        assert abs(bd["bound"] - info["budget"]) <= 1e-12 * info["budget"]
        err = O.norm1(F.to_dense() - ref)
        assert err <= eps_tol * (1 + e_r), (case, eps_tol, err, info["N"])


def test_banded_test_set_generator():
    # test set 2: equal lower and upper bandwidth b, every in-band entry drawn
    # from N(0, 1), 1000 x 1000
    for bw in (1, 7, 15):
        Z = G.banded_sweep_matrix(bw, 1000, seed=1000 * bw + 3)
        d = Z.to_dense()
        i, j = np.nonzero(d)
        assert Z.n == 1000 and np.abs(i - j).max() == bw
        assert Z.nnz == sum(1000 - abs(k) for k in range(-bw, bw + 1))
        assert abs(Z.val.mean()) < 4.0 / np.sqrt(Z.nnz) and abs(Z.val.std() - 1.0) < 0.05


def test_series_coefficient_generators_exact():
    # sin, Neumann and log(I + Z) coefficients are the correctly rounded
    # doubles of their rational values
    s, nm, lg = G.sin_coeffs(21), G.neumann_coeffs(9), G.log1p_coeffs(12)
    for k in range(22):
        want = Fraction((-1) ** (k // 2), math.factorial(k)) if k % 2 else Fraction(0)
        assert s[k] == float(want)
    assert np.all(nm == 1.0)
    assert lg[0] == 0.0 and all(lg[k] == float(Fraction((-1) ** (k + 1), k)) for k in range(1, 13))


@pytest.mark.parametrize("case", ["sin_lap2d", "neumann_band", "log1p_lap1d", "sin_rand"])
def test_series_mode_other_functions(case):
    # Algorithm 2 on other power series: ||f(Z) - F||_1 <= eps_tol against
    # scipy's dense sinm, inv(I - Z) and logm(I + Z)
    import scipy.linalg as sl

    if case == "sin_lap2d":
        Z, a, ref = G.laplacian_2d(10, 2.0), G.sin_coeffs(70), None
        ref = sl.sinm(Z.to_dense())
    elif case == "neumann_band":
        Z, a = G.random_banded(150, 3, 0.6, 0.5, seed=2), G.neumann_coeffs(220)
        ref = np.linalg.inv(np.eye(Z.n) - Z.to_dense())
    elif case == "log1p_lap1d":
        Z, a = G.laplacian_1d(120, 0.6), G.log1p_coeffs(220)
        ref = sl.logm(np.eye(Z.n) + Z.to_dense()).real
    else:
        Z, a = G.random_sparse(60, 0.1, 4, 0.5), G.sin_coeffs(70)
        ref = sl.sinm(Z.to_dense())
    for eps_tol in (1e-6, 1e-11):
        F, info, st, a1 = O.series(Z, a, eps_tol, 0.1)
        check_canonical(F)
        assert info["tail"] <= 0.5 * eps_tol
        err = O.norm1(F.to_dense() - ref)
        assert err <= eps_tol * 1.1 + 1e-13 * O.norm1(ref), (case, eps_tol, err, info["N"])
