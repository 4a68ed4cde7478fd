"""Exact-arithmetic pins for the oracle's filtering thresholds and Algorithm 1.

The oracle evaluates eqs. 21-28 and eq. 37 in floating point and runs
Algorithm 1 with a quantised candidate norm.  These tests tie those routines to
values derived without them:

- eqs. 21-26 and 28 recomputed in exact rationals from the same double inputs;
- d_k of eq. 24 and the weights of eq. 23 obtained a second way, as the exact
  first-order sensitivity of the Paterson-Stockmeyer result (eqs. 11-14) to
  the matrix removed at each filtered stage, by running the scheme on a scalar
  in dual numbers over the rationals (for a positive scalar and nonnegative
  coefficients every norm inequality of eqs. 19-26 holds with equality);
- alpha of Lemma 1 / eq. 37 checked against exact rational powers;
- Algorithm 1 (Section 3.1.1) rewritten from the paper with the exact 1-norm
  (exactly rounded column sums), compared with the oracle's integer-quantised
  norm on every pinned matrix, plus one constructed case inside the window
  where the two readings part.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from fps_inputs import generators as G

U = Fraction(1, 2 ** 53)


# ---------------------------------------------------------------------------
# eqs. 21-26 and 28 in exact rationals
# ---------------------------------------------------------------------------

def _schedule(m, s):
    N = m + 1
    q = s
    b = -(-N // q)
    g = 1 if N - q * (b - 1) == 1 else 0
    return N, q, b, g


def _exact_fnt(c, m, s, eps, z):
    """zeta_k (k = 2..q) and sigma_j (j = 0..b-1) of eq. 28, exactly."""
    N, q, b, g = _schedule(m, s)
    a = [abs(Fraction(float(c[k]))) if k <= m else Fraction(0) for k in range(q * b + q + 1)]
    Z = [Fraction(float(v)) for v in z]

    def beta(i, j):  # eq. 21, beta_{i,q} = 0
        return sum((a[i * q + k] * Z[k - j] for k in range(j, q)), Fraction(0))

    nB = [sum((a[i * q + j] * Z[j] for j in range(q)), Fraction(0)) for i in range(b)]  # eq. 25
    nS = [nB[b - 1]]  # eq. 26
    for i in range(1, b):
        nS.append(nB[b - 1 - i] + Z[q] * nS[i - 1])

    def S(j):
        return Fraction(0) if j < 0 else nS[j]

    M = q + b - 2 - g  # eq. 28
    zeta = {}
    for k in range(2, q + 1):
        d = sum((Z[q * (b - 1 - j)] * (beta(b - 1 - j, k) + Z[q - k] * S(j - 1)) for j in range(b)), Fraction(0))
        zeta[k] = Fraction(eps) / (d * M)
    sigma = {j: Fraction(eps) / (Z[q * (b - 1 - j)] * M) for j in range(b)}
    return zeta, sigma


@pytest.mark.parametrize("m,s,series", [(16, 4, "exp"), (30, 6, "exp"), (24, 5, "cos"), (40, 8, "exp"),
                                         (20, 4, "rand"), (21, 5, "rand"), (35, 3, "cos"), (9, 2, "exp"),
                                         (39, 7, "rand"), (12, 8, "exp")])
def test_fnt_thresholds_exact_rationals(m, s, series):
    rng = np.random.default_rng(1000 + 31 * m + s)
    if series == "exp":
        c = G.exp_coeffs(m)
    elif series == "cos":
        c = G.cos_coeffs(m)
    else:
        c = G.random_series_coeffs(m, rng)
    N, q, b, g = _schedule(m, s)
    assert b >= 2
    tmax = max(q, q * (b - 1))
    # positive norm bounds with the shape of ||Z^t||: gamma^t with noise
    gamma = float(rng.uniform(0.4, 2.5))
    z = np.array([1.0] + [gamma ** t * float(rng.uniform(0.5, 1.0)) for t in range(1, tmax + 1)])
    eps = float(10.0 ** rng.uniform(-14, -6))
    zeta, sigma = O.fnt_thresholds(c, m, s, eps, z)
    ez, es = _exact_fnt(c, m, s, eps, z)
    # every quantity is a sum of products of nonnegative doubles: the rounded
    # evaluation is within (operations) u of the exact value
    ops = 4 * (b + q) + 8
    for k in range(2, q + 1):
        err = abs(Fraction(float(zeta[k])) - ez[k])
        assert err <= ops * U * ez[k], (k, float(err / ez[k] / U))
    for j in range(b):
        err = abs(Fraction(float(sigma[j])) - es[j])
        assert err <= 4 * U * es[j], (j, float(err / es[j] / U))


# ---------------------------------------------------------------------------
# d_k and the Horner weights as first-order sensitivities of the scheme
# ---------------------------------------------------------------------------

class Dual:
    """a + b*e with e^2 = 0, over exact rationals."""

    __slots__ = ("a", "b")

    def __init__(self, a, b=Fraction(0)):
        self.a, self.b = Fraction(a), Fraction(b)

    def __add__(self, o):
        o = o if isinstance(o, Dual) else Dual(o)
        return Dual(self.a + o.a, self.b + o.b)

    __radd__ = __add__

    def __sub__(self, o):
        o = o if isinstance(o, Dual) else Dual(o)
        return Dual(self.a - o.a, self.b - o.b)

    def __mul__(self, o):
        o = o if isinstance(o, Dual) else Dual(o)
        return Dual(self.a * o.a, self.a * o.b + self.b * o.a)

    __rmul__ = __mul__


def _scalar_ps_with_removal(lam, c, m, s, where):
    """The PS scheme of eqs. 11-14 on the 1 x 1 matrix lam, exactly, with the
    matrix removed at one filtered stage set to the infinitesimal e: where =
    ("power", k) removes it from P_k, ("horner", j) from S_j.  Returns the
    result as a dual number and the number of filtered stages the scheme ran."""
    N, q, b, g = _schedule(m, s)
    a = [Fraction(float(c[k])) if k <= m else Fraction(0) for k in range(q * b + q + 1)]
    e = Dual(0, 1)
    P = [Dual(1), Dual(lam)]
    filtered = 0
    for k in range(2, q + 1):  # eq. 11
        x = Dual(lam) * P[k - 1]
        filtered += 1
        if where == ("power", k):
            x = x - e
        P.append(x)

    def B(i):  # eq. 13
        return sum((a[i * q + j] * P[j] for j in range(q)), Dual(0))

    S = B(b - 1)  # eq. 14
    start = 1
    if g:  # S_1 = B_{b-2} + a_{(b-1)q} P_q, no product and no filter
        S = B(b - 2) + a[(b - 1) * q] * P[q]
        start = 2
    for j in range(start, b):
        S = B(b - 1 - j) + P[q] * S
        filtered += 1
        if where == ("horner", j):
            S = S - e
    return S, filtered


@pytest.mark.parametrize("m,s,lam", [(16, 4, Fraction(3, 4)), (30, 6, Fraction(3, 2)), (20, 5, Fraction(5, 4)),
                                     (24, 5, Fraction(1, 2)), (13, 3, Fraction(7, 8)), (21, 4, Fraction(5, 8))])
def test_eq24_d_k_is_the_schemes_sensitivity(m, s, lam):
    # with Z = lam > 0 and |coefficients|, ||Z^t|| = lam^t exactly, and the
    # sensitivity of F to the removed power zeta_k is -d_k, to the removed
    # Horner term Sigma_j is -||Z^{q(b-1-j)}||: eq. 28 is eps / (that * M)
    c = np.abs(G.exp_coeffs(m)) if m != 24 else np.abs(G.cos_coeffs(m))
    N, q, b, g = _schedule(m, s)
    tmax = max(q, q * (b - 1))
    z = np.array([float(lam ** t) for t in range(tmax + 1)])
    assert all(Fraction(float(z[t])) == lam ** t for t in range(tmax + 1))  # exact in binary64
    eps = 1e-10
    zeta, sigma = O.fnt_thresholds(c, m, s, eps, z)
    for k in range(2, q + 1):
        F, M = _scalar_ps_with_removal(lam, c, m, s, ("power", k))
        d_k = -F.b
        assert M == q + b - 2 - g
        got_d = Fraction(eps) / (Fraction(float(zeta[k])) * M)
        assert abs(got_d - d_k) <= 64 * (b + q) * U * d_k, (k, float(got_d), float(d_k))
    for j in range(1 + g, b):
        F, M = _scalar_ps_with_removal(lam, c, m, s, ("horner", j))
        w = -F.b
        assert w == lam ** (q * (b - 1 - j))
        got_w = Fraction(eps) / (Fraction(float(sigma[j])) * M)
        assert abs(got_w - w) <= 8 * U * w


# ---------------------------------------------------------------------------
# Lemma 1 / eq. 37: alpha = max_{k=5..10} z_k^(1/k)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_eq37_alpha_exact(seed):
    rng = np.random.default_rng(70 + seed)
    n = 30
    Z = G.random_sparse(n, 0.15, seed=80 + seed, scale=float(rng.uniform(0.3, 1.5)))
    tmax = 24
    z = O.power_norm_bounds(Z, tmax)
    est = [O.normest1_power(Z, p)["est"] for p in range(11)]
    assert z[0] == 1.0 and all(z[i] == est[i] for i in range(1, 11))
    # z_i = alpha^i with alpha = max_{k=5..10} z_k^(1/k): in exact arithmetic,
    # z_i^k >= z_k^i for every k (alpha is at least every root) and
    # z_i^k <= z_k^i for the best k, each up to the rounding of pow
    cands = [(k, Fraction(float(est[k]))) for k in range(5, 11)]
    for i in range(11, tmax + 1):
        zi = Fraction(float(z[i]))
        lo = 1 - Fraction(8 * i, 2 ** 53)
        hi = 1 + Fraction(8 * i, 2 ** 53)
        for k, zk in cands:
            assert zi ** k >= zk ** i * lo ** k, (i, k)
        assert any(zi ** k <= zk ** i * hi ** k for k, zk in cands), i


# ---------------------------------------------------------------------------
# Algorithm 1 with the exact 1-norm against the oracle's quantised norm
# ---------------------------------------------------------------------------

def _alg1_exact(M, eps_g, e_r, max_iter=200):
    """Algorithm 1 as printed (Section 3.1.1), with c = ||c_i||_1 taken as the
    largest exactly rounded column sum.  The candidate matrix c_i loses the
    entries above each new threshold for good; c_0 = 1 only starts the loop.
    Returns (iterations, final threshold, dropped mask, final norm)."""
    absv = np.abs(np.asarray(M.val, dtype=np.float64))
    cols = np.asarray(M.col)
    cand = absv > 0
    target = eps_g * (1.0 + e_r)
    m_i = 1.0
    it = 0
    while True:
        t = eps_g / m_i
        cand = cand & (absv <= t)
        per_col = {}
        for p in np.nonzero(cand)[0]:
            per_col.setdefault(int(cols[p]), []).append(float(absv[p]))
        c = max((math.fsum(v) for v in per_col.values()), default=0.0)
        m_i = c / t
        it += 1
        if not (c > target):
            return it, t, cand, c
        if it >= max_iter:
            raise RuntimeError("no convergence")


def _oracle_dropped(M, F):
    kept = set()
    for r in range(F.n):
        for p in range(F.row_ptr[r], F.row_ptr[r + 1]):
            kept.add((r, int(F.col[p])))
    mask = np.zeros(M.nnz, dtype=bool)
    for r in range(M.n):
        for p in range(M.row_ptr[r], M.row_ptr[r + 1]):
            mask[p] = (r, int(M.col[p])) not in kept
    return mask


def _compare_alg1(M, eps_g, e_r):
    F, st = O.alg1_filter(M, eps_g, e_r)
    it, t, drop, c = _alg1_exact(M, eps_g, e_r)
    assert st["iters"] == it, (st["iters"], it)
    if it == 1:
        assert st["threshold"] == t == eps_g
    else:  # thresholds eps_g / m differ only through the quantised norm
        assert abs(st["threshold"] - t) <= 2.0 ** -30 * t
    np.testing.assert_array_equal(_oracle_dropped(M, F), drop)
    # the quantised norm bounds the exact one from above, within 2^-40 eps_g
    # per candidate entry of the column
    assert c <= st["dropped"] * (1 + 1e-15) + 1e-300
    assert st["dropped"] <= c + M.n * 2.0 ** -40 * eps_g
    return it


def _alg1_cases():
    cases = []
    for seed in range(6):  # random near-sparse matrices with many small entries
        rng = np.random.default_rng(40 + seed)
        n = int(rng.integers(5, 60))
        d = np.where(rng.random((n, n)) < 0.3, 10.0 ** rng.uniform(-16, -9, (n, n)), 0.0)
        d *= np.where(rng.random((n, n)) < 0.5, -1.0, 1.0)
        cases.append((G.from_dense(d), float(10.0 ** rng.uniform(-13, -10)), 0.1))
    eps = 1e-10
    d = np.zeros((12, 12))
    d[:10, 3] = 0.5 * eps
    d[11, 11] = 1.0
    cases.append((G.from_dense(d), eps, 0.1))
    d = np.zeros((25, 25))
    d[:20, 0] = eps * 2.0 ** -np.arange(1, 21)
    d[24, 24] = 1.0
    cases.append((G.from_dense(d), eps, 0.1))
    cases.append((G.diagonal([0.3 * eps, 0.9 * eps, 2 * eps]), eps, 0.0))
    d = np.zeros((3, 3))
    d[0, 1], d[1, 1], d[2, 2] = eps, 0.2 * eps, 1.0
    cases.append((G.from_dense(d), eps, 0.1))
    return cases


@pytest.mark.parametrize("idx", range(10))
def test_alg1_quantised_norm_matches_exact_norm(idx):
    M, eps_g, e_r = _alg1_cases()[idx]
    _compare_alg1(M, eps_g, e_r)


@pytest.mark.parametrize("case", ["c1", "lap2d", "band", "cos3d"])
def test_alg1_stages_of_adaptive_runs_match_exact_norm(case):
    # every filtered stage of the adaptive scheme (eq. 28 thresholds), with the
    # unfiltered product the oracle forms, filtered both ways
    if case == "c1":
        Z, c, m, s = G.laplacian_1d(300, 1.0), G.exp_coeffs(16), 16, 4
    elif case == "lap2d":
        Z, c, m, s = G.laplacian_2d(18, 2.0), G.exp_coeffs(30), 30, 6
    elif case == "band":
        Z, c, m, s = G.random_banded(200, 3, 0.6, 1.5, seed=5), G.exp_coeffs(20), 20, 4
    else:
        Z, c, m, s = G.laplacian_3d_perturbed(5, seed=3, norm1=1.5), G.cos_coeffs(24), 24, 5
    sc = O.schedule(m, s)
    q, b = sc["q"], sc["b"]
    from oracle.bound import power_norms
    z = power_norms(Z, max(q, q * (b - 1)))
    eps, e_r = 1e-11, 0.1
    zeta, sigma = O.fnt_thresholds(c, m, s, eps, z)
    iters = []
    P = {1: Z}
    for k in range(2, q + 1):
        pre = O.spgemm(Z, P[k - 1], None, 0.0)[0]
        iters.append(_compare_alg1(pre, float(zeta[k]), e_r))
        P[k] = O.alg1_filter(pre, float(zeta[k]), e_r)[0]

    def block(i, jmax):
        idx = [j for j in range(jmax + 1) if i * q + j <= m and c[i * q + j] != 0.0]
        return O.axpy(Z.n, [c[i * q + j] for j in idx], [None if j == 0 else P[j] for j in idx])[0]

    S = block(b - 2, q) if sc["g"] else block(b - 1, q - 1)
    for j in range(sc["start"], b):
        pre = O.spgemm(P[q], S, block(b - 1 - j, q - 1), 0.0)[0]
        iters.append(_compare_alg1(pre, float(sigma[j]), e_r))
        S = O.alg1_filter(pre, float(sigma[j]), e_r)[0]
    assert max(iters) >= 1
    # the stagewise replay reproduces the oracle's adaptive scheme
    F, _, _ = O.filtered_ps_adaptive(Z, c, m, s, eps, e_r, z)
    assert np.array_equal(F.row_ptr, S.row_ptr) and np.array_equal(F.col, S.col)
    assert np.array_equal(F.val.view(np.uint64), S.val.view(np.uint64))


def test_alg1_quantisation_window():
    # Inside the window the readings part: a column whose exact candidate
    # norm is at most the target, but whose quantised norm (each |x| rounded
    # up to a multiple of 2^-40 eps_g) exceeds it.  Exact: one iteration,
    # both entries dropped.  Quantised: a second iteration with a threshold
    # just below eps_g that protects the large entry, which is then kept (the
    # quantised reading drops a subset: its error stays within the budget).
    eps_g, e_r = 1.0, 0.0
    u = 1.0 - 2.0 ** -42
    v = 2.0 ** -42 - 2.0 ** -60
    d = np.zeros((3, 3))
    d[0, 0], d[1, 0], d[2, 2] = u, v, 4.0
    M = G.from_dense(d)
    it, t, drop, c = _alg1_exact(M, eps_g, e_r)
    assert it == 1 and t == 1.0 and drop.sum() == 2 and c <= eps_g
    F, st = O.alg1_filter(M, eps_g, e_r)
    assert st["iters"] == 2 and st["threshold"] < u
    assert F.nnz == 2 and u in F.val
    assert st["dropped"] <= eps_g * (1 + e_r)
    # the window: exact norm within (candidates in the column) * 2^-40 eps_g
    # below the target
    assert eps_g * (1 + e_r) - c <= 2 * 2.0 ** -40 * eps_g


def test_alg1_refuses_columns_beyond_exact_integer_sums():
    # 2^24 rows or more: a column could hold 2^24 candidates, whose integer
    # sums (at most 2^40 + 1 each) would wrap in 64 bits
    n = 1 << 24
    M = G.CSR(n, np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0))
    with pytest.raises(RuntimeError):
        O.alg1_filter(M, 1e-10, 0.1)
