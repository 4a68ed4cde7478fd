"""The paper's a-posteriori bound on the error that filtering introduces.

Test infrastructure only (see the package docstring).

Given the 1-norms of the dropped matrices recorded by the oracle (zeta_k for
the powers, Sigma_j for the Horner steps) and norms ||Z^t||, this evaluates the
first-order bound of Section 3.1.3:

    ||Delta S_{b-1}|| <= sum_{k=2..q} d_k ||zeta_k||
                          + sum_{filtered steps j} ||Z^{q(b-1-j)}|| ||Sigma_j||     (eq. 23)

with d_k from eq. 24, beta_{i,j} from eq. 21 and the block / Horner-state norm
bounds of eqs. 25-26.  The sum over j runs over the Horner steps that are
actually filtered (j = 1+g .. b-1): the shortcut step of eq. 14 (g = 1) drops
nothing, which is how the upper limit b-1-g of eq. 23 is read here.
"""

from __future__ import annotations

import numpy as np


def power_norms(Z, tmax: int, exact_limit: int = 1500) -> np.ndarray:
    """z[t] >= ||Z^t||_1 for t = 0..tmax.

    For n <= exact_limit the powers are formed densely (their rounding is far
    below any tolerance used with them); otherwise the submultiplicative bound
    ||Z||_1^t is used (Section 2.2, after eq. 9)."""
    z = np.zeros(tmax + 1)
    z[0] = 1.0
    if Z.n <= exact_limit:
        d = Z.to_dense()
        p = np.eye(Z.n)
        for t in range(1, tmax + 1):
            p = p @ d
            z[t] = float(np.max(np.sum(np.abs(p), axis=0))) if Z.n else 0.0
        return z
    cs = np.zeros(Z.n)
    np.add.at(cs, Z.col, np.abs(Z.val))
    z1 = float(cs.max()) if Z.n else 0.0
    for t in range(1, tmax + 1):
        z[t] = z1 ** t
    return z


def filtering_bound(coeffs, m: int, s: int, stats, z) -> dict:
    """Evaluate eq. 23 from the per-stage dropped 1-norms in ``stats``.

    ``z[t]`` must bound ||Z^t||_1 for t up to q*(b-1).  Returns the bound and
    its pieces."""
    c = np.asarray(coeffs, dtype=np.float64)
    N = m + 1
    q = s
    b = -(-N // q)
    g = 1 if N - q * (b - 1) == 1 else 0

    def a(k):
        return abs(float(c[k])) if 0 <= k <= m else 0.0

    def zn(t):
        return float(z[t])

    # eq. 21: beta_{i,j} = sum_{k=j}^{q-1} |a_{iq+k}| ||Z^{k-j}||;  beta_{i,q} = 0
    def beta(i, j):
        if j >= q:
            return 0.0
        return sum(a(i * q + k) * zn(k - j) for k in range(j, q))

    # eq. 25: ||B_i|| <= sum_{j<q} |a_{iq+j}| ||Z^j||
    nb = [sum(a(i * q + j) * zn(j) for j in range(q)) for i in range(b)]
    # eq. 26: ||S_0|| = ||B_{b-1}||, ||S_i|| <= ||B_{b-1-i}|| + ||Z^q|| ||S_{i-1}||
    ns = [0.0] * b
    ns[0] = nb[b - 1]
    for i in range(1, b):
        ns[i] = nb[b - 1 - i] + zn(q) * ns[i - 1]

    def s_norm(j):  # ||S_{j}|| with ||S_{-1}|| = 0
        return 0.0 if j < 0 else ns[j]

    # eq. 24: d_k = sum_{j=0}^{b-1} ||Z^{q(b-1-j)}|| (beta_{b-1-j,k} + ||Z^{q-k}|| ||S_{j-1}||)
    d = {}
    for k in range(2, q + 1):
        d[k] = sum(zn(q * (b - 1 - j)) * (beta(b - 1 - j, k) + zn(q - k) * s_norm(j - 1)) for j in range(b))

    zeta = {st["index"]: st["dropped_1norm"] for st in stats if st["kind"] == 0}
    sigma = {st["index"]: st["dropped_1norm"] for st in stats if st["kind"] == 3}
    power_part = sum(d[k] * zeta.get(k, 0.0) for k in range(2, q + 1))
    horner_part = sum(zn(q * (b - 1 - j)) * sigma.get(j, 0.0) for j in range(1 + g, b))
    return dict(bound=power_part + horner_part, power_part=power_part, horner_part=horner_part, d=d,
                q=q, b=b, g=g)


def rounding_slack(coeffs, m: int, z1: float) -> float:
    """A generous allowance for floating-point rounding in either evaluation:
    100 (m+1) u sum_k |c_k| ||Z||_1^k with u = 2^-53."""
    c = np.asarray(coeffs, dtype=np.float64)
    u = 2.0 ** -53
    return 100.0 * (m + 1) * u * float(sum(abs(c[k]) * z1 ** k for k in range(m + 1)))
