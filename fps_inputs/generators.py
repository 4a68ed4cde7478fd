"""Seeded generators for the matrices and series the method is run on.

Every generator is deterministic in its arguments (numpy PCG64 through
``numpy.random.default_rng``).  Matrices come out in canonical CSR: int64 row
pointers, int32 column indices sorted and unique within each row, float64
values with no stored zeros.

The workload shapes follow the problem statement of the paper (a sparse Z and
the coefficients of a truncated power series, eqs. 1 and 8) and the synthetic
stand-ins used for measurement: 1D/2D/3D Dirichlet Laplacians, random banded
matrices (the paper's second test set, Section 4), and mixes of those.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction

import numpy as np
import scipy.sparse as sp


@dataclass
class CSR:
    """Canonical CSR matrix held in host memory (numpy arrays)."""

    n: int
    row_ptr: np.ndarray  # int64, n+1
    col: np.ndarray  # int32, nnz
    val: np.ndarray  # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n), dtype=np.float64)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        d[rows, self.col] = self.val
        return d


def _from_scipy(m: sp.spmatrix) -> CSR:
    m = sp.csr_matrix(m, dtype=np.float64)
    m.sum_duplicates()
    m.eliminate_zeros()
    m.sort_indices()
    return CSR(
        n=m.shape[0],
        row_ptr=np.ascontiguousarray(m.indptr, dtype=np.int64),
        col=np.ascontiguousarray(m.indices, dtype=np.int32),
        val=np.ascontiguousarray(m.data, dtype=np.float64),
    )


def from_dense(d: np.ndarray) -> CSR:
    return _from_scipy(sp.csr_matrix(np.asarray(d, dtype=np.float64)))


def _colmax_abs(m: sp.spmatrix) -> float:
    return float(np.max(np.asarray(abs(m).sum(axis=0)).ravel()))


def _scaled(m: sp.spmatrix, target_norm1: float) -> CSR:
    """Scale so that the largest column absolute sum equals ``target_norm1``."""
    m = sp.csr_matrix(m, dtype=np.float64)
    m.sum_duplicates()
    m.eliminate_zeros()
    return _from_scipy(m * (target_norm1 / _colmax_abs(m)))


def _tridiag(n: int) -> sp.spmatrix:
    e = np.ones(n)
    return sp.diags([e[:-1], -2.0 * e, e[:-1]], [-1, 0, 1], shape=(n, n), format="csr")


def laplacian_1d(n: int = 1000, norm1: float = 1.0) -> CSR:
    """alpha * tridiag(1,-2,1), alpha chosen so that ||Z||_1 = norm1."""
    return _scaled(_tridiag(n), norm1)


def _laplacian_nd(sides) -> sp.spmatrix:
    """Kronecker sum of tridiag(1,-2,1) over the grid dimensions (Dirichlet)."""
    mats = [_tridiag(s) for s in sides]
    out = None
    for d in range(len(sides)):
        term = None
        for e in range(len(sides)):
            f = mats[e] if e == d else sp.identity(sides[e], format="csr")
            term = f if term is None else sp.kron(term, f, format="csr")
        out = term if out is None else out + term
    return sp.csr_matrix(out)


def laplacian_2d(side: int = 200, norm1: float = 2.0) -> CSR:
    """5-point Dirichlet Laplacian on a side x side grid, scaled to ||Z||_1 = norm1."""
    return _scaled(_laplacian_nd([side, side]), norm1)


def laplacian_3d_perturbed(side: int = 50, extra_per_row: int = 2, sigma: float = 0.1,
                           norm1: float = 1.5, seed: int = 3) -> CSR:
    """7-point 3D Laplacian plus a symmetric random long-range perturbation.

    For each row i, ``extra_per_row`` columns j != i are drawn uniformly and
    R[i, j] = v with v ~ N(0, sigma^2); the perturbation R + R^T (duplicates
    summed) is added and the sum is scaled to ||Z||_1 = norm1.
    """
    rng = np.random.default_rng(seed)
    lap = _laplacian_nd([side, side, side])
    n = lap.shape[0]
    rows = np.repeat(np.arange(n), extra_per_row)
    cols = rng.integers(0, n - 1, size=n * extra_per_row)
    cols = cols + (cols >= rows)  # uniform over j != i
    vals = rng.normal(0.0, sigma, size=n * extra_per_row)
    r = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    return _scaled(lap + r + r.T, norm1)


def random_banded(n: int, half_bw: int, density: float = 0.6, norm1: float | None = None,
                  seed: int = 0) -> CSR:
    """Banded matrix: each (i, j) with |i-j| <= half_bw (diagonal included) is
    kept with probability ``density`` and gets an N(0, 1) value; optionally
    scaled to ||Z||_1 = norm1."""
    rng = np.random.default_rng(seed)
    offs = np.arange(-half_bw, half_bw + 1)
    rows = np.repeat(np.arange(n), offs.size)
    cols = rows + np.tile(offs, n)
    ok = (cols >= 0) & (cols < n)
    rows, cols = rows[ok], cols[ok]
    keep = rng.random(rows.size) < density
    vals = rng.standard_normal(rows.size)
    rows, cols, vals = rows[keep], cols[keep], vals[keep]
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    if norm1 is None:
        return _from_scipy(m)
    return _scaled(m, norm1)


def banded_sweep_matrix(half_bw: int, n: int = 1000, seed: int = 0) -> CSR:
    """The paper's second test set (Section 4): n x n, equal lower and upper
    bandwidth, every in-band entry N(0, 1)."""
    return random_banded(n, half_bw, density=1.0, norm1=None, seed=seed)


def shift_matrix(n: int, k: int = 1, value: float = 1.0) -> CSR:
    """value * J^k with J the upper shift (ones on the first superdiagonal)."""
    if k >= n:
        return CSR(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    return _from_scipy(sp.diags([np.full(n - k, value)], [k], shape=(n, n), format="csr"))


def diagonal(lams) -> CSR:
    lams = np.asarray(lams, dtype=np.float64)
    return _from_scipy(sp.diags([lams], [0], format="csr"))


def random_sparse(n: int, density: float, seed: int, scale: float = 1.0,
                  strictly_upper: bool = False) -> CSR:
    """Unstructured nonsymmetric random sparse matrix with N(0, scale^2) entries."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    if strictly_upper:
        mask &= np.triu(np.ones((n, n), dtype=bool), 1)
    d = np.where(mask, rng.standard_normal((n, n)) * scale, 0.0)
    return from_dense(d)


def empty_matrix(n: int) -> CSR:
    return CSR(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))


# ----------------------------------------------------------------------------
# Series coefficients (correctly rounded doubles of the exact rationals)
# ----------------------------------------------------------------------------

def exp_coeffs(m: int) -> np.ndarray:
    """c_k = 1/k! (exponential series, eq. 38)."""
    return np.array([float(Fraction(1, math.factorial(k))) for k in range(m + 1)])


def cos_coeffs(m: int) -> np.ndarray:
    """c_{2k} = (-1)^k/(2k)!, odd coefficients 0 (cosine series, eq. 40)."""
    c = np.zeros(m + 1)
    for k in range(0, m + 1, 2):
        c[k] = float(Fraction((-1) ** (k // 2), math.factorial(k)))
    return c


def sin_coeffs(m: int) -> np.ndarray:
    """c_{2k+1} = (-1)^k/(2k+1)!, even coefficients 0 (sine series)."""
    c = np.zeros(m + 1)
    for k in range(1, m + 1, 2):
        c[k] = float(Fraction((-1) ** (k // 2), math.factorial(k)))
    return c


def neumann_coeffs(m: int) -> np.ndarray:
    """c_k = 1 (Neumann series of (I - Z)^{-1}, convergent for rho(Z) < 1)."""
    return np.ones(m + 1)


def log1p_coeffs(m: int) -> np.ndarray:
    """c_0 = 0, c_k = (-1)^(k+1)/k (log(I + Z), convergent for rho(Z) < 1)."""
    c = np.zeros(m + 1)
    for k in range(1, m + 1):
        c[k] = float(Fraction((-1) ** (k + 1), k))
    return c


def random_series_coeffs(m: int, rng: np.random.Generator) -> np.ndarray:
    """c_k = x_k / k! with x_k ~ N(0, 1), correctly rounded."""
    x = rng.standard_normal(m + 1)
    return np.array([float(Fraction(float(x[k])) / math.factorial(k)) for k in range(m + 1)])


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def config1():
    """1D Laplacian n=1000, ||Z||_1=1, exp m=16, s=4, tau=1e-14*||Z||_1."""
    z = laplacian_1d(1000, 1.0)
    return dict(name="lap1d_n1000_exp_m16_s4", Z=z, coeffs=exp_coeffs(16), m=16, s=4, tau=1e-14)


def config2(side: int = 200):
    """2D 5-point Laplacian (side^2 unknowns), ||Z||_1=2, exp m=30, s=6, tau=1e-12."""
    z = laplacian_2d(side, 2.0)
    return dict(name=f"lap2d_n{side * side}_exp_m30_s6", Z=z, coeffs=exp_coeffs(30), m=30, s=6,
                tau=1e-12)


def config3(side: int = 50, seed: int = 3):
    """3D 7-point Laplacian + random links, ||Z||_1=1.5, cos m=24, s=5, tau=1e-12."""
    z = laplacian_3d_perturbed(side, seed=seed)
    return dict(name=f"lap3d_pert_n{side ** 3}_cos_m24_s5", Z=z, coeffs=cos_coeffs(24), m=24,
                s=5, tau=1e-12)


def batch_instances(count: int = 512, seed: int = 4, n_lo: int = 500, n_hi: int = 20000, m: int = 20):
    """Uneven batch: n log-uniform in [n_lo, n_hi], half-bandwidth in {1..5},
    in-band density 0.6, N(0,1) entries, ||Z||_1 ~ U(0.5, 2), exp series,
    tau = 1e-12 * ||Z||_1."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        w = int(rng.integers(1, 6))
        nrm = float(rng.uniform(0.5, 2.0))
        s_seed = int(rng.integers(0, 2**63 - 1))
        z = random_banded(n, w, 0.6, nrm, s_seed)
        out.append(dict(name=f"band_{i}", Z=z, coeffs=exp_coeffs(m), m=m, tau=1e-12 * nrm,
                        n=n, half_bw=w, norm1=nrm))
    return out


def serving_requests(count: int, seed: int = 5, n_lo: int = 1000, n_hi: int = 60000):
    """Mixed request stream: n log-uniform, half 2D Laplacians (side round(sqrt n)),
    half random banded; exp / cos / random series in equal shares; m in U{12..30};
    tau = 1e-12; ||Z||_1 ~ U(0.5, 2)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        nrm = float(rng.uniform(0.5, 2.0))
        m = int(rng.integers(12, 31))
        fn = int(rng.integers(0, 3))
        if rng.random() < 0.5:
            side = max(2, int(round(math.sqrt(n))))
            z = laplacian_2d(side, nrm)
            kind = "lap2d"
        else:
            w = int(rng.integers(1, 6))
            z = random_banded(n, w, 0.6, nrm, int(rng.integers(0, 2**63 - 1)))
            kind = "banded"
        if fn == 0:
            c, fname = exp_coeffs(m), "exp"
        elif fn == 1:
            c, fname = cos_coeffs(m), "cos"
        else:
            c, fname = random_series_coeffs(m, rng), "rand"
        out.append(dict(name=f"req_{i}_{kind}_{fname}", Z=z, coeffs=c, m=m, tau=1e-12, kind=kind,
                        fn=fname, norm1=nrm))
    return out
