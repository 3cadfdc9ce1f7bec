"""Seeded synthetic inputs for kernel-ridge systems (K + lambda I) x = b.

This module only draws random data of the shapes and distributions used by the
workloads (points X, right-hand sides b, Gaussian test matrices Omega,
regularisation grids).  It holds none of the solver's arithmetic: no kernel
evaluation, no products with K, no factorisations.  Both the CPU oracle and the
GPU library consume what it returns, so neither depends on the other.

The paper (section "Problem Classes", eq. rlaopt-krr) defines the system class
but fixes no kernel data set; every recipe below is synthetic, with the
distribution stated per workload.  All draws use numpy's PCG64 generator
(numpy.random.default_rng) in float64; the sketch matrix uses the seed offset
by 1000 so that it is independent of the data draw.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

RBF = 0
LAPLACIAN = 1

OMEGA_SEED_OFFSET = 1000


@dataclass
class Workload:
    """One synthetic kernel-ridge problem.

    X        (n, d) float64 points, row-major.
    B        (n, nrhs) float64 right-hand sides.
    lambdas  regularisation values; the solve has len(lambdas)*nrhs columns,
             column c using lambdas[c // nrhs] and B[:, c % nrhs].
    kind     RBF or LAPLACIAN; sigma the bandwidth.
    r        Nystrom sketch size.
    tol      stopping tolerance on the relative residual.
    prec     "fp64" | "fp32" | "bf16x3": arithmetic of the kernel product.
    refine_every  inner iterations between FP64 residual refinements (0 = off).
    Xval, yval  optional validation split (differentiation workload).
    """

    name: str
    X: np.ndarray
    B: np.ndarray
    lambdas: list
    kind: int
    sigma: float
    r: int
    tol: float
    prec: str
    refine_every: int = 0
    seed: int = 0
    Xval: np.ndarray | None = None
    yval: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def d(self) -> int:
        return self.X.shape[1]


def standardised_gaussian(rng: np.random.Generator, n: int, d: int) -> np.ndarray:
    """X ~ N(0,1) i.i.d., then each column shifted/scaled to mean 0, std 1."""
    X = rng.standard_normal((n, d))
    X -= X.mean(axis=0, keepdims=True)
    X /= X.std(axis=0, keepdims=True)
    return X


def gaussian_test_matrix(n: int, r: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Omega ~ N(0,1)^{n x r}, the random test matrix of the Nystrom sketch."""
    rng = np.random.default_rng(seed + OMEGA_SEED_OFFSET)
    return rng.standard_normal((n, r), dtype=dtype)


def small_problem(n: int, d: int, seed: int = 0, nrhs: int = 1, kind: int = RBF,
                  sigma: float | None = None, lam: float | None = None, r: int = 16,
                  tol: float = 1e-10, prec: str = "fp64") -> Workload:
    """Generic small case in the recipe of the plain FP64 workload (used by tests)."""
    rng = np.random.default_rng(seed)
    X = standardised_gaussian(rng, n, d)
    W = rng.standard_normal((d, nrhs)) / math.sqrt(d)
    B = np.sin(X @ W) + 0.1 * rng.standard_normal((n, nrhs))
    sigma = math.sqrt(d) if sigma is None else sigma
    lam = 1e-3 * n if lam is None else lam
    return Workload(f"small_n{n}_d{d}", X, B, [lam], kind, sigma, min(r, n), tol, prec, seed=seed)


def plain_fp64(seed: int = 0, n: int = 2000) -> Workload:
    """Plain NysPCG in FP64: n=2000, d=10, standardised Gaussian X, RBF sigma=sqrt(d),
    b = sin(Xw) + 0.1 N(0,1) with w ~ N(0, I/d), lambda = 1e-3 n, r = 50, tol 1e-8."""
    d = 10
    rng = np.random.default_rng(seed)
    X = standardised_gaussian(rng, n, d)
    w = rng.standard_normal(d) / math.sqrt(d)
    b = np.sin(X @ w) + 0.1 * rng.standard_normal(n)
    return Workload("plain_fp64_n2000_d10", X, b[:, None], [1e-3 * n], RBF, math.sqrt(d),
                    50, 1e-8, "fp64", seed=seed)


def matrix_free_fp32(seed: int = 0, n: int = 200_000) -> Workload:
    """Plain NysPCG, FP32 matrix-free: n=2e5, d=20; 19 N(0,1) columns plus one
    Student-t (nu=3) column (5% of 20 columns, the last); b = tanh(Xw) + 0.05 N(0,1);
    RBF sigma = sqrt(20); lambda = 1e-6 n; r = 200; tol 1e-6."""
    d = 20
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    n_heavy = int(math.ceil(0.05 * d))
    X[:, d - n_heavy:] = rng.standard_t(3.0, size=(n, n_heavy))
    w = rng.standard_normal(d) / math.sqrt(d)
    b = np.tanh(X @ w) + 0.05 * rng.standard_normal(n)
    return Workload("matrix_free_fp32_n200k_d20", X, b[:, None], [1e-6 * n], RBF, math.sqrt(d),
                    200, 1e-6, "fp32", seed=seed)


def precision_variant(seed: int = 0, n: int = 500_000) -> Workload:
    """Precision variant: n=5e5, d=32, standardised Gaussian X, b = sin(Xw)+0.1 noise,
    RBF sigma = sqrt(32), lambda = 1e-5 n, r = 400, BF16x3 product, FP32 CG and an FP64
    residual refinement every 20 inner iterations."""
    d = 32
    rng = np.random.default_rng(seed)
    X = standardised_gaussian(rng, n, d)
    w = rng.standard_normal(d) / math.sqrt(d)
    b = np.sin(X @ w) + 0.1 * rng.standard_normal(n)
    return Workload("precision_bf16x3_n500k_d32", X, b[:, None], [1e-5 * n], RBF, math.sqrt(d),
                    400, 1e-6, "bf16x3", refine_every=20, seed=seed)


def differentiation(seed: int = 0, n_train: int = 100_000, n_val: int = 20_000) -> Workload:
    """Differentiation workload: 1e5 train + 2e4 validation rows of one standardised
    Gaussian draw with d=16, y = sin(Xw) + 0.1 noise, Laplacian kernel sigma0 = 4,
    lambda0 = 1e-3 n_train, r = 200, FP64."""
    d = 16
    rng = np.random.default_rng(seed)
    Xall = standardised_gaussian(rng, n_train + n_val, d)
    w = rng.standard_normal(d) / math.sqrt(d)
    yall = np.sin(Xall @ w) + 0.1 * rng.standard_normal(n_train + n_val)
    X, Xv = Xall[:n_train], Xall[n_train:]
    y, yv = yall[:n_train], yall[n_train:]
    return Workload("differentiation_laplacian_n100k_d16", X, y[:, None], [1e-3 * n_train],
                    LAPLACIAN, 4.0, 200, 1e-10, "fp64", seed=seed, Xval=Xv, yval=yv)


def batched_lambda_grid(seed: int = 0, n: int = 1_000_000, nrhs: int = 64, nlam: int = 8,
                        r: int = 500) -> Workload:
    """Batching workload: n=1e6, d=16, standardised Gaussian X, RBF sigma = 4,
    64 right-hand sides b_c = sign(X w_c) (w_c ~ N(0, I), sign(0) = +1), 8 lambdas
    log-spaced over [1e-7 n, 1e-3 n], shared sketch r = 500, BF16x3, tol 1e-6."""
    d = 16
    rng = np.random.default_rng(seed)
    X = standardised_gaussian(rng, n, d)
    Wc = rng.standard_normal((d, nrhs))
    B = np.where(X @ Wc >= 0.0, 1.0, -1.0)
    lams = list(np.logspace(math.log10(1e-7 * n), math.log10(1e-3 * n), nlam))
    return Workload(f"batched_{nrhs}rhs_x_{nlam}lam_n{n}_d{d}", X, B, lams, RBF, 4.0, r, 1e-6,
                    "bf16x3", refine_every=20, seed=seed)


WORKLOADS = {
    "plain_fp64": plain_fp64,
    "matrix_free_fp32": matrix_free_fp32,
    "precision_variant": precision_variant,
    "differentiation": differentiation,
    "batched_lambda_grid": batched_lambda_grid,
}
