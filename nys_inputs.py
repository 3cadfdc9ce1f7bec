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


# ----------------------------------------------------------------------------- ridge regression

def fwht(A: np.ndarray) -> np.ndarray:
    """Unnormalised fast Walsh-Hadamard transform of the columns of A (axis 0 of
    length 2^k): H A with H_ij = (-1)^popcount(i & j)."""
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    if n & (n - 1):
        raise ValueError("length must be a power of two")
    rest = A.shape[1:]
    h = 1
    while h < n:
        B = A.reshape((n // (2 * h), 2, h) + rest)
        a, b = B[:, 0].copy(), B[:, 1].copy()
        B[:, 0], B[:, 1] = a + b, a - b
        A = B.reshape((n,) + rest)
        h *= 2
    return A


def sorf_columns(n: int, r: int, signs: np.ndarray) -> np.ndarray:
    """The first r columns of the n x n orthogonal matrix H D1 H D2 H D3 (H the
    normalised Walsh-Hadamard matrix, D_i = diag(signs[i]) with +-1 entries): the SORF
    construction of Yu et al. (2016), the generator the paper names for the ridge
    data's orthonormal factors."""
    M = np.zeros((n, r))
    M[np.arange(r), np.arange(r)] = signs[2][:r]
    s = 1.0 / math.sqrt(n)
    M = fwht(M) * s
    M *= signs[1][:, None]
    M = fwht(M) * s
    M *= signs[0][:, None]
    return fwht(M) * s


@dataclass
class RidgeProblem:
    """Ridge regression data of eq. experiment-ridge-data: X = U Sigma_alpha V^T with
    Sigma_alpha = diag(i^(-alpha/2)), i = 1..min(n, p), and y = U g / |g|."""
    X: np.ndarray
    y: np.ndarray
    U: np.ndarray
    V: np.ndarray
    sigma: np.ndarray
    alpha: float
    seed: int


def ridge_problem(n: int, p: int, alpha: float, seed: int = 0) -> RidgeProblem:
    """n >= p, both powers of two; U (n x r) and V (p x r), r = min(n, p), are the first
    columns of independent SORF matrices, g ~ N(0, I_r)."""
    if n < p:
        raise ValueError("the paper's ridge problems have n >= p")
    rng = np.random.default_rng(seed)
    r = min(n, p)
    su = rng.choice(np.array([-1.0, 1.0]), size=(3, n))
    sv = rng.choice(np.array([-1.0, 1.0]), size=(3, p))
    g = rng.standard_normal(r)
    U = sorf_columns(n, r, su)
    V = sorf_columns(p, r, sv)
    sig = np.arange(1, r + 1, dtype=np.float64) ** (-alpha / 2.0)
    X = (U * sig) @ V.T
    y = U @ (g / np.linalg.norm(g))
    return RidgeProblem(np.ascontiguousarray(X), y, U, V, sig, alpha, seed)


def ridge_problem_device(n: int, p: int, alpha: float, seed: int, device):
    """ridge_problem's X and y built on a GPU with torch in float64 (the paper's sizes,
    n = p = 2^16, are beyond host generation): the same sign and g draws from the same
    numpy generator, the same Walsh-Hadamard stages and the same product, so the result
    equals the host version up to rounding order.  Returns (X, y) as device tensors."""
    import torch

    if n < p:
        raise ValueError("the paper's ridge problems have n >= p")
    rng = np.random.default_rng(seed)
    r = min(n, p)
    su = rng.choice(np.array([-1.0, 1.0]), size=(3, n))
    sv = rng.choice(np.array([-1.0, 1.0]), size=(3, p))
    g = rng.standard_normal(r)

    def fwht_(A):
        m = A.shape[0]
        h = 1
        while h < m:
            B = A.view(m // (2 * h), 2, h, A.shape[1])
            a = B[:, 0].clone()
            B[:, 0].add_(B[:, 1])
            B[:, 1].neg_().add_(a)
            del a
            h *= 2
        return A

    def sorf(m, signs):
        M = torch.zeros((m, r), dtype=torch.float64, device=device)
        M[torch.arange(r, device=device), torch.arange(r, device=device)] = torch.from_numpy(signs[2][:r]).to(device)
        s = 1.0 / math.sqrt(m)
        fwht_(M).mul_(s)
        M.mul_(torch.from_numpy(signs[1]).to(device)[:, None])
        fwht_(M).mul_(s)
        M.mul_(torch.from_numpy(signs[0]).to(device)[:, None])
        return fwht_(M).mul_(s)

    gt = torch.from_numpy(g / np.linalg.norm(g)).to(device)
    U = sorf(n, su)
    y = U @ gt
    U.mul_(torch.arange(1, r + 1, dtype=torch.float64, device=device).pow_(-alpha / 2.0))
    V = sorf(p, sv)
    X = U @ V.T
    del U, V
    return X.contiguous(), y


# ----------------------------------------------------------------------------- bounded elastic net

@dataclass
class ElasticNetProblem:
    """Bounded elastic net data (eq. experiment-bounded-en): dense random-feature
    matrix X (n x p), centred and scaled target y, lam1 = lam2 = 0.1 lam_max with
    lam_max = |X^T (y - ybar)|_inf / n."""
    X: np.ndarray
    y: np.ndarray
    lam1: float
    lam2: float
    seed: int


def elastic_net_problem(n: int, d_in: int, p: int, seed: int = 0) -> ElasticNetProblem:
    """Synthetic stand-in for the paper's dense random-feature problems (its data
    table: standardised inputs, Gaussian random features): inputs Z (n x d_in)
    column-standardised N(0, 1); features X = sqrt(2/p) cos(Z W / sqrt(d_in) + c)
    with W ~ N(0, 1), c ~ U[0, 2 pi) (random Fourier features of a Gaussian kernel of
    unit bandwidth in the scaled inputs); target t = tanh(Z v) + 0.1 N(0, 1), v ~
    N(0, I/d_in), centred and divided by its standard deviation."""
    rng = np.random.default_rng(seed)
    Z = standardised_gaussian(rng, n, d_in)
    W = rng.standard_normal((d_in, p))
    c = rng.uniform(0.0, 2.0 * math.pi, size=p)
    X = math.sqrt(2.0 / p) * np.cos(Z @ W / math.sqrt(d_in) + c)
    v = rng.standard_normal(d_in) / math.sqrt(d_in)
    t = np.tanh(Z @ v) + 0.1 * rng.standard_normal(n)
    y = (t - t.mean()) / t.std()
    lam_max = float(np.max(np.abs(X.T @ (y - y.mean())))) / n
    return ElasticNetProblem(np.ascontiguousarray(X), y, 0.1 * lam_max, 0.1 * lam_max, seed)
