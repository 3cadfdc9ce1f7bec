"""Plain CPU float64 oracle for Nystrom-preconditioned CG on kernel systems.

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously correct reference
that the GPU library is checked against.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the library itself
never does, and this module imports nothing from the library.

What it computes (all in float64, dense, no blocking or fusion):

* The regularised kernel system (K + lambda I) x = b of the section
  "Positive-Definite Linear Systems" (eq. rlaopt-regularized-linear-system), with
  K_ij = k(x_i, x_j) as in kernel ridge regression (eq. rlaopt-krr).  The paper
  names no kernel; the two used here are the Gaussian RBF
  exp(-|x-y|^2 / (2 sigma^2)) and the Laplacian exp(-|x-y|_2 / sigma) (L2 norm).
* The direct solution by a Cholesky factorisation, the method the same section
  names as the O(n^3) baseline.
* The randomized Nystrom approximation the paper cites for its preconditioner
  (section "Related Work", large-scale linear systems; its configuration is
  table tab:rlaopt-nystrom-config).  The paper prints no steps, so the steps are
  those of the cited method: the stabilised fixed-rank Nystrom approximation
  (orthonormalised Gaussian test matrix, shift nu, Cholesky of the shifted core,
  SVD of the factor, shift removed from the eigenvalues).
* The Nystrom preconditioner P = K_hat + lambda I (damping mode "non_adaptive"
  with base damping lambda in table tab:rlaopt-nystrom-config), applied through
  its closed-form inverse.
* Textbook preconditioned CG with the stopping rule of table
  tab:rlaopt-pcg-stopping (|r_k| <= tol |b| for every right-hand side, or the
  iteration cap), and the float64 relative residual of the common accuracy
  check (section "Common Accuracy Checks", eq. experiment-relative-residual).
* A validation loss through the solution and its exact gradient with respect
  to (lambda, sigma), for the bilevel problem of eq. rlaopt-bilevel.

Every function is pinned by tests that check it against closed forms, library
routines or brute force; see the test suite for the list.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

RBF = 0
LAPLACIAN = 1


# ---------------------------------------------------------------------------
# Kernel matrix (eq. rlaopt-krr: K_ij = k(x_i, x_j))
# ---------------------------------------------------------------------------

def squared_distances(Xr: np.ndarray, Xc: np.ndarray) -> np.ndarray:
    """|x_i - y_j|^2 from direct coordinate differences (not the expanded
    |x|^2 + |y|^2 - 2 x.y form), so identical points give exactly 0."""
    Xr = np.asarray(Xr, dtype=np.float64)
    Xc = np.asarray(Xc, dtype=np.float64)
    D = np.zeros((Xr.shape[0], Xc.shape[0]))
    for l in range(Xr.shape[1]):
        diff = Xr[:, l][:, None] - Xc[:, l][None, :]
        D += diff * diff
    return D


def kernel_matrix(Xr, Xc, kind: int, sigma: float) -> np.ndarray:
    """K(Xr, Xc) with K_ij = k(x_i, y_j)."""
    D = squared_distances(Xr, Xc)
    if kind == RBF:
        return np.exp(-D / (2.0 * sigma * sigma))
    if kind == LAPLACIAN:
        return np.exp(-np.sqrt(D) / sigma)
    raise ValueError("unknown kernel kind")


def kernel_dsigma_matrix(Xr, Xc, kind: int, sigma: float) -> np.ndarray:
    """Entrywise derivative dK/dsigma.
    RBF:       d/ds exp(-D/(2 s^2)) = exp(-D/(2 s^2)) * D / s^3
    Laplacian: d/ds exp(-sqrt(D)/s)  = exp(-sqrt(D)/s) * sqrt(D) / s^2
    """
    D = squared_distances(Xr, Xc)
    if kind == RBF:
        return np.exp(-D / (2.0 * sigma * sigma)) * D / sigma ** 3
    if kind == LAPLACIAN:
        dist = np.sqrt(D)
        return np.exp(-dist / sigma) * dist / sigma ** 2
    raise ValueError("unknown kernel kind")


def kernel_matvec(Xr, Xc, V, kind: int, sigma: float, deriv: int = 0,
                  alpha: float = 1.0, beta: float = 0.0, Out=None) -> np.ndarray:
    """Out = alpha * K(Xr, Xc) V + beta * Out   (deriv=1: dK/dsigma in place of K)."""
    V = np.asarray(V, dtype=np.float64)
    M = kernel_dsigma_matrix(Xr, Xc, kind, sigma) if deriv else kernel_matrix(Xr, Xc, kind, sigma)
    res = alpha * (M @ V)
    if beta != 0.0:
        res = res + beta * np.asarray(Out, dtype=np.float64)
    return res


def kernel_matvec_rows(Xr, Xc, V, kind: int, sigma: float, deriv: int = 0) -> np.ndarray:
    """K(Xr, Xc) V evaluated one block of rows at a time, for row samples of
    problems too large for a dense K: the same definition, bounded memory."""
    out = np.empty((np.asarray(Xr).shape[0],) + np.asarray(V).shape[1:])
    step = max(1, int(2e8 // max(1, np.asarray(Xc).shape[0])))
    for s in range(0, out.shape[0], step):
        out[s:s + step] = kernel_matvec(Xr[s:s + step], Xc, V, kind, sigma, deriv)
    return out


# ---------------------------------------------------------------------------
# Direct solve (section "Positive-Definite Linear Systems")
# ---------------------------------------------------------------------------

def direct_solve(K: np.ndarray, b: np.ndarray, lam: float) -> np.ndarray:
    """x* = (K + lam I)^{-1} b by Cholesky."""
    A = K + lam * np.eye(K.shape[0])
    c = sla.cho_factor(A, lower=True)
    return sla.cho_solve(c, b)


def relative_residual(K: np.ndarray, x: np.ndarray, b: np.ndarray, lam: float) -> np.ndarray:
    """Per-column |(K + lam I) x - b|_2 / |b|_2 in float64 (eq.
    experiment-relative-residual, with K in place of X^T X and b in place of X^T y)."""
    x = np.asarray(x, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
        b = b[:, None]
    res = K @ x + lam * x - b
    nb = np.linalg.norm(b, axis=0)
    nr = np.linalg.norm(res, axis=0)
    return np.where(nb > 0, nr / np.where(nb > 0, nb, 1.0), nr)


# ---------------------------------------------------------------------------
# Randomized Nystrom approximation (the cited method; config table
# tab:rlaopt-nystrom-config)
# ---------------------------------------------------------------------------

def float_spacing(t: float) -> float:
    """eps(t) = 2^(floor(log2 t) - 52): the gap between t and the next float64."""
    return float(np.spacing(np.float64(t)))


def nystrom(apply_K, Omega: np.ndarray):
    """Stabilised fixed-rank Nystrom approximation K_hat = U diag(lam_hat) U^T.

    apply_K(V) must return K @ V.  Steps of the cited method:
      1. Q = thin QR of the Gaussian test matrix Omega.
      2. Y = K Q.
      3. nu = sqrt(n) * eps(|Y|_2).
      4. Y_nu = Y + nu Q.
      5. C = upper Cholesky factor of (Q^T Y_nu + Y_nu^T Q) / 2.
      6. B = Y_nu C^{-1}.
      7. [U, S, ~] = thin SVD of B.
      8. lam_hat = max(0, S^2 - nu).
    Returns (U, lam_hat, nu), lam_hat in descending order.
    """
    n = Omega.shape[0]
    Q, _ = np.linalg.qr(np.asarray(Omega, dtype=np.float64), mode="reduced")
    Y = np.asarray(apply_K(Q), dtype=np.float64)
    nu = math.sqrt(n) * float_spacing(np.linalg.norm(Y, 2))
    Ynu = Y + nu * Q
    core = Q.T @ Ynu
    core = 0.5 * (core + core.T)
    C = sla.cholesky(core, lower=False)
    B = sla.solve_triangular(C, Ynu.T, trans="T", lower=False).T   # B C = Y_nu
    U, S, _ = np.linalg.svd(B, full_matrices=False)
    lam_hat = np.maximum(0.0, S * S - nu)
    return U, lam_hat, nu


def nystrom_matrix(U: np.ndarray, lam_hat: np.ndarray) -> np.ndarray:
    """K_hat = U diag(lam_hat) U^T."""
    return (U * lam_hat) @ U.T


def precond_apply(U: np.ndarray, lam_hat: np.ndarray, lam, R: np.ndarray, shift: float = 0.0) -> np.ndarray:
    """P^{-1} R for P = U diag(lam_hat) U^T + rho I, rho = lam + shift, by its closed-form
    inverse P^{-1} = U diag(1 / (lam_hat + rho)) U^T + (I - U U^T) / rho.
    lam may be a scalar or one value per column of R.  shift is 0 for the damping mode
    "non_adaptive" and the smallest retained lam_hat for "adaptive" (table
    tab:rlaopt-nystrom-config; see damping_shift)."""
    R = np.asarray(R, dtype=np.float64)
    one = R.ndim == 1
    if one:
        R = R[:, None]
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), (R.shape[1],)) + float(shift)
    W = U.T @ R
    Z = U @ (W / (lam_hat[:, None] + lam[None, :])) + (R - U @ W) / lam[None, :]
    return Z[:, 0] if one else Z


# ---------------------------------------------------------------------------
# Rank adaptation and damping modes (table tab:rlaopt-nystrom-config)
# ---------------------------------------------------------------------------

def power_error(apply_K, U: np.ndarray, lam_hat: np.ndarray, v0: np.ndarray, iters: int) -> float:
    """Estimate of |K - K_hat|_2 by `iters` power iterations on E = K - U diag(lam_hat) U^T
    (the error estimation of rank adaptation, num_power_iters in table
    tab:rlaopt-nystrom-config): v = v0 / |v0|, then per iteration w = E v, the Rayleigh
    quotient v^T w, and v = w / |w|.  Returns the last Rayleigh quotient."""
    v = np.asarray(v0, dtype=np.float64).reshape(-1)
    v = v / np.linalg.norm(v)
    est = 0.0
    for _ in range(iters):
        w = np.asarray(apply_K(v[:, None]), dtype=np.float64).reshape(-1) - U @ (lam_hat * (U.T @ v))
        est = float(v @ w)
        nw = float(np.linalg.norm(w))
        if nw == 0.0:
            break
        v = w / nw
    return est


def nystrom_adaptive(apply_K, Omega_full: np.ndarray, rank_init: int, rank_max: int | None,
                     num_power_iters: int, error_tolerance: float, v0: np.ndarray):
    """Nystrom approximation with rank adaptation (table tab:rlaopt-nystrom-config:
    rank_init, rank_max, num_power_iters, error_tolerance).  The paper gives the
    parameters but not the loop; the reading taken here: start at rank_init, build the
    stabilised approximation from the first l columns of one test matrix, estimate
    |K - K_hat|_2 with num_power_iters power iterations, and stop when the estimate is
    at most error_tolerance times the largest approximate eigenvalue or l has reached
    rank_max (rank_max None: rank_init); otherwise double l (capped at rank_max).
    Returns (U, lam_hat, nu, l, error estimate)."""
    rmax = rank_init if rank_max is None else rank_max
    l = min(rank_init, rmax)
    while True:
        U, lam_hat, nu = nystrom(apply_K, Omega_full[:, :l])
        err = power_error(apply_K, U, lam_hat, v0, num_power_iters)
        if err <= error_tolerance * lam_hat[0] or l >= rmax:
            return U, lam_hat, nu, l, err
        l = min(2 * l, rmax)


def damping_shift(lam_hat: np.ndarray, mode: str) -> float:
    """Extra damping of the preconditioner: "adaptive" adds the smallest retained
    approximate eigenvalue to the base damping, "non_adaptive" adds nothing (table
    tab:rlaopt-nystrom-config)."""
    if mode == "adaptive":
        return float(lam_hat[-1])
    if mode == "non_adaptive":
        return 0.0
    raise ValueError("damping mode must be 'adaptive' or 'non_adaptive'")


# ---------------------------------------------------------------------------
# Preconditioned CG (stopping rule of table tab:rlaopt-pcg-stopping)
# ---------------------------------------------------------------------------

def pcg(apply_A, b: np.ndarray, apply_Pinv=None, tol: float = 1e-6, max_iters: int = 1000,
        x0: np.ndarray | None = None):
    """Textbook preconditioned conjugate gradient for one right-hand side.

    apply_A(v) = A v; apply_Pinv(r) = P^{-1} r (None: identity, i.e. plain CG).
    Stops when |r_k|_2 <= tol |b|_2 with r_k the recursively updated residual, or
    after max_iters products with A.  Returns (x, iterations, recursive relres).
    b = 0 returns x = 0 after 0 iterations.
    """
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    if bnorm == 0.0:
        return x, 0, 0.0
    r = b - apply_A(x) if x0 is not None else b.copy()
    if float(np.linalg.norm(r)) <= tol * bnorm:
        return x, 0, float(np.linalg.norm(r)) / bnorm
    z = apply_Pinv(r) if apply_Pinv is not None else r.copy()
    p = z.copy()
    rho = float(r @ z)
    it = 0
    rel = float(np.linalg.norm(r)) / bnorm
    while it < max_iters:
        w = apply_A(p)
        alpha = rho / float(p @ w)
        x = x + alpha * p
        r = r - alpha * w
        it += 1
        rel = float(np.linalg.norm(r)) / bnorm
        if rel <= tol:
            break
        z = apply_Pinv(r) if apply_Pinv is not None else r.copy()
        rho_new = float(r @ z)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return x, it, rel


def block_pcg(apply_A, B: np.ndarray, apply_Pinv=None, tol: float = 1e-6, max_iters: int = 1000):
    """O'Leary's block preconditioned CG for A X = B with the s columns of B sharing one
    block Krylov space (the block variant of the batched solve), x0 = 0.  Per iteration:
    Q = A P, alpha = (P^T Q)^{-1} (R^T Z), X += P alpha, R -= Q alpha, Z = M^{-1} R,
    beta = (R_old^T Z_old)^{-1} (R^T Z), P = Z + P beta, the s x s systems solved by
    Cholesky.  Stops when every column has |r_c| <= tol |b_c| (the per right-hand-side
    rule of table tab:rlaopt-pcg-stopping) or after max_iters products.  Returns
    (X, iterations, per-column recursive relres); a Cholesky failure (the block lost
    rank) raises numpy.linalg.LinAlgError."""
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    bn = np.linalg.norm(B, axis=0)
    bn_safe = np.where(bn > 0, bn, 1.0)
    X = np.zeros_like(B)
    R = B.copy()
    rel = np.linalg.norm(R, axis=0) / bn_safe
    if np.all(rel <= tol):
        return X, 0, rel
    Z = apply_Pinv(R) if apply_Pinv is not None else R.copy()
    P = Z.copy()
    RZ = R.T @ Z
    it = 0
    while it < max_iters:
        Q = apply_A(P)
        G = P.T @ Q
        alpha = sla.cho_solve(sla.cho_factor(0.5 * (G + G.T), lower=True), RZ)
        X = X + P @ alpha
        R = R - Q @ alpha
        it += 1
        rel = np.linalg.norm(R, axis=0) / bn_safe
        if np.all(rel <= tol):
            break
        Z = apply_Pinv(R) if apply_Pinv is not None else R.copy()
        RZn = R.T @ Z
        beta = sla.cho_solve(sla.cho_factor(0.5 * (RZ + RZ.T), lower=True), RZn)
        RZ = RZn
        P = Z + P @ beta
    return X, it, rel


def nyspcg_dense(X, B, lambdas, kind, sigma, Omega=None, tol=1e-6, max_iters=1000):
    """NysPCG on every column: column c uses lambdas[c // nrhs] and B[:, c % nrhs].
    Omega None -> plain CG.  Returns (Xsol (n, nlam*nrhs), iters list, recursive relres list,
    true FP64 relres array)."""
    K = kernel_matrix(X, X, kind, sigma)
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    nrhs = B.shape[1]
    if Omega is not None:
        U, lam_hat, _ = nystrom(lambda V: K @ V, Omega)
    cols, iters, rels, trues = [], [], [], []
    for lam in lambdas:
        for j in range(nrhs):
            b = B[:, j]
            Pinv = (lambda r, lam=lam: precond_apply(U, lam_hat, lam, r)) if Omega is not None else None
            x, it, rel = pcg(lambda v, lam=lam: K @ v + lam * v, b, Pinv, tol, max_iters)
            cols.append(x)
            iters.append(it)
            rels.append(rel)
            trues.append(float(relative_residual(K, x, b, lam)[0]))
    return np.stack(cols, axis=1), iters, rels, np.array(trues)


# ---------------------------------------------------------------------------
# Gradient of a validation loss through the solution (eq. rlaopt-bilevel)
# ---------------------------------------------------------------------------

def validation_loss(X, y, Xv, yv, kind, sigma, lam) -> float:
    """L(lambda, sigma) = mean((K(Xv, X) x* - yv)^2), x* = (K(X, X) + lambda I)^{-1} y."""
    K = kernel_matrix(X, X, kind, sigma)
    x = direct_solve(K, np.asarray(y, dtype=np.float64).reshape(-1), lam)
    pred = kernel_matrix(Xv, X, kind, sigma) @ x
    res = pred - np.asarray(yv, dtype=np.float64).reshape(-1)
    return float(res @ res) / res.shape[0]


def validation_loss_grad(X, y, Xv, yv, kind, sigma, lam):
    """Exact dense gradient of L with respect to (lambda, sigma).

    With x* = A^{-1} y, A = K + lambda I, e = (2/n_v)(K_vt x* - y_v) and
    a = A^{-1} K_vt^T e (the adjoint solution):
        dL/dlambda = -a^T x*
        dL/dsigma  = e^T (dK_vt/dsigma) x* - a^T (dK/dsigma) x*
    Returns (L, dL/dlambda, dL/dsigma, x*, a)."""
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    yv = np.asarray(yv, dtype=np.float64).reshape(-1)
    K = kernel_matrix(X, X, kind, sigma)
    x = direct_solve(K, y, lam)
    Kvt = kernel_matrix(Xv, X, kind, sigma)
    res = Kvt @ x - yv
    L = float(res @ res) / res.shape[0]
    e = (2.0 / res.shape[0]) * res
    a = direct_solve(K, Kvt.T @ e, lam)
    dlam = -float(a @ x)
    dK = kernel_dsigma_matrix(X, X, kind, sigma)
    dKvt = kernel_dsigma_matrix(Xv, X, kind, sigma)
    dsig = float(e @ (dKvt @ x)) - float(a @ (dK @ x))
    return L, dlam, dsig, x, a


# ---------------------------------------------------------------------------
# Unrolled differentiation (section "Differentiating Through the Solver")
# ---------------------------------------------------------------------------

def unrolled_validation_grad(X, y, Xv, yv, kind, sigma, lam, U, lam_hat, iters: int):
    """The validation loss after exactly `iters` textbook PCG iterations from x0 = 0,
    L_k = mean((K_vt x_k - y_v)^2), and its gradient with respect to (lambda, sigma)
    by differentiating through the iterations (reverse-mode automatic differentiation
    in float64, PyTorch on the CPU): the unrolled alternative to the implicit adjoint
    that the paper's differentiation section describes.  The preconditioner P =
    U diag(lam_hat) U^T + lam I is held fixed (its lam a constant, U and lam_hat
    given), as in the adjoint; as iters grows the result tends to the exact gradient
    of validation_loss_grad.  Returns (L_k, dL_k/dlambda, dL_k/dsigma)."""
    import torch

    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64))
    D, Dv = t(squared_distances(X, X)), t(squared_distances(Xv, X))
    lam_t = torch.tensor(float(lam), dtype=torch.float64, requires_grad=True)
    sig_t = torch.tensor(float(sigma), dtype=torch.float64, requires_grad=True)

    def kmat(Dm):
        if kind == RBF:
            return torch.exp(-Dm / (2.0 * sig_t * sig_t))
        return torch.exp(-torch.sqrt(Dm) / sig_t)

    K, Kvt = kmat(D), kmat(Dv)
    Ut, lh = t(U), t(lam_hat)
    lam0 = float(lam)

    def pinv(r):
        w = Ut.T @ r
        return Ut @ (w / (lh + lam0)) + (r - Ut @ w) / lam0

    b = t(y).reshape(-1)
    x = torch.zeros_like(b)
    r = b.clone()
    z = pinv(r)
    p = z.clone()
    rho = r @ z
    for _ in range(iters):
        w = K @ p + lam_t * p
        alpha = rho / (p @ w)
        x = x + alpha * p
        r = r - alpha * w
        z = pinv(r)
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    res = Kvt @ x - t(yv).reshape(-1)
    L = (res @ res) / res.shape[0]
    L.backward()
    return float(L.detach()), float(lam_t.grad), float(sig_t.grad)


# ---------------------------------------------------------------------------
# Ridge regression (section "Large-Scale Ridge Regression with NysPCG")
# ---------------------------------------------------------------------------

def ridge_normal_apply(X):
    """The normal matrix of eq. experiment-ridge as an operator, V -> X^T (X V), never
    forming X^T X (for nystrom and pcg)."""
    X = np.asarray(X, dtype=np.float64)
    return lambda V: X.T @ (X @ V)


def ridge_direct(X, y, lam):
    """w* = (X^T X + lam I)^{-1} X^T y by Cholesky of the formed normal matrix."""
    X = np.asarray(X, dtype=np.float64)
    A = X.T @ X + lam * np.eye(X.shape[1])
    c = sla.cho_factor(A, lower=True)
    return sla.cho_solve(c, X.T @ np.asarray(y, dtype=np.float64))


# ---------------------------------------------------------------------------
# NysADMM on the bounded elastic net (sections "Splitting for ADMM" and
# "Bounded Elastic Net with NysADMM"; tables tab:rlaopt-admm-config and
# tab:rlaopt-admm-stopping)
# ---------------------------------------------------------------------------

def elastic_net_objective(X, y, w, b, lam1, lam2):
    """(1/2n)|X w + b 1 - y|^2 + lam1 |w|_1 + lam2/2 |w|^2 (eq. experiment-bounded-en)."""
    X = np.asarray(X, dtype=np.float64)
    res = X @ w + b - np.asarray(y, dtype=np.float64)
    return float(res @ res) / (2 * X.shape[0]) + lam1 * float(np.abs(w).sum()) + 0.5 * lam2 * float(w @ w)


def elastic_net_prox(v, rho, lam1, lam2, lo, hi):
    """Proximal map of g(z) = lam1 |z|_1 + lam2/2 |z|^2 + indicator(lo <= z <= hi) with
    step 1/rho, coordinate by coordinate: the minimiser of lam1|z| + lam2/2 z^2 +
    rho/2 (z - v)^2 over the real line is soft(v, lam1/rho) rho/(rho + lam2), and for a
    convex function of one variable the minimiser over [lo, hi] is that point clipped."""
    v = np.asarray(v, dtype=np.float64)
    soft = np.sign(v) * np.maximum(np.abs(v) - lam1 / rho, 0.0)
    return np.clip(soft * (rho / (rho + lam2)), lo, hi)


def admm_subproblem_tol(k, gamma, r_pri_prev=None, r_dual_prev=None):
    """Relative-residual tolerance of the k-th x-subproblem solve (k = 1, 2, ...):
    min(1, sqrt(|r_pri| |r_dual|)) k^-gamma with the previous iteration's residual
    norms (1 at k = 1): the inexact solve tracks the ADMM residuals and the factor
    k^-gamma is summable for gamma > 1 (the decay exponent of table
    tab:rlaopt-admm-config; the paper names the exponent and the adaptive tolerance of
    the method it follows, and this is the reading of how they combine)."""
    scale = 1.0 if r_pri_prev is None else min(1.0, math.sqrt(r_pri_prev * r_dual_prev))
    return max(scale * float(k) ** (-gamma), 1e-15)


def nysadmm_elastic_net(X, y, lam1, lam2, lo=0.0, hi=1.0, rho=1.0, rho_update_factor=2.0,
                        rho_update_threshold=10.0, rho_update_freq=25, alpha=1.6, sigma=1e-6, gamma=1.2,
                        rank=50, precond_update_freq=20, max_iters=1000, eps_abs=1e-4, eps_rel=1e-4,
                        seed=0, pcg_max_iters=1000):
    """NysADMM for the bounded elastic net with an unregularised intercept.

    The intercept is eliminated by centring (X_c = X - 1 mu^T, y_c = y - ybar; at any w
    the best intercept is ybar - mu^T w).  Splitting x = z with
    f(x) = (1/2n)|X_c x - y_c|^2 and g the elastic-net penalty plus the box, each
    iteration k = 1, 2, ... does, with the scaled dual u:
      1. every precond_update_freq iterations, a fresh Nystrom approximation of the
         Hessian H = X_c^T X_c / n from the test matrix Philox(seed + refresh count);
      2. x-subproblem (H + (rho + sigma) I) x = X_c^T y_c / n + rho (z - u) + sigma x_prev
         by NysPCG warm-started at x_prev, to relative residual admm_subproblem_tol
         (preconditioner P = H_hat + (rho + sigma) I);
      3. over-relaxation xh = alpha x + (1 - alpha) z;
      4. z = elastic_net_prox(xh + u, rho, ...);  5. u = u + xh - z;
      6. residuals r_pri = x - z and r_dual = grad f(x) + rho u, stop when both meet
         the tolerances of table tab:rlaopt-admm-stopping (m = p constraints);
      7. every rho_update_freq iterations, residual balancing: rho times (divided by)
         the factor when |r_pri| exceeds (falls below 1/threshold of) |r_dual|, u
         rescaled to keep rho u.
    Returns a dict with w = z (feasible), b, iterations, convergence flag, the final
    residual norms and rho, and the PCG iteration count of every subproblem."""
    from . import philox

    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, p = X.shape
    mu = X.mean(axis=0)
    ybar = float(y.mean())
    Xc = X - mu
    yc = y - ybar
    H = lambda V: Xc.T @ (Xc @ V) / n
    c = Xc.T @ yc / n
    x = np.zeros(p)
    z = np.zeros(p)
    u = np.zeros(p)
    pcg_iters = []
    converged = False
    rp = rd = float("nan")
    k = 0
    for k in range(1, max_iters + 1):
        if (k - 1) % precond_update_freq == 0:
            Om = philox.gaussian_test_matrix(p, rank, seed + (k - 1) // precond_update_freq)
            Uh, lh, _ = nystrom(H, Om)
        lk = rho + sigma
        rhs = c + rho * (z - u) + sigma * x
        tol_k = admm_subproblem_tol(k, gamma, None if k == 1 else rp, None if k == 1 else rd)
        x, it, _ = pcg(lambda v: H(v) + lk * v, rhs, lambda r: precond_apply(Uh, lh, lk, r),
                       tol=tol_k, max_iters=pcg_max_iters, x0=x)
        pcg_iters.append(it)
        xh = alpha * x + (1.0 - alpha) * z
        z = elastic_net_prox(xh + u, rho, lam1, lam2, lo, hi)
        u = u + xh - z
        rp = float(np.linalg.norm(x - z))
        rd = float(np.linalg.norm(H(x) - c + rho * u))
        eps_pri = math.sqrt(p) * eps_abs + eps_rel * max(float(np.linalg.norm(x)), float(np.linalg.norm(z)))
        eps_dual = math.sqrt(p) * eps_abs + eps_rel * float(np.linalg.norm(rho * u))
        if rp <= eps_pri and rd <= eps_dual:
            converged = True
            break
        if k % rho_update_freq == 0:
            if rp > rho_update_threshold * rd:
                rho *= rho_update_factor
                u /= rho_update_factor
            elif rd > rho_update_threshold * rp:
                rho /= rho_update_factor
                u *= rho_update_factor
    return {"w": z, "b": ybar - float(mu @ z), "iters": k, "converged": converged, "r_pri": rp, "r_dual": rd,
            "rho": rho, "pcg_iters": pcg_iters}


def elastic_net_kkt(X, y, w, lam1, lam2, lo=0.0, hi=1.0):
    """Stationarity violation of a bounded elastic-net point w (intercept at its optimum):
    the distance from -grad of the smooth part to the subdifferential of
    lam1 |.|_1 + box at w, coordinate by coordinate, as an infinity norm."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = X.shape[0]
    mu = X.mean(axis=0)
    Xc = X - mu
    gsm = Xc.T @ (Xc @ w - (y - y.mean())) / n + lam2 * w
    viol = np.empty_like(w)
    for i, wi in enumerate(w):
        # subdifferential of lam1|t| at wi, plus the normal cone of [lo, hi]
        lo_s = lam1 * (np.sign(wi) if wi != 0 else -1.0)
        hi_s = lam1 * (np.sign(wi) if wi != 0 else 1.0)
        if wi <= lo:
            lo_s = -np.inf
        if wi >= hi:
            hi_s = np.inf
        t = -gsm[i]
        viol[i] = 0.0 if lo_s <= t <= hi_s else min(abs(t - lo_s), abs(t - hi_s))
    return float(np.max(np.abs(viol))) if w.size else 0.0
