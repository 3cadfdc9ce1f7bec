"""Pins for the CPU float64 oracle (no GPU).

Each test checks an oracle function against something other than itself: a
closed form derived by hand, brute-force loops over tiny inputs, an independent
library routine, or an invariant the mathematics fixes.  The mutation tests at
the end plant plausible mistakes in copies of oracle functions and show that
the corresponding pin catches them.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import nys_inputs as ni
import oracle as o

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "closed_forms.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


# ---------------------------------------------------------------- kernel matrix

def test_kernel_closed_form_triangle():
    g = golden()["triangle_3_4_5"]
    X = np.array([g["x"]])
    Y = np.array([g["y"]])
    s = g["sigma"]
    assert o.kernel_matrix(X, Y, o.RBF, s)[0, 0] == pytest.approx(g["rbf"], rel=1e-15)
    assert o.kernel_matrix(X, Y, o.LAPLACIAN, s)[0, 0] == pytest.approx(g["laplacian"], rel=1e-15)
    assert o.kernel_dsigma_matrix(X, Y, o.RBF, s)[0, 0] == pytest.approx(g["rbf_dsigma"], rel=1e-14)
    assert o.kernel_dsigma_matrix(X, Y, o.LAPLACIAN, s)[0, 0] == pytest.approx(g["laplacian_dsigma"], rel=1e-14)


@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
def test_kernel_bruteforce_loops(kind):
    rng = np.random.default_rng(3)
    Xr = rng.standard_normal((5, 3))
    Xc = rng.standard_normal((4, 3))
    s = 1.7
    K = o.kernel_matrix(Xr, Xc, kind, s)
    for i in range(5):
        for j in range(4):
            d2 = sum((float(Xr[i, l]) - float(Xc[j, l])) ** 2 for l in range(3))
            ref = math.exp(-d2 / (2 * s * s)) if kind == o.RBF else math.exp(-math.sqrt(d2) / s)
            assert K[i, j] == pytest.approx(ref, rel=1e-14)


@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
def test_kernel_special_cases(kind):
    rng = np.random.default_rng(4)
    X = rng.standard_normal((20, 4))
    # identical points -> exactly 1 on the diagonal (direct differences)
    K = o.kernel_matrix(X, X, kind, 2.0)
    assert np.all(np.diag(K) == 1.0)
    assert np.allclose(K, K.T, rtol=0, atol=0)
    # sigma -> infinity: K -> 1 1^T
    Kinf = o.kernel_matrix(X, X, kind, 1e9)
    assert np.max(np.abs(Kinf - 1.0)) < 1e-8
    # both kernels are positive definite on distinct points
    assert np.linalg.eigvalsh(K).min() > 0.0
    # sigma -> 0: K -> I
    K0 = o.kernel_matrix(X, X, kind, 1e-3)
    assert np.max(np.abs(K0 - np.eye(20))) < 1e-12


def test_kernel_two_point_eigs():
    g = golden()["two_point_eigs"]
    K = o.kernel_matrix(np.array(g["X"]), np.array(g["X"]), o.RBF, g["sigma"])
    assert np.allclose(np.sort(np.linalg.eigvalsh(K))[::-1], g["eigs"], rtol=1e-15)


@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
def test_dsigma_matches_central_difference(kind):
    rng = np.random.default_rng(5)
    Xr = rng.standard_normal((7, 3))
    Xc = rng.standard_normal((6, 3))
    s, h = 1.3, 1e-5
    fd = (o.kernel_matrix(Xr, Xc, kind, s + h) - o.kernel_matrix(Xr, Xc, kind, s - h)) / (2 * h)
    an = o.kernel_dsigma_matrix(Xr, Xc, kind, s)
    assert np.max(np.abs(fd - an)) <= 1e-8 * np.max(np.abs(an))


def test_kernel_matvec_alpha_beta():
    rng = np.random.default_rng(6)
    Xr, Xc = rng.standard_normal((5, 2)), rng.standard_normal((8, 2))
    V, Out = rng.standard_normal((8, 3)), rng.standard_normal((5, 3))
    K = o.kernel_matrix(Xr, Xc, o.RBF, 1.1)
    got = o.kernel_matvec(Xr, Xc, V, o.RBF, 1.1, 0, 2.0, -0.5, Out)
    ref = np.einsum("ij,jk->ik", K, V) * 2.0 - 0.5 * Out
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-14)
    rows = o.kernel_matvec_rows(Xr, Xc, V, o.RBF, 1.1)
    assert np.allclose(rows, K @ V, rtol=1e-14)


# ---------------------------------------------------------------- direct solve

def test_direct_solve_two_point_closed_form():
    g = golden()["two_point_solve"]
    X = np.array(g["X"])
    K = o.kernel_matrix(X, X, o.RBF, g["sigma"])
    x = o.direct_solve(K, np.array(g["b"]), g["lam"])
    assert np.allclose(x, g["x"], rtol=1e-14)


def test_direct_solve_vs_lapack_lu():
    w = ni.small_problem(300, 5, seed=1)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    x = o.direct_solve(K, w.B[:, 0], w.lambdas[0])
    ref = np.linalg.solve(K + w.lambdas[0] * np.eye(300), w.B[:, 0])
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
    assert o.relative_residual(K, x, w.B[:, 0], w.lambdas[0])[0] < 1e-13


def test_relative_residual_closed_form():
    """Per-column |(K + lam I) x - b| / |b| at perturbed iterates of the two-point system
    (values from the closed form in tests/golden), including a b = 0 column."""
    g = golden()["two_point_relative_residual"]
    X = np.array(g["X"])
    K = o.kernel_matrix(X, X, o.RBF, g["sigma"])
    rel = o.relative_residual(K, np.array(g["Xsol"]), np.array(g["B"]), g["lam"])
    assert np.allclose(rel, g["relres"], rtol=1e-12, atol=0)
    one = o.relative_residual(K, np.array(g["Xsol"])[:, 0], np.array(g["B"])[:, 0], g["lam"])
    assert one.shape == (1,) and abs(one[0] - g["relres"][0]) <= 1e-12 * g["relres"][0]


# ---------------------------------------------------------------- Nystrom

def _spd_test_matrix(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.logspace(0, -math.log10(cond), n)
    return (Q * ev) @ Q.T


def test_nystrom_closed_form():
    """With nu -> 0, K_hat = Y (Omega^T Y)^{-1} Y^T, Y = K Omega (invariant to
    orthonormalising Omega)."""
    K = _spd_test_matrix(30, 0, cond=10.0)
    Om = np.random.default_rng(1).standard_normal((30, 10))
    U, lh, nu = o.nystrom(lambda V: K @ V, Om)
    Y = K @ Om
    ref = Y @ np.linalg.solve(Om.T @ Y, Y.T)
    assert nu < 1e-12
    assert np.linalg.norm(o.nystrom_matrix(U, lh) - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
def test_nystrom_invariants(kind):
    w = ni.small_problem(400, 6, seed=2, kind=kind, r=40)
    K = o.kernel_matrix(w.X, w.X, kind, w.sigma)
    Om = ni.gaussian_test_matrix(400, 40, 2)
    U, lh, nu = o.nystrom(lambda V: K @ V, Om)
    assert np.all(lh >= 0.0)
    assert np.all(np.diff(lh) <= 0.0)
    assert np.max(np.abs(U.T @ U - np.eye(40))) < 1e-12
    Kh = o.nystrom_matrix(U, lh)
    # K_hat is PSD and K - K_hat is PSD up to the shift nu
    assert np.linalg.eigvalsh(Kh).min() >= -1e-12 * np.linalg.norm(K, 2)
    assert np.linalg.eigvalsh(K - Kh).min() >= -nu - 1e-12 * np.linalg.norm(K, 2)
    # the retained eigenvalues never exceed those of K (K_hat <= K)
    ev = np.sort(np.linalg.eigvalsh(K))[::-1]
    assert np.all(lh <= ev[:40] * (1 + 1e-12) + nu)


def test_nystrom_exact_recovery_low_rank():
    """A linear kernel K = X X^T of rank d <= r is recovered exactly; then the
    preconditioner equals A and PCG converges in one iteration."""
    rng = np.random.default_rng(7)
    X = rng.standard_normal((120, 5))
    K = X @ X.T
    Om = rng.standard_normal((120, 12))
    U, lh, nu = o.nystrom(lambda V: K @ V, Om)
    assert np.linalg.norm(o.nystrom_matrix(U, lh) - K) <= 1e-10 * np.linalg.norm(K)
    lam = 0.3
    b = rng.standard_normal(120)
    x, it, rel = o.pcg(lambda v: K @ v + lam * v, b, lambda r: o.precond_apply(U, lh, lam, r), 1e-10, 50)
    assert it == 1
    assert np.linalg.norm(x - np.linalg.solve(K + lam * np.eye(120), b)) <= 1e-9 * np.linalg.norm(x)


def test_precond_apply_is_inverse_of_khat_plus_lambda():
    w = ni.small_problem(200, 4, seed=3, r=20)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    U, lh, _ = o.nystrom(lambda V: K @ V, ni.gaussian_test_matrix(200, 20, 3))
    lam = 0.7
    Pm = o.nystrom_matrix(U, lh) + lam * np.eye(200)
    Pinv = o.precond_apply(U, lh, lam, np.eye(200))
    assert np.max(np.abs(Pinv - np.linalg.inv(Pm))) < 1e-10 * np.max(np.abs(np.linalg.inv(Pm)))
    # per-column lambdas
    lams = np.array([0.7, 2.0, 5.0])
    R = np.random.default_rng(0).standard_normal((200, 3))
    Z = o.precond_apply(U, lh, lams, R)
    for c in range(3):
        Pc = o.nystrom_matrix(U, lh) + lams[c] * np.eye(200)
        assert np.allclose(Z[:, c], np.linalg.solve(Pc, R[:, c]), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
def test_preconditioned_spectrum_at_least_one(kind):
    w = ni.small_problem(300, 5, seed=4, kind=kind, r=30)
    K = o.kernel_matrix(w.X, w.X, kind, w.sigma)
    U, lh, nu = o.nystrom(lambda V: K @ V, ni.gaussian_test_matrix(300, 30, 4))
    lam = 0.05
    A = K + lam * np.eye(300)
    Pinv = o.precond_apply(U, lh, lam, np.eye(300))
    # P^{-1} A is similar to P^{-1/2} A P^{-1/2}: real spectrum
    ev = np.sort(np.linalg.eigvals(Pinv @ A).real)
    assert ev[0] >= 1.0 - nu / lam - 1e-9
    assert ev[-1] <= 1.0 + np.linalg.norm(K - o.nystrom_matrix(U, lh), 2) / lam + 1e-9


# ---------------------------------------------------------------- PCG

def test_pcg_matches_cholesky_plain_workload():
    w = ni.plain_fp64(0)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    Om = ni.gaussian_test_matrix(w.n, w.r, 0)
    Xs, iters, rels, trues = o.nyspcg_dense(w.X, w.B, w.lambdas, w.kind, w.sigma, Om, tol=1e-10)
    ref = o.direct_solve(K, w.B[:, 0], w.lambdas[0])
    assert np.linalg.norm(Xs[:, 0] - ref) <= 1e-6 * np.linalg.norm(ref)
    assert trues[0] <= 1e-9
    # preconditioning pays: fewer iterations than plain CG
    _, it_cg, _, _ = o.nyspcg_dense(w.X, w.B, w.lambdas, w.kind, w.sigma, None, tol=1e-10)
    assert iters[0] < it_cg[0]


def test_plain_cg_matches_scipy_cg():
    w = ni.small_problem(250, 4, seed=5)
    A = o.kernel_matrix(w.X, w.X, w.kind, w.sigma) + w.lambdas[0] * np.eye(250)
    b = w.B[:, 0]
    x, it, rel = o.pcg(lambda v: A @ v, b, None, 1e-12, 1000)
    xs, info = spla.cg(A, b, rtol=1e-12, atol=0.0, maxiter=1000)
    assert info == 0
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_pcg_iteration_bound_and_edge_cases():
    w = ni.small_problem(300, 5, seed=6, r=30)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    U, lh, _ = o.nystrom(lambda V: K @ V, ni.gaussian_test_matrix(300, 30, 6))
    lam = 0.05
    A = K + lam * np.eye(300)
    Pinv = o.precond_apply(U, lh, lam, np.eye(300))
    ev = np.sort(np.linalg.eigvals(Pinv @ A).real)
    kappa = ev[-1] / ev[0]
    tol = 1e-8
    x, it, rel = o.pcg(lambda v: A @ v, w.B[:, 0], lambda r: o.precond_apply(U, lh, lam, r), tol, 1000)
    bound = math.ceil(0.5 * math.sqrt(kappa) * math.log(2 / tol)) + 1
    assert it <= bound
    # b = 0
    x0, it0, rel0 = o.pcg(lambda v: A @ v, np.zeros(300), None, tol, 10)
    assert it0 == 0 and np.all(x0 == 0)
    # iteration cap
    _, itc, relc = o.pcg(lambda v: A @ v, w.B[:, 0], None, 1e-14, 3)
    assert itc == 3 and relc > 1e-14
    # K -> I (sigma tiny): A = (1 + lam) I converges in one iteration
    Ki = o.kernel_matrix(w.X, w.X, o.RBF, 1e-4)
    _, it1, _ = o.pcg(lambda v: Ki @ v + lam * v, w.B[:, 0], None, 1e-12, 10)
    assert it1 == 1


def test_pcg_residuals_are_preconditioner_orthogonal():
    """r_i^T P^{-1} r_j = 0 for i != j in exact arithmetic (checked on a few steps)."""
    w = ni.small_problem(150, 3, seed=7, r=10)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    U, lh, _ = o.nystrom(lambda V: K @ V, ni.gaussian_test_matrix(150, 10, 7))
    lam = 0.5
    A = K + lam * np.eye(150)
    b = w.B[:, 0]
    rs = []
    x = np.zeros(150); r = b.copy(); z = o.precond_apply(U, lh, lam, r); p = z.copy(); rho = r @ z
    for _ in range(4):
        rs.append(r.copy())
        wv = A @ p; al = rho / (p @ wv); x = x + al * p; r = r - al * wv
        z = o.precond_apply(U, lh, lam, r); rn = r @ z; p = z + (rn / rho) * p; rho = rn
    G = np.array([[ri @ o.precond_apply(U, lh, lam, rj) for rj in rs] for ri in rs])
    off = G - np.diag(np.diag(G))
    assert np.max(np.abs(off)) <= 1e-9 * np.max(np.abs(np.diag(G)))


def test_multi_column_lambda_grid_independent():
    w = ni.small_problem(200, 4, seed=8, nrhs=2, r=20)
    Om = ni.gaussian_test_matrix(200, 20, 8)
    lams = [0.1, 1.0, 10.0]
    Xs, iters, rels, trues = o.nyspcg_dense(w.X, w.B, lams, w.kind, w.sigma, Om, tol=1e-10)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    for c in range(6):
        ref = o.direct_solve(K, w.B[:, c % 2], lams[c // 2])
        assert np.linalg.norm(Xs[:, c] - ref) <= 1e-7 * np.linalg.norm(ref)


# ---------------------------------------------------------------- gradient

@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
def test_gradient_matches_central_differences(kind):
    w = ni.small_problem(240, 4, seed=9, kind=kind)
    X, y = w.X[:200], w.B[:200, 0]
    Xv, yv = w.X[200:], w.B[200:, 0]
    lam, sig = 0.5, 1.5
    L, dlam, dsig, _, _ = o.validation_loss_grad(X, y, Xv, yv, kind, sig, lam)
    h = 1e-4
    f = lambda tl, ts: o.validation_loss(X, y, Xv, yv, kind, math.exp(ts), math.exp(tl))
    tl, ts = math.log(lam), math.log(sig)
    fd_l = (f(tl + h, ts) - f(tl - h, ts)) / (2 * h)
    fd_s = (f(tl, ts + h) - f(tl, ts - h)) / (2 * h)
    assert L == pytest.approx(f(tl, ts), rel=1e-14)
    assert lam * dlam == pytest.approx(fd_l, rel=1e-5)
    assert sig * dsig == pytest.approx(fd_s, rel=1e-5)


# ---------------------------------------------------------------- inputs

def test_input_recipes_shapes():
    w = ni.plain_fp64(0)
    assert w.X.shape == (2000, 10) and w.B.shape == (2000, 1)
    assert np.allclose(w.X.mean(0), 0, atol=1e-12) and np.allclose(w.X.std(0), 1, atol=1e-12)
    g = ni.batched_lambda_grid(0, n=1000)
    assert g.B.shape == (1000, 64) and len(g.lambdas) == 8
    assert set(np.unique(g.B)) <= {-1.0, 1.0}
    assert g.lambdas[0] == pytest.approx(1e-7 * 1000) and g.lambdas[-1] == pytest.approx(1e-3 * 1000)
    f = ni.matrix_free_fp32(0, n=5000)
    assert f.X.shape == (5000, 20)
    # the heavy-tailed column has much larger extremes than the Gaussian ones
    assert np.abs(f.X[:, -1]).max() > 2 * np.abs(f.X[:, :-1]).max()


# ---------------------------------------------------------------- planted mistakes

def test_mutant_rbf_normalisation_is_caught():
    g = golden()["triangle_3_4_5"]
    def mutant(Xr, Xc, s):
        return np.exp(-o.squared_distances(Xr, Xc) / (s * s))      # 2 sigma^2 -> sigma^2
    got = mutant(np.array([g["x"]]), np.array([g["y"]]), g["sigma"])[0, 0]
    assert abs(got - g["rbf"]) > 1e-3


def test_mutant_dsigma_power_is_caught():
    rng = np.random.default_rng(5)
    Xr, Xc = rng.standard_normal((4, 3)), rng.standard_normal((4, 3))
    s, h = 1.3, 1e-5
    fd = (o.kernel_matrix(Xr, Xc, o.RBF, s + h) - o.kernel_matrix(Xr, Xc, o.RBF, s - h)) / (2 * h)
    mutant = o.kernel_matrix(Xr, Xc, o.RBF, s) * o.squared_distances(Xr, Xc) / s ** 2
    assert np.max(np.abs(fd - mutant)) > 1e-3 * np.max(np.abs(fd))


def test_mutant_precond_missing_complement_is_caught():
    w = ni.small_problem(120, 3, seed=3, r=10)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    U, lh, _ = o.nystrom(lambda V: K @ V, ni.gaussian_test_matrix(120, 10, 3))
    lam = 0.7
    mutant = U @ np.diag(1.0 / (lh + lam)) @ U.T                   # dropped (I - UU^T)/lam
    Pinv = np.linalg.inv(o.nystrom_matrix(U, lh) + lam * np.eye(120))
    assert np.max(np.abs(mutant - Pinv)) > 1e-2 * np.max(np.abs(Pinv))


def test_mutant_gradient_sign_is_caught():
    w = ni.small_problem(140, 3, seed=11)
    X, y, Xv, yv = w.X[:120], w.B[:120, 0], w.X[120:], w.B[120:, 0]
    lam, sig = 0.5, 1.2
    _, dlam, _, x, a = o.validation_loss_grad(X, y, Xv, yv, o.RBF, sig, lam)
    h = 1e-4
    fd = (o.validation_loss(X, y, Xv, yv, o.RBF, sig, lam * math.exp(h))
          - o.validation_loss(X, y, Xv, yv, o.RBF, sig, lam * math.exp(-h))) / (2 * h)
    mutant = +float(a @ x)                                           # sign flipped
    assert abs(lam * mutant - fd) > 1e-3 * abs(fd)
    assert abs(lam * dlam - fd) <= 1e-5 * abs(fd)


@pytest.mark.parametrize("mistake", ["norm_squared", "no_square_root"])
def test_mutant_relative_residual_normalisation_is_caught(mistake):
    g = golden()["two_point_relative_residual"]
    X = np.array(g["X"])
    K = o.kernel_matrix(X, X, o.RBF, g["sigma"])
    x, b = np.array(g["Xsol"])[:, :2], np.array(g["B"])[:, :2]
    res = K @ x + g["lam"] * x - b
    if mistake == "norm_squared":
        mutant = np.linalg.norm(res, axis=0) / np.sum(b * b, axis=0)
    else:
        mutant = np.sum(res * res, axis=0) / np.sum(b * b, axis=0)
    assert np.max(np.abs(mutant - np.array(g["relres"][:2]))) > 1e-2 * max(g["relres"][:2])


# ---------------------------------------------------------------- counter-based test matrix

def test_philox_known_answers():
    """Philox4x32-10 against the known-answer vectors published with the generator's
    reference implementation (all-zero counter and key; the hexadecimal digits of pi)."""
    from oracle import philox as ph
    kat = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
           ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
            (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in kat:
        got = ph.philox4x32_10(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
        assert [int(v) for v in got] == list(want)


def test_philox_gaussian_test_matrix_distribution():
    """The oracle's seeded test matrix is standard normal (Kolmogorov-Smirnov against
    the normal CDF), its cosine and sine halves are uncorrelated, different seeds give
    different draws, and a row range is a pure function of (seed, index)."""
    import scipy.stats as st
    from oracle import philox as ph
    Z = ph.gaussian_test_matrix(400, 250, 12345)
    assert st.kstest(Z.reshape(-1), "norm").pvalue > 1e-3
    assert abs(np.corrcoef(Z.reshape(-1)[0::2], Z.reshape(-1)[1::2])[0, 1]) < 0.02
    assert not np.allclose(Z, ph.gaussian_test_matrix(400, 250, 12346))
    assert np.array_equal(ph.gaussian_test_matrix(401, 250, 12345)[:400], Z)


# ---------------------------------------------------------------- rank adaptation, damping modes

def test_power_error_against_dense_spectrum():
    """The power estimate of |K - K_hat|_2 approaches the largest eigenvalue of the
    PSD residual from below (dense eigvalsh on a tiny case with a spectral gap)."""
    w = ni.small_problem(300, 4, seed=21, r=12)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    U, lh, nu = o.nystrom(lambda V: K @ V, ni.gaussian_test_matrix(300, 12, 21))
    E = K - o.nystrom_matrix(U, lh)
    ev = np.linalg.eigvalsh(0.5 * (E + E.T))
    v0 = np.random.default_rng(5).standard_normal(300)
    e3 = o.power_error(lambda V: K @ V, U, lh, v0, 3)
    e30 = o.power_error(lambda V: K @ V, U, lh, v0, 30)
    assert e3 <= ev[-1] * (1 + 1e-10) and e30 <= ev[-1] * (1 + 1e-10)
    assert e30 >= 0.999 * ev[-1] and e30 >= e3 - 1e-12 * ev[-1]


def test_rank_adaptation_stops_at_exact_low_rank():
    """A rank-5 PSD matrix (linear kernel of 5-dimensional points): from rank 2 the
    rank doubles to 4 (error still large), then 8 >= 5 recovers K up to the shift,
    and the loop stops there; with rank_max 4 it stops at 4."""
    rng = np.random.default_rng(22)
    Z = rng.standard_normal((200, 5))
    K = Z @ Z.T
    Om = rng.standard_normal((200, 32))
    v0 = rng.standard_normal(200)
    U, lh, nu, l, err = o.nystrom_adaptive(lambda V: K @ V, Om, 2, 32, 10, 1e-2, v0)
    assert l == 8 and err <= 1e-8 * lh[0]
    assert np.max(np.abs(o.nystrom_matrix(U, lh) - K)) <= 1e-8 * lh[0]
    U4, lh4, _, l4, err4 = o.nystrom_adaptive(lambda V: K @ V, Om, 2, 4, 10, 1e-2, v0)
    assert l4 == 4 and err4 > 1e-2 * lh4[0]
    _, _, _, l1, _ = o.nystrom_adaptive(lambda V: K @ V, Om, 2, None, 10, 1e-2, v0)
    assert l1 == 2


def test_adaptive_damping_preconditioner():
    """P = K_hat + (lam + lam_hat_min) I: the closed-form apply is the dense inverse, and
    the preconditioned spectrum lies in [lam / (lam + lam_hat_min), 1 + |K - K_hat| /
    (lam + lam_hat_min)] (K_hat <= K up to nu)."""
    w = ni.small_problem(250, 4, seed=23, r=20)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    U, lh, nu = o.nystrom(lambda V: K @ V, ni.gaussian_test_matrix(250, 20, 23))
    lam = 0.05
    sh = o.damping_shift(lh, "adaptive")
    assert sh == lh[-1] and o.damping_shift(lh, "non_adaptive") == 0.0
    P = o.nystrom_matrix(U, lh) + (lam + sh) * np.eye(250)
    R = np.random.default_rng(6).standard_normal((250, 3))
    assert np.allclose(o.precond_apply(U, lh, lam, R, shift=sh), np.linalg.solve(P, R), rtol=1e-9, atol=1e-12)
    A = K + lam * np.eye(250)
    L = np.linalg.cholesky(P)
    M = np.linalg.solve(L, np.linalg.solve(L, A).T).T
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    Enorm = np.linalg.norm(K - o.nystrom_matrix(U, lh), 2)
    assert ev[0] >= lam / (lam + sh) * (1 - 1e-9) - nu / lam
    assert ev[-1] <= 1 + Enorm / (lam + sh) + 1e-9
    # the adaptive preconditioner still gives the direct solution through PCG
    b = w.B[:, 0]
    x, it, _ = o.pcg(lambda v: A @ v, b, lambda r: o.precond_apply(U, lh, lam, r, shift=sh), tol=1e-12)
    assert np.linalg.norm(x - o.direct_solve(K, b, lam)) <= 1e-9 * np.linalg.norm(x)


# ---------------------------------------------------------------- unrolled differentiation

@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
def test_unrolled_gradient_tends_to_the_exact_gradient(kind):
    """Differentiating through k PCG iterations: after enough iterations the unrolled
    gradient is the implicit (exact) one of validation_loss_grad."""
    w = ni.small_problem(260, 4, seed=51, kind=kind, r=20)
    X, y, Xv, yv = w.X[:200], w.B[:200, 0], w.X[200:], w.B[200:, 0]
    lam, sig = 0.3, 1.4
    K = o.kernel_matrix(X, X, kind, sig)
    U, lh, _ = o.nystrom(lambda V: K @ V, ni.gaussian_test_matrix(200, 20, 51))
    L, dlam, dsig, _, _ = o.validation_loss_grad(X, y, Xv, yv, kind, sig, lam)
    Lk, gl, gs = o.unrolled_validation_grad(X, y, Xv, yv, kind, sig, lam, U, lh, 60)
    assert Lk == pytest.approx(L, rel=1e-10)
    assert gl == pytest.approx(dlam, rel=1e-8)
    assert gs == pytest.approx(dsig, rel=1e-8)


def test_unrolled_gradient_matches_differences_of_the_truncated_loss():
    """After 3 iterations (far from converged) the unrolled gradient is the derivative
    of the 3-iteration loss itself: central differences of L_3 in lambda and sigma
    (with the preconditioner fixed) agree, and both differ from the exact gradient."""
    w = ni.small_problem(220, 3, seed=52, r=10)
    X, y, Xv, yv = w.X[:180], w.B[:180, 0], w.X[180:], w.B[180:, 0]
    lam, sig = 0.2, 1.1
    K = o.kernel_matrix(X, X, o.RBF, sig)
    U, lh, _ = o.nystrom(lambda V: K @ V, ni.gaussian_test_matrix(180, 10, 52))

    def L3(lm, sg):
        # the same truncated solve with the preconditioner's damping held at lam
        Km = o.kernel_matrix(X, X, o.RBF, sg)
        x = np.zeros(180)
        r = y.copy()
        z = o.precond_apply(U, lh, lam, r)
        p, rho = z.copy(), r @ z
        for _ in range(3):
            wv = Km @ p + lm * p
            al = rho / (p @ wv)
            x, r = x + al * p, r - al * wv
            z = o.precond_apply(U, lh, lam, r)
            rn = r @ z
            p, rho = z + (rn / rho) * p, rn
        res = o.kernel_matrix(Xv, X, o.RBF, sg) @ x - yv
        return float(res @ res) / len(yv)

    _, gl, gs = o.unrolled_validation_grad(X, y, Xv, yv, o.RBF, sig, lam, U, lh, 3)
    h = 1e-6
    fl = (L3(lam + h, sig) - L3(lam - h, sig)) / (2 * h)
    fs = (L3(lam, sig + h) - L3(lam, sig - h)) / (2 * h)
    assert gl == pytest.approx(fl, rel=1e-6)
    assert gs == pytest.approx(fs, rel=1e-6)
    _, dlam, dsig, _, _ = o.validation_loss_grad(X, y, Xv, yv, o.RBF, sig, lam)
    assert abs(gs - dsig) > 1e-4 * abs(dsig)


# ---------------------------------------------------------------- ridge regression

def test_sorf_factor_against_explicit_hadamard():
    """The SORF factor equals H D1 H D2 H D3 built from scipy's Hadamard matrix, and
    has orthonormal columns."""
    import scipy.linalg as sl
    rng = np.random.default_rng(3)
    n = 64
    signs = rng.choice(np.array([-1.0, 1.0]), size=(3, n))
    H = sl.hadamard(n) / math.sqrt(n)
    S = H @ np.diag(signs[0]) @ H @ np.diag(signs[1]) @ H @ np.diag(signs[2])
    cols = ni.sorf_columns(n, 40, signs)
    assert np.allclose(cols, S[:, :40], atol=1e-13)
    assert np.allclose(cols.T @ cols, np.eye(40), atol=1e-13)


@pytest.mark.parametrize("alpha", [0.5, 2.0])
def test_ridge_spectrum_and_closed_form(alpha):
    """X^T X + lam I has eigenvalues i^-alpha + lam (the paper's statement for n >= p),
    and the direct solution is the closed form V diag(s / (s^2 + lam)) U^T y."""
    pr = ni.ridge_problem(256, 128, alpha, seed=4)
    lam = 1e-3
    ev = np.sort(np.linalg.eigvalsh(pr.X.T @ pr.X + lam * np.eye(128)))[::-1]
    want = np.arange(1, 129) ** (-alpha) + lam
    assert np.allclose(ev, want, rtol=1e-10, atol=1e-13)
    w = o.ridge_direct(pr.X, pr.y, lam)
    closed = pr.V @ ((pr.sigma / (pr.sigma ** 2 + lam)) * (pr.U.T @ pr.y))
    assert np.linalg.norm(w - closed) <= 1e-9 * np.linalg.norm(closed)
    assert abs(np.linalg.norm(pr.y) - 1.0) < 1e-12


def test_ridge_nyspcg_beats_cg_when_ill_conditioned():
    """The oracle's NysPCG on the normal operator converges to the direct solution, in
    far fewer iterations than CG when the spectrum decays fast and lambda is small."""
    pr = ni.ridge_problem(512, 512, 2.0, seed=5)
    lam = 1e-6
    apply_K = o.ridge_normal_apply(pr.X)
    U, lh, _ = o.nystrom(apply_K, ni.gaussian_test_matrix(512, 64, 5))
    A = lambda v: apply_K(v) + lam * v
    b = pr.X.T @ pr.y
    x, it_p, _ = o.pcg(A, b, lambda r: o.precond_apply(U, lh, lam, r), tol=1e-10, max_iters=5000)
    _, it_cg, _ = o.pcg(A, b, None, tol=1e-10, max_iters=5000)
    ref = o.ridge_direct(pr.X, pr.y, lam)
    assert np.linalg.norm(x - ref) <= 1e-4 * np.linalg.norm(ref)
    assert it_p * 5 < it_cg


# ---------------------------------------------------------------- NysADMM (bounded elastic net)

def _bvls_elastic_net(X, y, lam1, lam2, lo=0.0, hi=1.0):
    """Exact bounded elastic net on [0, 1]^p (where |w|_1 = 1^T w) by SciPy's bounded
    least squares: (1/2n)|X_c w - y_c|^2 + lam2/2|w|^2 + lam1 1^T w equals, up to a
    constant, 1/2 |[X_c / sqrt(n); sqrt(lam2) I] w - [y_c / sqrt(n); -lam1/sqrt(lam2) 1]|^2."""
    from scipy.optimize import lsq_linear
    n, p = X.shape
    Xc = X - X.mean(axis=0)
    yc = y - y.mean()
    A = np.vstack([Xc / math.sqrt(n), math.sqrt(lam2) * np.eye(p)])
    b = np.concatenate([yc / math.sqrt(n), -lam1 / math.sqrt(lam2) * np.ones(p)])
    return lsq_linear(A, b, bounds=(lo, hi), method="bvls", tol=1e-14).x


def test_elastic_net_prox_against_brute_force():
    rng = np.random.default_rng(70)
    grid = np.linspace(-0.5, 1.5, 400001)
    for _ in range(30):
        v, rho, l1, l2 = rng.normal(0, 1), rng.uniform(0.1, 3), rng.uniform(0, 0.5), rng.uniform(0, 0.5)
        zs = np.clip(grid, 0.0, 1.0)
        obj = l1 * np.abs(zs) + 0.5 * l2 * zs ** 2 + 0.5 * rho * (zs - v) ** 2
        z_bf = zs[np.argmin(obj)]
        z = float(o.elastic_net_prox(np.array([v]), rho, l1, l2, 0.0, 1.0)[0])
        assert abs(z - z_bf) <= 1e-5


def test_kkt_measure_vanishes_at_the_exact_solution_only():
    pr = ni.elastic_net_problem(600, 8, 40, seed=71)
    w = _bvls_elastic_net(pr.X, pr.y, pr.lam1, pr.lam2)
    assert o.elastic_net_kkt(pr.X, pr.y, w, pr.lam1, pr.lam2) <= 1e-10
    assert 0.0 < w.max() and w.min() == 0.0                     # some bounds are active
    w2 = w.copy()
    w2[np.argmax(w)] *= 0.9
    assert o.elastic_net_kkt(pr.X, pr.y, w2, pr.lam1, pr.lam2) > 1e-4


@pytest.mark.parametrize("seed", [72, 73])
def test_nysadmm_reaches_the_bounded_least_squares_solution(seed):
    """The oracle's NysADMM, run to tight tolerances, lands on the exact solution of the
    bounded problem (computed independently by SciPy's BVLS) and on its intercept; at
    the paper's default tolerances it meets its own stopping rule with a small
    stationarity violation."""
    pr = ni.elastic_net_problem(800, 8, 48, seed=seed)
    ref = _bvls_elastic_net(pr.X, pr.y, pr.lam1, pr.lam2)
    res = o.nysadmm_elastic_net(pr.X, pr.y, pr.lam1, pr.lam2, rank=16, eps_abs=1e-10, eps_rel=1e-10,
                                max_iters=3000, seed=seed)
    assert res["converged"]
    assert np.max(np.abs(res["w"] - ref)) <= 1e-7
    b_ref = pr.y.mean() - pr.X.mean(axis=0) @ ref
    assert abs(res["b"] - b_ref) <= 1e-7
    assert o.elastic_net_kkt(pr.X, pr.y, res["w"], pr.lam1, pr.lam2) <= 1e-8
    obj_ref = o.elastic_net_objective(pr.X, pr.y, ref, b_ref, pr.lam1, pr.lam2)
    assert abs(o.elastic_net_objective(pr.X, pr.y, res["w"], res["b"], pr.lam1, pr.lam2) - obj_ref) <= 1e-9
    loose = o.nysadmm_elastic_net(pr.X, pr.y, pr.lam1, pr.lam2, rank=16, seed=seed)
    assert loose["converged"] and loose["iters"] < res["iters"]
    assert o.elastic_net_kkt(pr.X, pr.y, loose["w"], pr.lam1, pr.lam2) <= 1e-2


def test_nysadmm_without_penalties_or_active_bounds_is_ridge():
    """lam1 = 0 and bounds that never bind: the fixed point is the ridge solution
    (X_c^T X_c / n + lam2 I)^{-1} X_c^T y_c / n."""
    pr = ni.elastic_net_problem(500, 6, 30, seed=74)
    lam2 = 0.05
    res = o.nysadmm_elastic_net(pr.X, pr.y, 0.0, lam2, lo=-1e6, hi=1e6, rank=10, eps_abs=1e-11, eps_rel=1e-11,
                                max_iters=3000, seed=74)
    Xc = pr.X - pr.X.mean(axis=0)
    yc = pr.y - pr.y.mean()
    ref = np.linalg.solve(Xc.T @ Xc / 500 + lam2 * np.eye(30), Xc.T @ yc / 500)
    assert res["converged"] and np.max(np.abs(res["w"] - ref)) <= 1e-8


# ---------------------------------------------------------------- block PCG (O'Leary)

def test_block_pcg_with_one_column_is_pcg():
    """A block of one column is textbook PCG: the same iterates and iteration count (on a
    well-conditioned system, where the two roundings cannot steer the paths apart)."""
    w = ni.small_problem(400, 5, seed=90, r=20)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    U, lh, _ = o.nystrom(lambda V: K @ V, ni.gaussian_test_matrix(400, 20, 90))
    lam = 1.0
    A = lambda V: K @ V + lam * V
    Pinv = lambda R: o.precond_apply(U, lh, lam, R)
    b = w.B[:, 0]
    Xb, itb, _ = o.block_pcg(A, b[:, None], Pinv, tol=1e-8)
    x, it, _ = o.pcg(lambda v: A(v[:, None])[:, 0], b, lambda r: Pinv(r[:, None])[:, 0], tol=1e-8)
    assert itb == it and np.max(np.abs(Xb[:, 0] - x)) <= 1e-12 * np.max(np.abs(x))


def test_block_pcg_terminates_in_n_over_s_steps():
    """In exact arithmetic block CG ends after at most ceil(n / s) block steps (the block
    Krylov space fills R^n); on a small well-conditioned system it reaches the direct
    solution within that count plus a few rounding steps, and far fewer than column CG."""
    rng = np.random.default_rng(91)
    n, s = 48, 6
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * np.linspace(1.0, 50.0, n)) @ Q.T
    B = rng.standard_normal((n, s))
    X, it, rel = o.block_pcg(lambda V: A @ V, B, None, tol=1e-11, max_iters=200)
    assert it <= n // s + 2
    assert np.max(np.abs(X - np.linalg.solve(A, B))) <= 1e-9 * np.max(np.abs(X))
    its = [o.pcg(lambda v: A @ v, B[:, c], None, tol=1e-11, max_iters=200)[1] for c in range(s)]
    assert it < min(its)


def test_block_pcg_matches_direct_solves_on_a_kernel_system():
    w = ni.small_problem(600, 6, seed=92, nrhs=8, r=30)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    U, lh, _ = o.nystrom(lambda V: K @ V, ni.gaussian_test_matrix(600, 30, 92))
    lam = 1e-3
    X, it, rel = o.block_pcg(lambda V: K @ V + lam * V, w.B, lambda R: o.precond_apply(U, lh, lam, R), tol=1e-10,
                             max_iters=3000)
    ref = np.linalg.solve(K + lam * np.eye(600), w.B)
    assert np.all(rel <= 1e-10)
    assert np.max(np.abs(X - ref)) <= 1e-6 * np.max(np.abs(ref))
