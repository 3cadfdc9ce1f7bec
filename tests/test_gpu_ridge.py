"""GPU parity of the ridge-regression path (the normal equations (X^T X + lambda I) w =
X^T y with X^T X applied matrix-free) against the CPU float64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import nys_inputs as ni
import oracle as o

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, torch.float64)


@pytest.mark.parametrize("n,p,r", [(512, 256, 40), (300, 300, 300), (1024, 128, 1)])
def test_ridge_sketch_and_preconditioner_match_oracle(nys, n, p, r):
    """Y = X^T X Q for the device's orthonormalised Omega, Omega left untouched, and the
    preconditioner built from (Y, Q) equal to the oracle's Nystrom approximation of the
    normal matrix for the same Omega.  p = 300 is not a power of two: a random
    Gaussian X stands in for the SORF data there."""
    print(f"case ridge sketch n={n} p={p} r={r}", flush=True)
    if p & (p - 1):
        X = np.random.default_rng(8).standard_normal((n, p)) / np.sqrt(n)
    else:
        X = ni.ridge_problem(n, p, 1.0, seed=8).X
    Om = ni.gaussian_test_matrix(p, r, 8)
    tX, tOm = T(X), T(Om)
    before = tOm.clone()
    Y, Q = nys.nys_ridge_sketch(tX, tOm)
    torch.cuda.synchronize()
    assert torch.equal(before, tOm)
    Qh, Yh = Q.cpu().numpy(), Y.cpu().numpy()
    assert np.max(np.abs(Qh.T @ Qh - np.eye(r))) <= 1e-11
    A = X.T @ X
    scale = np.linalg.norm(A, 2)
    assert np.max(np.abs(Yh - A @ Qh)) <= 64 * np.finfo(float).eps * n * scale
    P = nys.nys_precond_build(Y, Q)
    _, lho, _ = o.nystrom(o.ridge_normal_apply(X), Om)
    assert np.max(np.abs(P.lam_hat.cpu().numpy() - lho)) <= 1e-9 * lho[0]


def test_ridge_sketch_seed_mode_matches_oracle_generator(nys):
    from oracle import philox as ph
    pr = ni.ridge_problem(256, 256, 2.0, seed=9)
    Y, Q = nys.nys_ridge_sketch(T(pr.X), None, seed=123, r=32)
    P = nys.nys_precond_build(Y, Q)
    _, lho, _ = o.nystrom(o.ridge_normal_apply(pr.X), ph.gaussian_test_matrix(256, 32, 123))
    assert np.max(np.abs(P.lam_hat.cpu().numpy() - lho)) <= 1e-9 * lho[0]


@pytest.mark.parametrize("alpha,lams", [(2.0, [1e-6, 1e-4, 1e-2]), (0.5, [1e-3])])
def test_ridge_solve_matches_closed_form(nys, alpha, lams):
    """NysPCG on the paper's ridge data (eq. experiment-ridge-data) for several lambdas
    and two targets at once, against the closed-form solution
    w = V diag(s / (s^2 + lambda)) U^T y: the error is at most cond(A) times the
    reported float64 residual, and that residual is recomputed on the host."""
    n, p, r = 2048, 1024, 128
    print(f"case ridge solve alpha={alpha} lams={lams}", flush=True)
    pr = ni.ridge_problem(n, p, alpha, seed=10)
    y2 = np.random.default_rng(11).standard_normal(n)
    Yt = np.stack([pr.y, y2], axis=1)
    tX = T(pr.X)
    Y, Q = nys.nys_ridge_sketch(tX, T(ni.gaussian_test_matrix(p, r, 10)))
    P = nys.nys_precond_build(Y, Q)
    tol = 1e-10
    W, info, rc = nys.nys_ridge_solve(tX, T(Yt), lams, P, tol=tol, max_iters=2000, check_true=True)
    assert rc == nys.OK
    Wh = W.cpu().numpy()
    A0 = pr.X.T @ pr.X
    for li, lam in enumerate(lams):
        for j in range(2):
            c = li * 2 + j
            w = Wh[:, c]
            b = pr.X.T @ Yt[:, j]
            res = np.linalg.norm(A0 @ w + lam * w - b) / np.linalg.norm(b)
            assert info[c]["status"] == nys.OK
            assert info[c]["relres_recursive"] <= tol
            # the float64 residual itself carries rounding of order n u |A| |w| / |b|
            floor = 4 * n * np.finfo(float).eps * np.linalg.norm(w) / np.linalg.norm(b)
            assert abs(res - info[c]["relres_true"]) <= 1e-2 * res + floor
            assert res <= 10 * tol + floor
            ref = pr.V @ ((pr.sigma / (pr.sigma ** 2 + lam)) * (pr.U.T @ Yt[:, j]))
            cond = (pr.sigma[0] ** 2 + lam) / (pr.sigma[-1] ** 2 + lam)
            err = np.linalg.norm(w - ref) / np.linalg.norm(ref)
            assert err <= 2 * cond * max(res, 1e-15) + 1e-12


def test_ridge_nyspcg_needs_far_fewer_iterations_than_cg(nys):
    """At alpha = 2 and lambda = 1e-6 the normal matrix has about 1000 eigenvalues above
    lambda; a rank-256 Nystrom preconditioner cuts the iteration count several-fold, and
    both solves agree with the oracle's Cholesky solution."""
    n = p = 2048
    pr = ni.ridge_problem(n, p, 2.0, seed=12)
    lam, tol = 1e-6, 1e-8
    tX, ty = T(pr.X), T(pr.y)
    Y, Q = nys.nys_ridge_sketch(tX, None, seed=12, r=256)
    P = nys.nys_precond_build(Y, Q)
    w_p, info_p, _ = nys.nys_ridge_solve(tX, ty, lam, P, tol=tol, max_iters=20000, check_true=True)
    w_c, info_c, _ = nys.nys_ridge_solve(tX, ty, lam, None, tol=tol, max_iters=20000, check_true=True)
    it_p, it_c = info_p[0]["iters"], info_c[0]["iters"]
    print(f"ridge n=p={n} lambda={lam}: NysPCG {it_p} iterations, CG {it_c}", flush=True)
    assert info_p[0]["status"] == nys.OK and info_c[0]["status"] == nys.OK
    assert it_p * 4 < it_c
    ref = o.ridge_direct(pr.X, pr.y, lam)
    cond = (1.0 + lam) / (pr.sigma[-1] ** 2 + lam)
    for w, inf in ((w_p, info_p[0]), (w_c, info_c[0])):
        err = np.linalg.norm(w.cpu().numpy() - ref) / np.linalg.norm(ref)
        assert err <= 2 * cond * inf["relres_true"] + 1e-9


def test_ridge_argument_errors(nys):
    X = torch.zeros((8, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        nys.nys_ridge_sketch(X, torch.zeros((5, 2), dtype=torch.float64, device=DEV))
    with pytest.raises(nys.NysError):
        nys.nys_ridge_sketch(X, None, r=5)            # r > p
    with pytest.raises(nys.NysError):
        nys.nys_ridge_solve(X, torch.zeros(8, dtype=torch.float64, device=DEV), [0.0])
    with pytest.raises(nys.NysError):                 # a rank-deficient Omega
        nys.nys_ridge_sketch(X, torch.ones((4, 2), dtype=torch.float64, device=DEV))
