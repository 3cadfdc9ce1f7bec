"""GPU parity of the sketch, preconditioner build/apply, NysPCG solve and
backward against the CPU float64 oracle.  All calls go through the C ABI."""
import math

import numpy as np
import pytest
import torch

import nys_inputs as ni
import oracle as o

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def T(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


def build(nys, X, Om, kind, sigma, prec=0):
    tX, tO = T(X), T(Om)
    P = nys.build_preconditioner(tX, tO, kind, sigma, prec)
    torch.cuda.synchronize()
    return tX, P


# ------------------------------------------------------------------ preconditioner

@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
def test_precond_matches_oracle_fp64(nys, kind):
    w = ni.small_problem(600, 6, seed=1, kind=kind, r=40)
    Om = ni.gaussian_test_matrix(w.n, w.r, 1)
    K = o.kernel_matrix(w.X, w.X, kind, w.sigma)
    Uo, lho, nuo = o.nystrom(lambda V: K @ V, Om)
    tX, P = build(nys, w.X, Om, kind, w.sigma)
    lh = P.lam_hat.cpu().numpy()
    U = P.U.cpu().numpy()
    scale = lho[0]
    assert P.rank <= w.r
    # eigenvalues (descending) and the approximation itself; U only up to rotations
    assert np.max(np.abs(lh - lho)) <= 1e-9 * scale
    Kh = (U * lh) @ U.T
    assert np.max(np.abs(Kh - o.nystrom_matrix(Uo, lho))) <= 1e-9 * scale
    k = P.rank
    assert np.max(np.abs(U[:, :k].T @ U[:, :k] - np.eye(k))) <= 1e-10
    # apply, several lambdas at once, FP64 and FP32
    R = np.random.default_rng(2).standard_normal((w.n, 3))
    lams = np.array([0.01, 1.0, 30.0])
    Zo = o.precond_apply(Uo, lho, lams, R)
    Z = nys.nys_precond_apply(P, T(lams), T(R), 0).cpu().numpy()
    assert np.max(np.abs(Z - Zo)) <= 1e-8 * np.max(np.abs(Zo))
    Z32 = nys.nys_precond_apply(P, T(lams), T(R, torch.float32), 1).double().cpu().numpy()
    assert np.max(np.abs(Z32 - Zo)) <= 1e-4 * np.max(np.abs(Zo))


def test_precond_low_precision_sketch_is_valid(nys):
    """FP32 and bf16/fp16-split sketches: the preconditioner stays SPD (U orthonormal,
    lam_hat >= 0) and close to the FP64 one."""
    w = ni.small_problem(1500, 10, seed=3, r=60)
    Om = ni.gaussian_test_matrix(w.n, w.r, 3)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    _, lho, _ = o.nystrom(lambda V: K @ V, Om)
    for prec in (1, 2, 3, 4, 5):
        _, P = build(nys, w.X, Om, w.kind, w.sigma, prec)
        lh = P.lam_hat.cpu().numpy()
        U = P.U.cpu().numpy()
        k = P.rank
        assert np.all(lh >= 0)
        assert np.max(np.abs(U[:, :k].T @ U[:, :k] - np.eye(k))) <= 1e-8
        assert np.max(np.abs(lh[:10] - lho[:10])) <= 1e-3 * lho[0]


def test_sketch_rank_deficient_omega_is_reported(nys):
    w = ni.small_problem(200, 4, seed=4, r=8)
    Om = ni.gaussian_test_matrix(w.n, w.r, 4)
    Om[:, 3] = Om[:, 2]       # duplicated column: Omega^T Omega singular
    with pytest.raises(nys.NysError) as e:
        build(nys, w.X, Om, w.kind, w.sigma)
    assert e.value.code == nys.ENOTPD


# ------------------------------------------------------------------ solve

def test_solve_plain_fp64_workload_matches_cholesky(nys):
    w = ni.plain_fp64(0)
    Om = ni.gaussian_test_matrix(w.n, w.r, 0)
    tX, P = build(nys, w.X, Om, w.kind, w.sigma)
    x, info, rc = nys.nyspcg_solve(tX, T(w.B), w.lambdas, w.kind, w.sigma, P, tol=1e-10, prec=0, check_true=True)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    ref = o.direct_solve(K, w.B[:, 0], w.lambdas[0])
    xs = x.cpu().numpy().reshape(-1)
    rel = np.linalg.norm(xs - ref) / np.linalg.norm(ref)
    print("plain fp64: iters", info[0]["iters"], "rel err", rel, "true relres", info[0]["relres_true"])
    assert rc == nys.OK
    assert rel <= 1e-6
    assert info[0]["relres_true"] <= 1e-9
    # the same workload at its own tolerance 1e-8
    x8, info8, _ = nys.nyspcg_solve(tX, T(w.B), w.lambdas, w.kind, w.sigma, P, tol=1e-8, prec=0)
    assert info8[0]["relres_recursive"] <= 1e-8
    # iterations follow the oracle's textbook PCG closely
    _, it_o, _, _ = o.nyspcg_dense(w.X, w.B, w.lambdas, w.kind, w.sigma, Om, tol=1e-8)
    assert abs(info8[0]["iters"] - it_o[0]) <= 2


def test_plain_cg_matches_cholesky(nys):
    w = ni.small_problem(800, 5, seed=5, lam=2.0)
    tX = T(w.X)
    x, info, rc = nys.nyspcg_solve(tX, T(w.B), w.lambdas, w.kind, w.sigma, None, tol=1e-11, prec=0)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    ref = o.direct_solve(K, w.B[:, 0], w.lambdas[0])
    assert np.linalg.norm(x.cpu().numpy().reshape(-1) - ref) <= 1e-8 * np.linalg.norm(ref)


def test_lambda_grid_and_many_rhs_match_independent_solves(nys):
    w = ni.small_problem(700, 6, seed=6, nrhs=3, r=30)
    Om = ni.gaussian_test_matrix(w.n, w.r, 6)
    tX, P = build(nys, w.X, Om, w.kind, w.sigma)
    lams = [0.05, 0.7, 9.0, 120.0]
    B = w.B.copy()
    B[:, 1] = 0.0          # a zero right-hand side: x = 0 after 0 iterations
    X, info, rc = nys.nyspcg_solve(tX, T(B), lams, w.kind, w.sigma, P, tol=1e-10, prec=0, check_true=True)
    X = X.cpu().numpy()
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    for c in range(12):
        lam, j = lams[c // 3], c % 3
        ref = o.direct_solve(K, B[:, j], lam)
        if j == 1:
            assert np.all(X[:, c] == 0) and info[c]["iters"] == 0
            continue
        assert np.linalg.norm(X[:, c] - ref) <= 1e-6 * np.linalg.norm(ref), c
        assert info[c]["relres_true"] <= 1e-9
    # larger lambda converges in fewer iterations
    its = [info[l * 3]["iters"] for l in range(4)]
    assert its == sorted(its, reverse=True)


def test_iteration_cap_reports_not_converged(nys):
    w = ni.small_problem(500, 5, seed=7, lam=0.01)
    tX = T(w.X)
    x, info, rc = nys.nyspcg_solve(tX, T(w.B), w.lambdas, w.kind, w.sigma, None, tol=1e-12, max_iters=3, prec=0)
    assert rc == nys.NOT_CONVERGED and info[0]["iters"] == 3 and info[0]["status"] == nys.NOT_CONVERGED
    assert torch.isfinite(x).all()


def test_nan_rhs_is_reported(nys):
    w = ni.small_problem(300, 4, seed=8)
    B = w.B.copy()
    B[5, 0] = np.nan
    with pytest.raises(nys.NysError) as e:
        nys.nyspcg_solve(T(w.X), T(B), w.lambdas, w.kind, w.sigma, None, tol=1e-8, prec=0)
    assert e.value.code == nys.ENUMERIC


@pytest.mark.parametrize("prec,mode,every", [(1, 0, 20), (2, 0, 20), (2, 1, 20), (5, 1, 20), (5, 1, 0),
                                              (5, 2, 0), (3, 0, 0)])
def test_low_precision_with_fp64_refinement_reaches_true_tolerance(nys, prec, mode, every):
    """Low-precision products (FP32, BF16X3, D6, F16X3_D10) with float32 CG accept a
    column only on its float64 true residual, with periodic (every 20) or cycle
    (every 0) refinement in each restart mode; the result is checked against the
    oracle's direct solve."""
    w = ni.small_problem(3000, 10, seed=9, lam=0.3, r=80)
    Om = ni.gaussian_test_matrix(w.n, w.r, 9)
    tX, P = build(nys, w.X, Om, w.kind, w.sigma, prec)
    x, info, rc = nys.nyspcg_solve(tX, T(w.B), w.lambdas, w.kind, w.sigma, P, tol=1e-6, prec=prec,
                                   refine_every=every, refine_mode=mode, check_true=True)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    ref = o.direct_solve(K, w.B[:, 0], w.lambdas[0])
    xs = x.cpu().numpy().reshape(-1)
    true = o.relative_residual(K, xs, w.B[:, 0], w.lambdas[0])[0]
    err = np.linalg.norm(xs - ref) / np.linalg.norm(ref)
    print(f"prec {prec} mode {mode}: iters {info[0]['iters']} refinements {info[0]['refinements']} "
          f"true relres {true:.3e} (lib {info[0]['relres_true']:.3e}) rel err vs oracle {err:.3e}")
    assert rc == nys.OK
    assert true <= 1e-6
    assert abs(info[0]["relres_true"] - true) <= 1e-8


def test_fp32_without_refinement_stops_on_recursive_residual(nys):
    w = ni.small_problem(2000, 8, seed=10, lam=1.0, r=50)
    Om = ni.gaussian_test_matrix(w.n, w.r, 10)
    tX, P = build(nys, w.X, Om, w.kind, w.sigma, 1)
    x, info, rc = nys.nyspcg_solve(tX, T(w.B), w.lambdas, w.kind, w.sigma, P, tol=1e-5, prec=1,
                                   refine_every=-1, check_true=True)
    assert info[0]["refinements"] == 0 and info[0]["relres_recursive"] <= 1e-5
    assert info[0]["relres_true"] <= 1e-4


@pytest.mark.parametrize("prec", [0, 2, 5])
def test_solve_deterministic(nys, prec):
    """Bitwise repeatable solves: ordered reductions, no atomics (12 columns put the
    float64 product on its pipelined tile)."""
    w = ni.small_problem(1200, 6, seed=11, nrhs=6, r=30)
    Om = ni.gaussian_test_matrix(w.n, w.r, 11)
    tX, P = build(nys, w.X, Om, w.kind, w.sigma, prec)
    kw = dict(tol=1e-6, prec=prec) if prec == 0 else dict(tol=1e-6, prec=prec, refine_every=20)
    a, _, _ = nys.nyspcg_solve(tX, T(w.B), [0.5, 5.0], w.kind, w.sigma, P, **kw)
    b, _, _ = nys.nyspcg_solve(tX, T(w.B), [0.5, 5.0], w.kind, w.sigma, P, **kw)
    assert torch.equal(a, b)


# ------------------------------------------------------------------ backward

@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
def test_backward_matches_dense_gradient(nys, kind):
    w = ni.small_problem(900, 6, seed=12, kind=kind, r=40)
    X, y = w.X[:750], w.B[:750, 0]
    Xv, yv = w.X[750:], w.B[750:, 0]
    lam, sig = 0.8, 2.0
    L, dlam_o, dsig_o, x_o, a_o = o.validation_loss_grad(X, y, Xv, yv, kind, sig, lam)
    Om = ni.gaussian_test_matrix(750, 40, 12)
    tX, P = build(nys, X, Om, kind, sig)
    x, info, _ = nys.nyspcg_solve(tX, T(y), [lam], kind, sig, P, tol=1e-12, prec=0)
    x = x.reshape(-1)
    # dL/dx through the validation prediction K_vt x, then the adjoint solve
    tXv = T(Xv)
    pred = nys.kernel_matvec(tXv, tX, x, kind, sig, 0)
    e = (2.0 / len(yv)) * (pred - T(yv))
    gx = nys.kernel_matvec(tX, tXv, e, kind, sig, 0)
    adj, dlam, dsig_impl, binfo = nys.nyspcg_backward(tX, lam, x, gx, kind, sig, P, tol=1e-12, prec=0)
    dsig_explicit = float(torch.dot(e, nys.kernel_matvec(tXv, tX, x, kind, sig, 0, deriv=1)))
    dsig = dsig_explicit + dsig_impl
    print(f"kind {kind}: dlam {dlam:.10e} vs {dlam_o:.10e}; dsig {dsig:.10e} vs {dsig_o:.10e}")
    assert np.linalg.norm(adj.cpu().numpy() - a_o) <= 1e-8 * np.linalg.norm(a_o)
    assert dlam == pytest.approx(dlam_o, rel=1e-7)
    assert dsig == pytest.approx(dsig_o, rel=1e-7)


@pytest.mark.parametrize("prec,mode", [(3, 0), (3, 1), (4, 1), (5, 1)])
def test_batched_lambda_grid_bf16x3_cycles_reach_true_tolerance(nys, prec, mode):
    """The batched workload's recipe at n = 4000 (sign labels, lambdas from 1e-7 n to
    1e-3 n): BF16X3_D6 / BF16X3_D10 / F16X3_D10 products, float32 CG, cycle refinement.  Every column
    must meet the float64 true relative residual 1e-6, checked by the oracle's dense residual."""
    w = ni.batched_lambda_grid(0, n=4000, nrhs=3, nlam=4, r=120)
    Om = ni.gaussian_test_matrix(w.n, w.r, 0)
    tX, P = build(nys, w.X, Om, w.kind, w.sigma, prec)
    X, info, rc = nys.nyspcg_solve(tX, T(w.B), w.lambdas, w.kind, w.sigma, P, tol=1e-6, prec=prec,
                                   refine_every=0, refine_mode=mode, refine_reduction=1e-3, max_iters=3000)
    X = X.cpu().numpy()
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    worst = 0.0
    for c in range(12):
        lam, j = w.lambdas[c // 3], c % 3
        rel = o.relative_residual(K, X[:, c], w.B[:, j], lam)[0]
        worst = max(worst, rel)
        assert abs(rel - info[c]["relres_true"]) <= 1e-3 * rel + 1e-12
    its = [info[l * 3]["iters"] for l in range(4)]
    refs = [info[l * 3]["refinements"] for l in range(4)]
    print(f"prec {prec} mode {mode}: iters per lambda {its} refinements {refs} worst true relres {worst:.3e}")
    assert rc == nys.OK and worst <= 1e-6


def test_backward_low_precision_adjoint(nys):
    """The adjoint solve on F16X3_D10 products with float64 refinement (tol 1e-9) gives
    the dense oracle's gradient to the accuracy the tolerance allows."""
    w = ni.small_problem(900, 6, seed=12, kind=o.RBF, r=40)
    X, y = w.X[:750], w.B[:750, 0]
    Xv, yv = w.X[750:], w.B[750:, 0]
    lam, sig = 0.8, 2.0
    L, dlam_o, dsig_o, x_o, a_o = o.validation_loss_grad(X, y, Xv, yv, o.RBF, sig, lam)
    Om = ni.gaussian_test_matrix(750, 40, 12)
    tX, P = build(nys, X, Om, o.RBF, sig, 5)
    x, info, rc = nys.nyspcg_solve(tX, T(y), [lam], o.RBF, sig, P, tol=1e-9, prec=5, refine_every=0,
                                   refine_mode=1)
    assert rc == nys.OK
    x = x.reshape(-1)
    tXv = T(Xv)
    pred = nys.kernel_matvec(tXv, tX, x, o.RBF, sig, 0)
    e = (2.0 / len(yv)) * (pred - T(yv))
    gx = nys.kernel_matvec(tX, tXv, e, o.RBF, sig, 0)
    adj, dlam, dsig_impl, binfo = nys.nyspcg_backward(tX, lam, x, gx, o.RBF, sig, P, tol=1e-9, prec=5,
                                                      refine_every=0, refine_mode=1)
    dsig = float(torch.dot(e, nys.kernel_matvec(tXv, tX, x, o.RBF, sig, 0, deriv=1))) + dsig_impl
    print(f"adjoint iters {binfo['iters']} refinements {binfo['refinements']}; dlam {dlam:.8e} vs {dlam_o:.8e}; "
          f"dsig {dsig:.8e} vs {dsig_o:.8e}")
    assert np.linalg.norm(adj.cpu().numpy() - a_o) <= 1e-6 * np.linalg.norm(a_o)
    assert dlam == pytest.approx(dlam_o, rel=1e-5)
    assert dsig == pytest.approx(dsig_o, rel=1e-5)
