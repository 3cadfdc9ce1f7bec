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
    for prec in (1, 2, 3, 4, 5, 6):
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
                                              (5, 2, 0), (3, 0, 0), (6, 1, 0)])
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
    dsig_explicit = nys.kernel_dot(tXv, tX, e, x, kind, sig, deriv=1)
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
    dsig = nys.kernel_dot(tXv, tX, e, x, o.RBF, sig, deriv=1) + dsig_impl
    print(f"adjoint iters {binfo['iters']} refinements {binfo['refinements']}; dlam {dlam:.8e} vs {dlam_o:.8e}; "
          f"dsig {dsig:.8e} vs {dsig_o:.8e}")
    assert np.linalg.norm(adj.cpu().numpy() - a_o) <= 1e-6 * np.linalg.norm(a_o)
    assert dlam == pytest.approx(dlam_o, rel=1e-5)
    assert dsig == pytest.approx(dsig_o, rel=1e-5)


@pytest.mark.parametrize("prec,n,nrhs,lam_lo,lam_hi,r", [(5, 10_000, 64, 1e-7, 1e-3, 500),
                                                          (6, 10_000, 64, 1e-7, 1e-3, 500),
                                                          (2, 4_000, 40, 1e-5, 1e-1, 200)])
def test_headline_column_count_matches_oracle(nys, prec, n, nrhs, lam_lo, lam_hi, r):
    """The batched workload's recipe at the headline's column count: nrhs sign labels x
    8 lambdas log-spaced over [lam_lo n, lam_hi n] (512 columns for F16X3_D10 and D6, 320 for
    BF16X3, whose three-term distance needs lambda above ~1e-5 n).  The solve runs its
    256-column chunks with narrower last chunks, compacts the active columns as they
    converge across widths, and batches float64 refinements of 48 to 256 columns.
    Every column's float64 relative residual, recomputed by the oracle with the dense
    K, must meet 1e-6 (table tab:rlaopt-pcg-stopping: the criterion holds for every
    right-hand side), and the solver's own float64 residual must agree with it."""
    w = ni.batched_lambda_grid(0, n=n, nrhs=nrhs, nlam=8, r=r)
    lams = list(np.logspace(math.log10(lam_lo * n), math.log10(lam_hi * n), 8))
    Om = ni.gaussian_test_matrix(w.n, w.r, 0)
    tX, P = build(nys, w.X, Om, w.kind, w.sigma, prec)
    print(f"case headline columns prec={prec} n={n} columns={8 * nrhs}", flush=True)
    X, info, rc = nys.nyspcg_solve(tX, T(w.B), lams, w.kind, w.sigma, P, tol=1e-6, prec=prec,
                                   refine_every=0, refine_mode=1, refine_reduction=1e-3, max_iters=1000)
    X = X.cpu().numpy()
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    m = 8 * nrhs
    B = w.B[:, [c % nrhs for c in range(m)]]
    lam_col = np.array([lams[c // nrhs] for c in range(m)])
    res = K @ X + lam_col * X - B
    rel = np.linalg.norm(res, axis=0) / np.linalg.norm(B, axis=0)
    mine = np.array([c["relres_true"] for c in info])
    its = [max(info[l * nrhs + j]["iters"] for j in range(nrhs)) for l in range(8)]
    refs = sum(c["refinements"] for c in info)
    print(f"  iters per lambda {its}, refinements {refs}, worst oracle relres {rel.max():.3e}", flush=True)
    assert rc == nys.OK
    assert np.all(rel <= 1e-6), f"{int(np.sum(rel > 1e-6))} columns above 1e-6 (worst {rel.max():.3e})"
    assert np.all(np.abs(rel - mine) <= 1e-3 * rel + 1e-12)


def test_non_finite_points_in_solve_and_sketch(nys):
    """NaN coordinates reach NYS_ENUMERIC in the sketch and in the solve."""
    w = ni.small_problem(400, 5, seed=2, r=20)
    X = w.X.copy()
    X[123, 2] = np.nan
    tX = T(X)
    with pytest.raises(nys.NysError) as ei:
        nys.build_preconditioner(tX, T(ni.gaussian_test_matrix(w.n, w.r, 2)), w.kind, w.sigma, 0)
    assert ei.value.code == nys.ENUMERIC
    for prec in (0, 5, 6):
        with pytest.raises(nys.NysError) as ei:
            nys.nyspcg_solve(tX, T(w.B), w.lambdas, w.kind, w.sigma, None, tol=1e-8, prec=prec,
                             refine_every=0)
        assert ei.value.code == nys.ENUMERIC


# ------------------------------------------------------------------ device test matrix, const Omega

def test_device_test_matrix_matches_oracle_generator(nys):
    """nys_test_matrix (Philox4x32-10 + Box-Muller on the device) against the oracle's
    own implementation of the same published definitions, element by element."""
    from oracle import philox as ph
    for n, r, seed in ((1000, 37, 0), (777, 500, 2**40 + 12345), (5, 3, 7)):
        print(f"case test matrix n={n} r={r} seed={seed}", flush=True)
        got = nys.nys_test_matrix(seed, n, r).cpu().numpy()
        ref = ph.gaussian_test_matrix(n, r, seed)
        assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_sketch_keeps_omega_and_seed_mode_matches_oracle(nys):
    """nys_sketch reads Omega without writing it, and with Omega NULL draws the test
    matrix from the seed: the preconditioner then equals the oracle's Nystrom
    approximation for the oracle-drawn matrix of the same seed."""
    from oracle import philox as ph
    w = ni.small_problem(700, 6, seed=31, r=40)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    Om = ni.gaussian_test_matrix(w.n, w.r, 31)
    tX, tOm = T(w.X), T(Om)
    before = tOm.clone()
    Y, Q = nys.nys_sketch(tX, tOm, w.kind, w.sigma, 0)
    torch.cuda.synchronize()
    assert torch.equal(before, tOm)
    assert torch.allclose(Q.T @ Q, torch.eye(w.r, dtype=torch.float64, device=DEV), atol=1e-12)
    P = nys.build_preconditioner(tX, None, w.kind, w.sigma, 0, r=w.r, seed=99)
    _, lho, _ = o.nystrom(lambda V: K @ V, ph.gaussian_test_matrix(w.n, w.r, 99))
    assert np.max(np.abs(P.lam_hat.cpu().numpy() - lho)) <= 1e-9 * lho[0]


def test_kernel_dot_matches_oracle(nys):
    rng = np.random.default_rng(41)
    Xr, Xc = rng.standard_normal((300, 7)), rng.standard_normal((500, 7))
    u, v = rng.standard_normal(300), rng.standard_normal(500)
    for kind in (o.RBF, o.LAPLACIAN):
        for deriv in (0, 1):
            M = o.kernel_dsigma_matrix(Xr, Xc, kind, 1.7) if deriv else o.kernel_matrix(Xr, Xc, kind, 1.7)
            ref = float(u @ M @ v)
            got = nys.kernel_dot(T(Xr), T(Xc), T(u), T(v), kind, 1.7, deriv)
            assert abs(got - ref) <= 1e-12 * float(np.abs(u) @ np.abs(M) @ np.abs(v))


# ------------------------------------------------------------------ rank adaptation, damping modes

@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
def test_adaptive_rank_matches_oracle(nys, kind):
    """nys_precond_adaptive against the oracle's rank adaptation on the same Philox test
    matrix and start vector: the same final rank, the same approximate eigenvalues and
    error estimate, and the adaptive damping shift (smallest retained lam_hat)."""
    from oracle import philox as ph
    w = ni.small_problem(1200, 5, seed=33, kind=kind, r=8)
    K = o.kernel_matrix(w.X, w.X, kind, w.sigma)
    seed, rinit, rmax = 5, 8, 128
    Om = ph.gaussian_test_matrix(w.n, rmax, seed)
    v0 = ph.gaussian_test_matrix(w.n, 1, seed + 1)[:, 0]
    for tol in (1e-1, 1e-3, 1e-12):
        Uo, lho, nuo, lo, erro = o.nystrom_adaptive(lambda V: K @ V, Om, rinit, rmax, 10, tol, v0)
        print(f"case adaptive kind={kind} tol={tol}: oracle rank {lo}, error {erro:.4e} vs {tol * lho[0]:.4e}",
              flush=True)
        P, err = nys.nys_precond_adaptive(T(w.X), kind, w.sigma, rinit, rmax, 10, tol, "adaptive", 0, seed)
        assert P.r == lo
        lh = P.lam_hat.cpu().numpy()
        assert np.max(np.abs(lh - lho)) <= 1e-8 * lho[0]
        assert abs(err - erro) <= 1e-6 * abs(erro) + 1e-10 * lho[0]
        assert P.shift == pytest.approx(o.damping_shift(lho[:P.rank], "adaptive"), rel=1e-8)
        Kh = (P.U.cpu().numpy() * lh) @ P.U.cpu().numpy().T
        assert np.max(np.abs(Kh - o.nystrom_matrix(Uo, lho))) <= 1e-8 * lho[0]


def test_adaptive_damping_preconditioner_apply_and_solve(nys):
    """The adaptive damping (lambda + smallest retained lam_hat) in the apply and in
    NysPCG: the apply matches the oracle's closed form, and the solve matches Cholesky."""
    w = ni.small_problem(900, 6, seed=34, r=30, lam=0.05)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    P, _ = nys.nys_precond_adaptive(T(w.X), w.kind, w.sigma, 30, 30, 0, 1e-2, "adaptive", 0, 3)
    assert P.shift > 0
    U, lh = P.U.cpu().numpy(), P.lam_hat.cpu().numpy()
    R = np.random.default_rng(8).standard_normal((w.n, 2))
    lams = np.array([0.05, 2.0])
    Z = nys.nys_precond_apply(P, T(lams), T(R), 0).cpu().numpy()
    Zo = o.precond_apply(U, lh, lams, R, shift=P.shift)
    assert np.max(np.abs(Z - Zo)) <= 1e-10 * np.max(np.abs(Zo))
    x, info, rc = nys.nyspcg_solve(T(w.X), T(w.B), w.lambdas, w.kind, w.sigma, P, tol=1e-11, prec=0)
    ref = o.direct_solve(K, w.B[:, 0], w.lambdas[0])
    assert rc == nys.OK
    assert np.linalg.norm(x.cpu().numpy().reshape(-1) - ref) <= 1e-7 * np.linalg.norm(ref)
