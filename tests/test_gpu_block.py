"""GPU parity of block PCG (O'Leary; the right-hand sides of each lambda share one
block Krylov space) against the oracle's block_pcg and direct solves, through the C ABI."""
import numpy as np
import pytest
import torch

import nys_inputs as ni
import oracle as o

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, torch.float64)


def setup(n, d, nrhs, r, seed, kind=o.RBF):
    w = ni.small_problem(n, d, seed=seed, nrhs=nrhs, kind=kind, r=r)
    B = np.where(w.X @ np.random.default_rng(seed).standard_normal((d, nrhs)) >= 0, 1.0, -1.0)
    Om = ni.gaussian_test_matrix(n, r, seed)
    return w, B, Om


@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
def test_fp64_block_pcg_matches_oracle(nys, kind):
    """Float64 block PCG: iteration counts near the oracle's block_pcg, solutions equal to
    direct solves, and fewer iterations than column PCG on the same systems."""
    n, nrhs, lams = 1500, 8, [1e-3, 1e-1, 10.0]
    w, B, Om = setup(n, 6, nrhs, 40, 100 + kind, kind)
    K = o.kernel_matrix(w.X, w.X, kind, w.sigma)
    U, lh, _ = o.nystrom(lambda V: K @ V, Om)
    tX = T(w.X)
    P = nys.build_preconditioner(tX, T(Om), kind, w.sigma, nys.FP64)
    tol = 1e-10
    Xs, info, rc = nys.nyspcg_solve(tX, T(B), lams, kind, w.sigma, P, tol=tol, max_iters=3000, prec=nys.FP64,
                                    block=True, check_true=True)
    _, info_c, _ = nys.nyspcg_solve(tX, T(B), lams, kind, w.sigma, P, tol=tol, max_iters=3000, prec=nys.FP64)
    assert rc == nys.OK
    Xh = Xs.cpu().numpy()
    for li, lam in enumerate(lams):
        Xo, it_o, _ = o.block_pcg(lambda V: K @ V + lam * V, B, lambda R: o.precond_apply(U, lh, lam, R), tol=tol,
                                  max_iters=3000)
        it_g = info[li * nrhs]["iters"]
        it_col = max(info_c[li * nrhs + j]["iters"] for j in range(nrhs))
        print(f"kind {kind} lambda {lam:g}: block {it_g} iterations (oracle {it_o}), column PCG {it_col}", flush=True)
        # block CG in floating point loses conjugacy at its own pace (a restart on a
        # near-singular s x s system costs iterations): within 25% of the oracle's run,
        # and never more iterations than the column solver
        assert it_g <= 1.25 * it_o + 3 and it_o <= 1.25 * it_g + 3
        assert it_g <= it_col
        ref = np.linalg.solve(K + lam * np.eye(n), B)
        cols = slice(li * nrhs, (li + 1) * nrhs)
        assert np.max(np.abs(Xh[:, cols] - ref)) <= 1e-6 * np.max(np.abs(ref))
        for j in range(nrhs):
            c = info[li * nrhs + j]
            assert c["status"] == nys.OK and c["relres_recursive"] <= tol
            assert c["relres_true"] <= 10 * tol


@pytest.mark.parametrize("prec", [1, 5, 6])
def test_low_precision_block_pcg_reaches_true_tolerance(nys, prec):
    """Float32 vectors with the FP32, F16X3_D10 or F16X3_D6 product, block refinement cycles: every
    column's dense float64 oracle residual meets 1e-6 and equals the reported one."""
    n, nrhs, lams = 4000, 16, [1e-7 * 4000, 1e-5 * 4000, 1e-3 * 4000]
    w = ni.batched_lambda_grid(7, n=n, nrhs=nrhs, nlam=3, r=100)
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    tX = T(w.X)
    P = nys.build_preconditioner(tX, T(ni.gaussian_test_matrix(n, 100, 7)), w.kind, w.sigma, prec)
    Xs, info, rc = nys.nyspcg_solve(tX, T(w.B), lams, w.kind, w.sigma, P, tol=1e-6, max_iters=3000, prec=prec,
                                    refine_every=0, refine_mode=1, block=True)
    print(f"prec {prec}: iterations per lambda {[info[l * nrhs]['iters'] for l in range(3)]}, refinements "
          f"{[info[l * nrhs]['refinements'] for l in range(3)]}", flush=True)
    assert rc == nys.OK
    Xh = Xs.cpu().numpy()
    for li, lam in enumerate(lams):
        for j in range(nrhs):
            c = li * nrhs + j
            rr = o.relative_residual(K, Xh[:, c], w.B[:, j], lam)[0]
            assert rr <= 1e-6
            assert abs(rr - info[c]["relres_true"]) <= 1e-3 * rr + 1e-12


def test_block_pcg_is_deterministic(nys):
    w, B, Om = setup(900, 5, 4, 30, 110)
    tX = T(w.X)
    P = nys.build_preconditioner(tX, T(Om), w.kind, w.sigma, nys.FP64)
    a, _, _ = nys.nyspcg_solve(tX, T(B), [0.01, 1.0], w.kind, w.sigma, P, tol=1e-8, prec=nys.F16X3_D10,
                               refine_every=0, block=True)
    b, _, _ = nys.nyspcg_solve(tX, T(B), [0.01, 1.0], w.kind, w.sigma, P, tol=1e-8, prec=nys.F16X3_D10,
                               refine_every=0, block=True)
    assert torch.equal(a, b)


def test_block_pcg_argument_errors(nys):
    w, B, Om = setup(300, 4, 2, 10, 111)
    tX = T(w.X)
    with pytest.raises(nys.NysError):          # more than 64 right-hand sides per lambda
        nys.nyspcg_solve(tX, T(np.ones((300, 65))), [1.0], w.kind, w.sigma, None, block=True)
    Bz = B.copy()
    Bz[:, 1] = 0.0
    with pytest.raises(nys.NysError):          # a zero right-hand side beside a non-zero one
        nys.nyspcg_solve(tX, T(Bz), [1.0], w.kind, w.sigma, None, block=True)
    with pytest.raises(nys.NysError):          # periodic refinement is not a block mode
        nys.nyspcg_solve(tX, T(B), [1.0], w.kind, w.sigma, None, prec=nys.FP32, refine_every=20, block=True)
    Z, info, rc = nys.nyspcg_solve(tX, T(np.zeros((300, 2))), [1.0], w.kind, w.sigma, None, block=True)
    assert rc == nys.OK and float(Z.abs().max()) == 0.0 and all(c["iters"] == 0 for c in info)
