"""GPU parity of NysADMM on the bounded elastic net (eq. experiment-bounded-en) against
the CPU float64 oracle (same steps, same test matrices) and against SciPy's exact
bounded least-squares solution, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import nys_inputs as ni
import oracle as o

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, torch.float64)


def bvls(X, y, lam1, lam2):
    from scipy.optimize import lsq_linear
    n, p = X.shape
    Xc = X - X.mean(axis=0)
    yc = y - y.mean()
    A = np.vstack([Xc / math.sqrt(n), math.sqrt(lam2) * np.eye(p)])
    b = np.concatenate([yc / math.sqrt(n), -lam1 / math.sqrt(lam2) * np.ones(p)])
    return lsq_linear(A, b, bounds=(0.0, 1.0), method="bvls", tol=1e-14).x


@pytest.mark.parametrize("n,d_in,p,rank,seed", [(800, 8, 48, 16, 80), (301, 5, 37, 7, 81), (2000, 10, 130, 50, 82)])
def test_admm_matches_oracle_and_exact_solution(nys, n, d_in, p, rank, seed):
    """Tight tolerances: the GPU run follows the oracle's iteration (same penalty
    decisions, iteration counts within a few) and lands on the exact solution."""
    print(f"case admm n={n} p={p} rank={rank} seed={seed}", flush=True)
    pr = ni.elastic_net_problem(n, d_in, p, seed=seed)
    cfg = dict(rank=rank, eps_abs=1e-10, eps_rel=1e-10, max_iters=4000, seed=seed)
    w, info, rc = nys.nys_admm_elastic_net(T(pr.X), T(pr.y), pr.lam1, pr.lam2, **cfg)
    ref = o.nysadmm_elastic_net(pr.X, pr.y, pr.lam1, pr.lam2, rank=rank, eps_abs=1e-10, eps_rel=1e-10,
                                max_iters=4000, seed=seed)
    exact = bvls(pr.X, pr.y, pr.lam1, pr.lam2)
    wh = w.cpu().numpy()
    print(f"  gpu {info['iters']} iterations ({info['pcg_iters']} PCG), oracle {ref['iters']} "
          f"({sum(ref['pcg_iters'])} PCG); rho {info['rho']} vs {ref['rho']}", flush=True)
    assert rc == nys.OK and info["converged"] == 1 and ref["converged"]
    assert abs(info["iters"] - ref["iters"]) <= max(3, 0.02 * ref["iters"])
    assert info["rho"] == ref["rho"]
    # the same iteration as the oracle's, up to rounding
    assert np.max(np.abs(wh - ref["w"])) <= 1e-9
    assert np.all(wh >= 0.0) and np.all(wh <= 1.0)
    # distance to the exact minimiser: the objective is lam2-strongly convex, so
    # |w - w*| <= dist(0, subdifferential at w) / lam2 <= sqrt(p) kkt_inf(w) / lam2,
    # for the GPU point and for the BVLS reference alike
    kkt = o.elastic_net_kkt(pr.X, pr.y, wh, pr.lam1, pr.lam2)
    kkt_ref = o.elastic_net_kkt(pr.X, pr.y, exact, pr.lam1, pr.lam2)
    assert kkt <= 1e-8
    bound = math.sqrt(p) * (kkt + kkt_ref) / pr.lam2
    assert np.max(np.abs(wh - exact)) <= bound
    mu = pr.X.mean(axis=0)
    assert abs(info["intercept"] - (pr.y.mean() - mu @ exact)) <= np.sum(np.abs(mu)) * bound + 1e-12
    assert info["r_pri"] <= info["eps_pri"] and info["r_dual"] <= info["eps_dual"]


def test_admm_default_tolerances_and_penalty_updates(nys):
    """The paper's default configuration (eps 1e-4) from a badly balanced start
    (rho = 100, updated every 5 iterations): the penalty moves, and the GPU takes the
    oracle's decisions and stops where it does."""
    pr = ni.elastic_net_problem(1500, 8, 64, seed=83)
    cfg = dict(rank=20, rho=100.0, rho_update_freq=5, seed=83)
    w, info, rc = nys.nys_admm_elastic_net(T(pr.X), T(pr.y), pr.lam1, pr.lam2, **cfg)
    ref = o.nysadmm_elastic_net(pr.X, pr.y, pr.lam1, pr.lam2, **cfg)
    print(f"gpu {info['iters']} it rho {info['rho']}; oracle {ref['iters']} it rho {ref['rho']}", flush=True)
    assert rc == nys.OK and ref["converged"]
    assert ref["rho"] != 100.0 and info["rho"] == ref["rho"]
    assert abs(info["iters"] - ref["iters"]) <= 2
    assert np.max(np.abs(w.cpu().numpy() - ref["w"])) <= 1e-6
    assert o.elastic_net_kkt(pr.X, pr.y, w.cpu().numpy(), pr.lam1, pr.lam2) <= 1e-2


def test_admm_ridge_special_case(nys):
    """lam1 = 0 and bounds that never bind: the ridge solution."""
    pr = ni.elastic_net_problem(700, 6, 40, seed=84)
    lam2 = 0.05
    w, info, rc = nys.nys_admm_elastic_net(T(pr.X), T(pr.y), 0.0, lam2, lo=-1e6, hi=1e6, rank=10, eps_abs=1e-11,
                                           eps_rel=1e-11, max_iters=4000)
    Xc = pr.X - pr.X.mean(axis=0)
    ref = np.linalg.solve(Xc.T @ Xc / 700 + lam2 * np.eye(40), Xc.T @ (pr.y - pr.y.mean()) / 700)
    assert rc == nys.OK and np.max(np.abs(w.cpu().numpy() - ref)) <= 1e-8


def test_admm_iteration_cap_and_errors(nys):
    pr = ni.elastic_net_problem(400, 5, 24, seed=85)
    X, y = T(pr.X), T(pr.y)
    w, info, rc = nys.nys_admm_elastic_net(X, y, pr.lam1, pr.lam2, rank=8, max_iters=3, eps_abs=1e-12,
                                           eps_rel=1e-12)
    assert rc == nys.NOT_CONVERGED and info["iters"] == 3 and info["converged"] == 0
    assert torch.all(w >= 0) and torch.all(w <= 1)
    ybad = y.clone()
    ybad[7] = float("nan")
    with pytest.raises(nys.NysError):
        nys.nys_admm_elastic_net(X, ybad, pr.lam1, pr.lam2, rank=8)
    with pytest.raises(nys.NysError):
        nys.nys_admm_elastic_net(X, y, pr.lam1, pr.lam2, rank=25)          # rank > p
    with pytest.raises(nys.NysError):
        nys.nys_admm_elastic_net(X, y, pr.lam1, pr.lam2, alpha=2.0)
