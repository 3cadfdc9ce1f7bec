"""GPU parity of kernel_matvec against the CPU float64 oracle, element by element.

Tolerances are error bounds written against |K| |V| (row by row), derived from
the arithmetic of each precision:
  * the exponent t = kappa (2 x.y - |x|^2 - |y|^2) is formed by one MFMA chain;
    its absolute error is at most c u kappa (|x| + |y|)^2, so each kernel value
    carries a relative error of about u (1 + kappa_max (|x| + |y|)^2);
  * accumulation over the nc columns adds at most (nc/4 + 16) u relative to
    |K| |V| (sequential per-lane sums of nc/4 terms, then a 4-way reduction);
  * BF16X3 splits both distance operands into bf16 pairs (about 2^-16 relative
    per product) and, with >= 16 columns, also k and V.
"""
import math

import numpy as np
import pytest
import torch

import nys_inputs as ni
import oracle as o

pytestmark = pytest.mark.gpu

U = {0: 2.0 ** -53, 1: 2.0 ** -24, 2: 2.0 ** -16, 3: 2.0 ** -16, 4: 2.0 ** -16, 5: 2.0 ** -16}


def bound(Xr, Xc, V, kind, sigma, prec, deriv=0):
    """Row-wise bound on |gpu - oracle| from the arithmetic of `prec`."""
    K = o.kernel_dsigma_matrix(Xr, Xc, kind, sigma) if deriv else o.kernel_matrix(Xr, Xc, kind, sigma)
    mu = Xc.mean(0)
    nr_ = np.linalg.norm(Xr - mu, axis=1)
    nc_ = np.linalg.norm(Xc - mu, axis=1)
    span = (nr_.max() + nc_.max()) ** 2
    kap = 1.0 / (2 * sigma * sigma) if kind == o.RBF else 1.0
    u = U[prec]
    ent = 16 * u * (1.0 + kap * span)
    if kind == o.LAPLACIAN:
        # d = sqrt(d^2): an absolute error e in d^2 gives sqrt(e) in d near d = 0
        ent = 16 * u * (1.0 + kap * span) + math.sqrt(16 * u * span) / sigma
    if deriv:
        ent *= 4
    acc = (Xc.shape[0] / 4 + 16) * (2.0 ** -53 if prec == 0 else 2.0 ** -24)
    return (ent + acc) * (np.abs(K) @ np.abs(V)) + 1e-300


def run(nys, Xr, Xc, V, kind, sigma, prec, deriv=0, alpha=1.0, beta=0.0, out=None):
    dev = torch.device("cuda")
    tr = torch.from_numpy(np.ascontiguousarray(Xr)).to(dev)
    tc = tr if Xc is Xr else torch.from_numpy(np.ascontiguousarray(Xc)).to(dev)
    dt = torch.float64 if prec == 0 else torch.float32
    tv = torch.from_numpy(np.ascontiguousarray(V)).to(dev, dt)
    to = None if out is None else torch.from_numpy(np.ascontiguousarray(out)).to(dev, dt)
    res = nys.kernel_matvec(tr, tc, tv, kind, sigma, prec, deriv, alpha, beta, to)
    torch.cuda.synchronize()
    return res.double().cpu().numpy()


def check(nys, n_r, n_c, d, m, kind, prec, seed=0, same=True, deriv=0, heavy=False):
    if prec in (4, 5) and d > 24:
        # ten-term split: the packed K extent 10 d + 8 must fit the 256-wide tile
        with pytest.raises(nys.NysError, match="d out of range"):
            run(nys, np.zeros((2, d)), np.zeros((2, d)), np.zeros((2, m)), kind, 1.0, prec, deriv)
        return None, None
    rng = np.random.default_rng(seed)
    Xr = rng.standard_normal((n_r, d))
    if heavy:
        Xr[:, -1] = rng.standard_t(3.0, n_r)
    Xc = Xr if same else rng.standard_normal((n_c, d))
    V = rng.standard_normal((Xc.shape[0], m))
    if prec != 0:
        V = V.astype(np.float32).astype(np.float64)   # the float32 input the GPU sees
    sigma = math.sqrt(d)
    print(f"case n_r={n_r} n_c={Xc.shape[0]} d={d} m={m} kind={kind} prec={prec} deriv={deriv}", flush=True)
    got = run(nys, Xr, Xc, V, kind, sigma, prec, deriv)
    ref = o.kernel_matvec(Xr, Xc, V, kind, sigma, deriv)
    tol = bound(Xr, Xc, V, kind, sigma, prec, deriv)
    err = np.abs(got - ref)
    worst = float(np.max(err / tol))
    assert worst <= 1.0, f"max err/bound = {worst:.3g} (max abs err {err.max():.3g})"
    return got, ref


@pytest.mark.parametrize("prec", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
@pytest.mark.parametrize("n,d,m", [(1, 3, 1), (31, 10, 1), (257, 16, 3), (2000, 10, 1), (700, 20, 8),
                                   (513, 33, 16), (300, 1, 5)])
def test_matvec_small_m(nys, prec, kind, n, d, m):
    check(nys, n, n, d, m, kind, prec, seed=n + d + m)


@pytest.mark.parametrize("prec", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
@pytest.mark.parametrize("n,d,m", [(100, 10, 17), (1000, 16, 64), (777, 20, 50), (1500, 32, 200),
                                   (2000, 10, 300), (600, 13, 24), (500, 5, 40)])
def test_matvec_many_columns(nys, prec, kind, n, d, m):
    check(nys, n, n, d, m, kind, prec, seed=7 * n + m)


@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
@pytest.mark.parametrize("m", [2, 64])
def test_fp64_kernel_entries_over_the_whole_exponent_range(nys, kind, m):
    """Single K entries (V = unit columns) for exponents from 0 down past the float64
    underflow at -745: each within a few ulps plus the rounding of the exponent
    itself; results below 1e-300 (subnormal or flushed) count as zero."""
    n = 600
    x = (np.arange(n, dtype=np.float64) * 0.0703125)[:, None]   # 0 .. 42.1, dyadic
    sigma = 1.0 if kind == o.RBF else 1.0 / 20.0               # exponents down to -887 resp. -842
    V = np.zeros((n, m))
    cols = np.linspace(0, n - 1, m).astype(int)
    V[cols, np.arange(m)] = 1.0
    print(f"case exponent range kind={kind} m={m}", flush=True)
    got = run(nys, x, x, V, kind, sigma, 0)
    ref = o.kernel_matrix(x, x, kind, sigma)[:, cols]
    span = (x.max() - x.mean()) ** 2 * 4
    kap = 1.0 / (2 * sigma * sigma) if kind == o.RBF else 1.0
    u = 2.0 ** -53
    dt = 16 * u * (1.0 + kap * span)                           # error of the exponent
    if kind == o.LAPLACIAN:
        dt = 16 * u * (1.0 + span) + math.sqrt(16 * u * span) / sigma
    tol = ref * (8 * u + dt) + 1e-300
    assert np.all(np.abs(got - ref) <= tol), float(np.max(np.abs(got - ref) / tol))
    assert ref.min() == 0.0 and np.all(got[ref == 0.0] <= 1e-300) and got.min() >= 0.0


@pytest.mark.parametrize("prec", [0, 1, 2, 5])
@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
@pytest.mark.parametrize("m", [1, 40])
def test_matvec_duplicate_points(nys, prec, kind, m):
    """Every point three times: off-diagonal pairs at distance zero, whose computed
    exponent is a rounding residue of either sign (the RBF epilogue does not clamp it)."""
    rng = np.random.default_rng(17 + m)
    X = np.repeat(rng.standard_normal((200, 16)) * 3.0, 3, axis=0)
    V = rng.standard_normal((600, m))
    if prec != 0:
        V = V.astype(np.float32).astype(np.float64)
    sigma = 4.0
    print(f"case duplicates prec={prec} kind={kind} m={m}", flush=True)
    got = run(nys, X, X, V, kind, sigma, prec)
    ref = o.kernel_matvec(X, X, V, kind, sigma)
    assert np.max(np.abs(got - ref) / bound(X, X, V, kind, sigma, prec)) <= 1.0


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_matvec_rectangular(nys, prec):
    check(nys, 333, 1201, 16, 1, o.RBF, prec, same=False, seed=3)
    check(nys, 1201, 333, 16, 40, o.LAPLACIAN, prec, same=False, seed=4)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
@pytest.mark.parametrize("m", [1, 3, 6])
def test_matvec_dsigma(nys, prec, kind, m):
    check(nys, 600, 600, 16, m, kind, prec, deriv=1, seed=11 + m)


def test_matvec_heavy_tailed_column(nys):
    for prec in (0, 1, 2):
        check(nys, 3000, 3000, 20, 1, o.RBF, prec, heavy=True, seed=5)


def test_matvec_alpha_beta(nys):
    rng = np.random.default_rng(9)
    X = rng.standard_normal((400, 8))
    V = rng.standard_normal((400, 2))
    Out = rng.standard_normal((400, 2))
    got = run(nys, X, X, V, o.RBF, 2.0, 0, 0, 0.5, -2.0, Out)
    ref = o.kernel_matvec(X, X, V, o.RBF, 2.0, 0, 0.5, -2.0, Out)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # flash path with beta
    V2 = rng.standard_normal((400, 40))
    O2 = rng.standard_normal((400, 40))
    got = run(nys, X, X, V2, o.RBF, 2.0, 0, 0, 1.5, 0.25, O2)
    ref = o.kernel_matvec(X, X, V2, o.RBF, 2.0, 0, 1.5, 0.25, O2)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_matvec_diagonal_exact_for_identical_points(nys):
    """Symmetric products take K_ii = 1 exactly: with sigma tiny, K = I and K V = V."""
    rng = np.random.default_rng(10)
    X = rng.standard_normal((300, 12)) * 10
    V = rng.standard_normal((300, 3))
    for prec in (0, 1, 2):
        Vp = V if prec == 0 else V.astype(np.float32).astype(np.float64)
        got = run(nys, X, X, Vp, o.LAPLACIAN, 1e-3, prec)
        assert np.array_equal(got, Vp) or np.max(np.abs(got - Vp)) <= 1e-6 * np.max(np.abs(Vp))


def test_matvec_deterministic(nys):
    rng = np.random.default_rng(12)
    X = rng.standard_normal((5000, 16))
    V = rng.standard_normal((5000, 64))
    for prec in (0, 2):
        a = run(nys, X, X, V, o.RBF, 4.0, prec)
        b = run(nys, X, X, V, o.RBF, 4.0, prec)
        assert np.array_equal(a, b)


def test_matvec_large_sampled_rows(nys):
    """Full-size check on sampled rows: n = 1e6 points, d = 16 (the batched workload's
    point set), one and 512 columns in BF16X3; rows sampled and recomputed by the
    oracle one by one."""
    w = ni.batched_lambda_grid(0, n=1_000_000, nrhs=2, nlam=1)
    X = w.X
    dev = torch.device("cuda")
    tX = torch.from_numpy(X).to(dev)
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(X.shape[0], 24, replace=False))
    for m, prec in ((1, 2), (512, 2), (512, 3), (512, 4), (64, 4), (512, 5), (40, 5)):
        V = rng.standard_normal((X.shape[0], m)).astype(np.float32)
        tV = torch.from_numpy(V).to(dev)
        print(f"case n=1e6 d=16 m={m} prec={prec}", flush=True)
        out = nys.kernel_matvec(tX, tX, tV, o.RBF, w.sigma, prec)
        torch.cuda.synchronize()
        got = out[torch.from_numpy(rows).to(dev)].double().cpu().numpy()
        ref = o.kernel_matvec_rows(X[rows], X, V.astype(np.float64), o.RBF, w.sigma)
        Kabs = o.kernel_matvec_rows(X[rows], X, np.abs(V).astype(np.float64), o.RBF, w.sigma)
        mu = X.mean(0)
        span = (np.linalg.norm(X[rows] - mu, axis=1).max() + np.linalg.norm(X - mu, axis=1).max()) ** 2
        kap = 1 / (2 * w.sigma ** 2)
        tol = (16 * 2.0 ** -16 * (1 + kap * span) + (X.shape[0] / 4 + 16) * 2.0 ** -24) * Kabs
        assert np.max(np.abs(got - ref) / tol) <= 1.0
        del out, tV


def test_six_term_distance_is_more_accurate(nys):
    """BF16X3_D6 splits the distance operands into three bf16 parts.  Products with
    unit vectors return single kernel entries (no accumulation error), so the
    entry error of the two splits can be compared directly: about 2^-16 relative
    for three terms, float32 level for six."""
    rng = np.random.default_rng(21)
    X = rng.standard_normal((3000, 16))
    J = rng.choice(3000, 16, replace=False)
    V = np.zeros((3000, 16))
    V[J, np.arange(16)] = 1.0
    ref = o.kernel_matrix(X, X, o.RBF, 4.0)[:, J]
    e3 = np.max(np.abs(run(nys, X, X, V, o.RBF, 4.0, 2) - ref) / ref)
    e6 = np.max(np.abs(run(nys, X, X, V, o.RBF, 4.0, 3) - ref) / ref)
    print(f"max relative entry error: 3-term {e3:.3e}, 6-term {e6:.3e}")
    assert e3 < 2.0 ** -11
    assert e6 < e3 / 16 and e6 < 2.0 ** -18


def test_fp16_product_is_more_accurate(nys):
    """F16X3_D10 splits K and the column-scaled V into fp16 parts for the second MFMA
    (11 + 11 significand bits) where BF16X3_D10 uses bf16 parts (8 + 8).  With unit
    vectors as columns (17 of them: the MFMA product path) every output is a single
    kernel entry, so the entry error of the two products is compared directly."""
    rng = np.random.default_rng(22)
    X = rng.standard_normal((3000, 16))
    J = rng.choice(3000, 17, replace=False)
    V = np.zeros((3000, 17))
    V[J, np.arange(17)] = 1.0
    ref = o.kernel_matrix(X, X, o.RBF, 4.0)[:, J]
    e_bf = np.max(np.abs(run(nys, X, X, V, o.RBF, 4.0, 4) - ref) / ref)
    e_h = np.max(np.abs(run(nys, X, X, V, o.RBF, 4.0, 5) - ref) / ref)
    print(f"max relative entry error: bf16 product {e_bf:.3e}, fp16 product {e_h:.3e}")
    assert e_bf < 2.0 ** -15
    assert e_h < e_bf / 8 and e_h < 2.0 ** -19


@pytest.mark.parametrize("prec,widths", [(0, (16, 32, 48, 64, 96, 128, 256)), (1, (32, 64, 128)), (2, (32, 64, 128, 256)),
                                         (5, (16, 32, 64, 128, 256))])
def test_every_chunk_width_matches_oracle(nys, prec, widths):
    """Every column-chunk width the autotuner may choose gives the same products (to
    the precision's bound): each is forced for all column counts in turn."""
    try:
        for tm in widths:
            nys.nys_set_tile(prec, 1, 1024, tm)
            print(f"width {tm}", flush=True)
            check(nys, 700, 700, 12, 40, o.RBF, prec, seed=tm)
            check(nys, 300, 900, 12, 70, o.LAPLACIAN, prec, same=False, seed=tm + 1)
    finally:
        nys.nys_clear_tiles()


def test_autotune_records_a_valid_width(nys):
    rng = np.random.default_rng(5)
    X = torch.from_numpy(rng.standard_normal((6000, 16))).to(torch.device("cuda"))
    try:
        tm, ms = nys.nys_autotune(X, o.RBF, 4.0, nys.F16X3_D10, 100, m_lo=65, reps=1)
        print(f"chosen width {tm}, {ms:.3f} ms")
        assert tm in (32, 64, 128, 256) and ms > 0   # widths with <= 4 chunks, <= 2 x 128
        # the recorded width is used for 65..100 columns: products still match the oracle
        Xn = X.cpu().numpy()
        V = rng.standard_normal((6000, 80)).astype(np.float32).astype(np.float64)
        got = run(nys, Xn, Xn, V, o.RBF, 4.0, 5)
        ref = o.kernel_matvec(Xn, Xn, V, o.RBF, 4.0)
        assert np.max(np.abs(got - ref) / bound(Xn, Xn, V, o.RBF, 4.0, 5, 0)) <= 1.0
        t0, _ = nys.nys_autotune(X, o.RBF, 4.0, nys.F16X3_D10, 1, reps=1)   # one column: fp16 tile too
        assert t0 in (16, 32)
        assert nys.nys_autotune(X, o.RBF, 4.0, nys.FP64, 3, reps=1)[0] == 0  # row-sum tile: nothing to tune
    finally:
        nys.nys_clear_tiles()
