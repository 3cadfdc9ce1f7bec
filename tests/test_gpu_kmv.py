"""GPU parity of kernel_matvec against the CPU float64 oracle, element by element.

Every case runs twice, with random-sign V and with V >= 0 (where |K| |V| = |K V|, so
the bound is relative to the result itself).  The bounds (tests/kmv_bounds.py) are
derived from the arithmetic of each precision, pair by pair, and each case also
asserts that its largest tolerance is below a tenth of its largest |reference|
(an all-zero output, or a product that drops a split part, fails).
"""
import math

import numpy as np
import pytest
import torch

import kmv_bounds as kb
import nys_inputs as ni
import oracle as o

pytestmark = pytest.mark.gpu

GUARD = 0.1


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
    A, K = kb.entry_abs_bound(Xr, Xc, kind, sigma, prec, m, deriv, same=Xc is Xr)
    for name, VV in (("random-sign", V), ("nonnegative", np.abs(V))):
        print(f"case n_r={n_r} n_c={Xc.shape[0]} d={d} m={m} kind={kind} prec={prec} deriv={deriv} V {name}",
              flush=True)
        got = run(nys, Xr, Xc, VV, kind, sigma, prec, deriv)
        ref = K @ VV
        tol = kb.product_bound(Xr, Xc, VV, kind, sigma, prec, deriv, same=Xc is Xr)
        err = np.abs(got - ref)
        worst = float(np.max(err / tol))
        g = kb.guard(tol, ref)
        print(f"  max err/bound {worst:.3g}, bound guard {g:.3g}", flush=True)
        assert g < GUARD, f"bound too loose to fail: max tol / max |ref| = {g:.3g}"
        assert worst <= 1.0, f"max err/bound = {worst:.3g} (max abs err {err.max():.3g})"
    return got, ref


@pytest.mark.parametrize("prec", [0, 1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
@pytest.mark.parametrize("n,d,m", [(1, 3, 1), (31, 10, 1), (257, 16, 3), (2000, 10, 1), (700, 20, 8),
                                   (513, 33, 16), (300, 1, 5)])
def test_matvec_small_m(nys, prec, kind, n, d, m):
    check(nys, n, n, d, m, kind, prec, seed=n + d + m)


@pytest.mark.parametrize("prec", [0, 1, 2, 3, 4, 5, 6])
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


@pytest.mark.parametrize("prec", [0, 1, 2, 5, 6])
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
    for VV in (V, np.abs(V)):
        got = run(nys, X, X, VV, kind, sigma, prec)
        ref = o.kernel_matvec(X, X, VV, kind, sigma)
        tol = kb.product_bound(X, X, VV, kind, sigma, prec, same=True)
        assert kb.guard(tol, ref) < GUARD
        assert np.max(np.abs(got - ref) / tol) <= 1.0


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


def _sampled_bound(X, rows, V, sigma, prec):
    """Bound and reference for sampled rows of an n x n product (row blocks of the
    per-pair entry bound against all n points)."""
    A, K = kb.entry_abs_bound(X[rows], X, o.RBF, sigma, prec, V.shape[1], 0)
    for t, i in enumerate(rows):
        A[t, i] = 0.0                                    # K_ii = 1 exactly (symmetric product)
        K[t, i] = 1.0
    return K @ V, kb.bound_from(A, K, V, prec, V.shape[1], 0)


def test_matvec_large_sampled_rows(nys):
    """Full-size check on sampled rows: n = 1e6 points, d = 16 (the batched workload's
    point set), 1 ... 512 columns, random-sign and non-negative V; 24 rows sampled and
    recomputed by the oracle one by one against all 1e6 points."""
    w = ni.batched_lambda_grid(0, n=1_000_000, nrhs=2, nlam=1)
    X = w.X
    dev = torch.device("cuda")
    tX = torch.from_numpy(X).to(dev)
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(X.shape[0], 24, replace=False))
    trows = torch.from_numpy(rows).to(dev)
    Vs = {}
    for m, prec in ((1, 2), (512, 2), (256, 3), (128, 4), (64, 4), (512, 5), (40, 5), (1, 5), (512, 6), (64, 6),
                    (1, 6), (1, 0), (64, 0)):
        if m not in Vs:
            Vs[m] = rng.standard_normal((X.shape[0], m)).astype(np.float32).astype(np.float64)
        V = Vs[m]
        for name, VV in (("random-sign", V), ("nonnegative", np.abs(V))):
            dt = torch.float64 if prec == 0 else torch.float32
            tV = torch.from_numpy(VV).to(dev, dt)
            print(f"case n=1e6 d=16 m={m} prec={prec} V {name}", flush=True)
            out = nys.kernel_matvec(tX, tX, tV, o.RBF, w.sigma, prec)
            torch.cuda.synchronize()
            got = out[trows].double().cpu().numpy()
            ref, tol = _sampled_bound(X, rows, VV, w.sigma, prec)
            worst = float(np.max(np.abs(got - ref) / tol))
            g = kb.guard(tol, ref)
            print(f"  max err/bound {worst:.3g}, bound guard {g:.3g}", flush=True)
            assert g < GUARD
            assert worst <= 1.0
            del out, tV


@pytest.mark.parametrize("prec,widths", [(5, (16, 32, 64, 128, 256)), (6, (16, 64, 256)), (2, (32, 256)),
                                         (0, (16, 128, 256))])
def test_unit_vector_entries_every_width_n1e6(nys, prec, widths):
    """Single kernel entries of the full-size point set (n = 1e6, d = 16, sigma = 4)
    through every column-chunk width: V holds unit vectors e_j, so each output is one
    entry K_ij, held to the per-pair entry bound (no accumulation error).  The
    headline tile (fp16 product, 256-column chunk) is among them."""
    w = ni.batched_lambda_grid(0, n=1_000_000, nrhs=2, nlam=1)
    X = w.X
    n = X.shape[0]
    dev = torch.device("cuda")
    tX = torch.from_numpy(X).to(dev)
    rng = np.random.default_rng(31)
    rows = np.sort(rng.choice(n, 32, replace=False))
    trows = torch.from_numpy(rows).to(dev)
    dt = torch.float64 if prec == 0 else torch.float32
    try:
        for tm in widths:
            nys.nys_set_tile(prec, 1, 1024, tm)
            m = tm
            J = rng.choice(n, m, replace=False)
            J[:4] = rows[:4]                                # some diagonal entries too
            tV = torch.zeros((n, m), dtype=dt, device=dev)
            tV[torch.from_numpy(J).to(dev), torch.arange(m, device=dev)] = 1.0
            print(f"case unit vectors n=1e6 prec={prec} width={tm}", flush=True)
            out = nys.kernel_matvec(tX, tX, tV, o.RBF, w.sigma, prec)
            torch.cuda.synchronize()
            got = out[trows].double().cpu().numpy()
            A, K = kb.entry_abs_bound(X[rows], X[J], o.RBF, w.sigma, prec, m, 0, mu=X.mean(0))
            diag = rows[:, None] == J[None, :]
            K[diag] = 1.0
            A[diag] = 0.0
            err = np.abs(got - K)
            worst = float(np.max(err / (A + 1e-300)))
            print(f"  max err/bound {worst:.3g}, max relative entry error {np.max(err / K):.3g}", flush=True)
            assert worst <= 1.0
            assert np.all(got[diag] == 1.0) or prec != 0
            del out, tV
    finally:
        nys.nys_clear_tiles()


_ORACLE_CACHE = {}


@pytest.mark.parametrize("prec", [6, 5, 4, 1])
def test_row_sums_accumulated_in_bounded_ranges_n1e6(nys, prec):
    """Row sums K 1 of the full-size point set (n = 1e6, d = 16, sigma = 4) on 64
    sampled rows against the oracle.  Every term is positive, so a float32 accumulator
    grows with the sum and so does its rounding error: a sequential float32 sum of N
    similar positive terms, each rounding uniform within u = 2^-24 of the partial sum,
    has a relative RMS error of u sqrt(N) / 3, 3.5e-6 for N = 31250 column tiles of 32
    points.  The low-precision products sum ranges of at most 16384 points in float32
    and add the ranges in float64: u sqrt(512) / 3 / sqrt(62) = 6e-8 here, plus the
    output rounding (2^-24) and the unbiased entry errors, which average out over 1e6
    terms.  The bound, 5e-7 RMS and 2e-6 at worst, fails for one float32 range over
    all points (measured 5.2e-6 RMS, 2.7e-5 at worst)."""
    w = ni.batched_lambda_grid(0, n=1_000_000, nrhs=2, nlam=1)
    X = w.X
    n = X.shape[0]
    dev = torch.device("cuda")
    tX = torch.from_numpy(X).to(dev)
    rows = np.sort(np.random.default_rng(41).choice(n, 64, replace=False))
    if "rowsum" not in _ORACLE_CACHE:        # the same 64 oracle rows serve every precision
        _ORACLE_CACHE["rowsum"] = o.kernel_matvec_rows(X[rows], X, np.ones(n), o.RBF, w.sigma)
    ref = _ORACLE_CACHE["rowsum"]
    print(f"case row sums n=1e6 prec={prec}", flush=True)
    out = nys.kernel_matvec(tX, tX, torch.ones(n, dtype=torch.float32, device=dev), o.RBF, w.sigma, prec)
    torch.cuda.synchronize()
    got = out[torch.from_numpy(rows).to(dev)].double().cpu().numpy()
    rel = (got - ref) / ref
    rms = float(np.sqrt(np.mean(rel ** 2)))
    print(f"  relative error RMS {rms:.3g}, max {np.max(np.abs(rel)):.3g}", flush=True)
    assert rms <= 5e-7
    assert np.max(np.abs(rel)) <= 2e-6


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
                                         (5, (16, 32, 64, 128, 256)), (6, (16, 32, 64, 128, 256))])
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
        tol = kb.product_bound(Xn, Xn, V, o.RBF, 4.0, 5, 0, same=True)
        assert kb.guard(tol, ref) < GUARD
        assert np.max(np.abs(got - ref) / tol) <= 1.0
        t0, _ = nys.nys_autotune(X, o.RBF, 4.0, nys.F16X3_D10, 1, reps=1)   # one column: fp16 tile too
        assert t0 in (16, 32)
        assert nys.nys_autotune(X, o.RBF, 4.0, nys.FP64, 3, reps=1)[0] == 0  # row-sum tile: nothing to tune
    finally:
        nys.nys_clear_tiles()


def test_fp64_cost_table_autotune(nys):
    """The float64 cost-table tuning measures every width and replaces the planner's
    table: the plans it then makes are valid widths, float64 products at in-between
    widths still match the oracle, and clearing the tiles restores the default plans."""
    rng = np.random.default_rng(6)
    X = torch.from_numpy(rng.standard_normal((5000, 20))).to(torch.device("cuda"))
    before = {m: nys.nys_plan_chunks(nys.FP64, 5000, 20, m) for m in (40, 96, 200, 300)}
    try:
        res = nys.autotune_fp64_costs(X, o.RBF, 4.5, n_rows=2048)
        print("float64 cost tuning:", res)
        assert res["tm_at_256"] in (16, 32, 48, 64, 96, 128, 256) and res["ms_at_256"] > 0
        Xn = X.cpu().numpy()
        for m in (40, 96, 200, 300):
            tm, tail = nys.nys_plan_chunks(nys.FP64, 5000, 20, m)
            assert tm in (16, 32, 48, 64, 96, 128, 256) and (tail == 0 or tail < tm)
        V = rng.standard_normal((5000, 200))
        got = run(nys, Xn, Xn, V, o.RBF, 4.5, 0)
        ref = o.kernel_matvec(Xn, Xn, V, o.RBF, 4.5)
        tol = kb.product_bound(Xn, Xn, V, o.RBF, 4.5, 0, same=True)
        assert kb.guard(tol, ref) < GUARD
        assert np.max(np.abs(got - ref) / tol) <= 1.0
    finally:
        nys.nys_clear_tiles()
    assert {m: nys.nys_plan_chunks(nys.FP64, 5000, 20, m) for m in (40, 96, 200, 300)} == before


@pytest.mark.parametrize("prec", [0, 1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("kind", [o.RBF, o.LAPLACIAN])
@pytest.mark.parametrize("where", ["rows", "cols", "inf"])
def test_non_finite_points_are_rejected(nys, prec, kind, where):
    """A NaN or Inf coordinate in either point set returns NYS_ENUMERIC instead of a
    silently wrong product (a NaN column point would turn the centre, and with it every
    packed point, into NaN)."""
    rng = np.random.default_rng(40)
    Xr = rng.standard_normal((300, 8))
    Xc = rng.standard_normal((500, 8))
    if where == "rows":
        Xr[17, 3] = np.nan
    elif where == "cols":
        Xc[250, 0] = np.nan
    else:
        Xc[3, 7] = np.inf
    V = rng.standard_normal((500, 20))
    print(f"case non-finite prec={prec} kind={kind} where={where}", flush=True)
    with pytest.raises(nys.NysError) as ei:
        run(nys, Xr, Xc, V, kind, 2.0, prec)
    assert ei.value.code == nys.ENUMERIC
    # a finite input on the same buffers still works afterwards
    got = run(nys, np.nan_to_num(Xr, posinf=0.0), np.nan_to_num(Xc, posinf=0.0), V, kind, 2.0, prec)
    assert np.all(np.isfinite(got))
