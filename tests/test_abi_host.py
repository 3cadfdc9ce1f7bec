"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/nys.h declares, reports workspace sizes, and rejects invalid
arguments before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2609_08136_amd as nys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nys.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    return nys.load()


def test_header_declares_the_six_entry_points():
    names = declared_functions()
    for f in ("kernel_matvec", "nys_sketch", "nys_precond_build", "nys_precond_apply", "nyspcg_solve",
              "nyspcg_backward", "nys_workspace_bytes", "nys_last_error", "nys_version"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    for f in declared_functions():
        assert hasattr(lib, f), f
    assert set(nys.EXPORTS) <= set(declared_functions())
    assert nys.version().startswith("libnys")


def test_workspace_sizes(lib):
    small = nys.nys_workspace_bytes(nys.OP_KERNEL_MATVEC, 1000, 1000, 10, 0, 1, nys.FP64)
    big = nys.nys_workspace_bytes(nys.OP_KERNEL_MATVEC, 100000, 100000, 10, 0, 1, nys.FP64)
    assert 0 < small < big
    solve = nys.nys_workspace_bytes(nys.OP_SOLVE, 1_000_000, 0, 16, 500, 512, nys.BF16X3)
    # state vectors: at least 6 float32 n x m blocks
    assert solve >= 6 * 1_000_000 * 512 * 4
    for op in range(6):
        assert nys.nys_workspace_bytes(op, 2000, 2000, 10, 50, 4, nys.FP32) > 0


def test_workspace_query_rejects_bad_arguments(lib):
    b = ctypes.c_size_t(0)
    assert lib.nys_workspace_bytes(99, 10, 10, 2, 2, 2, 0, ctypes.byref(b)) == nys.EINVAL
    assert lib.nys_workspace_bytes(0, -1, 10, 2, 2, 2, 0, ctypes.byref(b)) == nys.EINVAL
    assert lib.nys_workspace_bytes(0, 10, 10, 2, 2, 2, 7, ctypes.byref(b)) == nys.EINVAL
    assert lib.nys_workspace_bytes(0, 10, 10, 2, 2, 2, 0, None) == nys.EINVAL


FAKE = ctypes.c_void_p(4096)   # never dereferenced: validation fails first


def test_kernel_matvec_argument_errors(lib):
    k = nys.NysKernel(nys.RBF, 0, 1.0)
    bad_sigma = nys.NysKernel(nys.RBF, 0, 0.0)
    bad_kind = nys.NysKernel(5, 0, 1.0)
    args = lambda kern, prec=0, d=3, deriv=0: lib.kernel_matvec(kern, deriv, prec, FAKE, 10, FAKE, 10, d, FAKE, 1,
                                                                  FAKE, 1.0, 0.0, FAKE, 0, None)
    assert args(bad_sigma) == nys.EINVAL
    assert b"sigma" in lib.nys_last_error()
    assert args(bad_kind) == nys.EINVAL
    assert b"kind" in lib.nys_last_error()
    assert args(k, prec=9) == nys.EINVAL
    assert args(k, d=0) == nys.EINVAL
    assert args(k, d=63, prec=nys.FP32) == nys.EINVAL
    assert args(k, d=42, prec=nys.BF16X3_D6) == nys.EINVAL
    assert args(k, d=25, prec=nys.BF16X3_D10) == nys.EINVAL
    assert args(k, d=25, prec=nys.F16X3_D10) == nys.EINVAL
    assert args(k, d=42, prec=nys.F16X3_D6) == nys.EINVAL
    assert args(k, deriv=2) == nys.EINVAL
    assert b"deriv" in lib.nys_last_error()
    # null workspace
    assert lib.kernel_matvec(k, 0, 0, FAKE, 10, FAKE, 10, 3, FAKE, 1, FAKE, 1.0, 0.0, None, 0, None) == nys.EINVAL


def test_solve_argument_errors(lib):
    k = nys.NysKernel(nys.RBF, 0, 1.0)
    info = (nys.NysColInfo * 4)()
    def solve(lams, tol=1e-6, prec=0, mode=0, nrhs=1, max_iters=10, join=0.0):
        arr = (ctypes.c_double * len(lams))(*lams)
        o = nys.NysPCGOpts(tol, max_iters, prec, -1, mode, 0, 0, 0.0, join)
        return lib.nyspcg_solve(k, FAKE, 10, 2, FAKE, nrhs, arr, len(lams), None, ctypes.byref(o), FAKE, info,
                                FAKE, 1 << 30, None)
    assert solve([0.0]) == nys.EINVAL          # lambda must be > 0 (eq. rlaopt-regularized-linear-system)
    assert solve([-1.0]) == nys.EINVAL
    assert solve([float("nan")]) == nys.EINVAL
    assert solve([1.0], tol=0.0) == nys.EINVAL
    assert solve([1.0], prec=7) == nys.EINVAL
    assert solve([1.0], mode=3) == nys.EINVAL
    assert solve([1.0], join=0.5) == nys.EINVAL     # a join window below the due point
    assert solve([1.0], join=float("inf")) == nys.EINVAL
    assert solve([1.0], max_iters=-1) == nys.EINVAL
    assert solve([1.0], nrhs=0) == nys.EINVAL
    assert b"lambda" in lib.nys_last_error() or b"nrhs" in lib.nys_last_error()


def test_sketch_and_build_argument_errors(lib):
    k = nys.NysKernel(nys.RBF, 0, 1.0)
    assert lib.nys_sketch(k, 0, FAKE, 10, 2, FAKE, 0, 11, FAKE, FAKE, FAKE, 0, None) == nys.EINVAL   # r > n
    assert lib.nys_sketch(k, 0, FAKE, 10, 2, FAKE, 0, 0, FAKE, FAKE, FAKE, 0, None) == nys.EINVAL    # r < 1
    # Q overlapping Omega
    assert lib.nys_sketch(k, 0, FAKE, 10, 2, FAKE, 0, 3, ctypes.c_void_p(4096 + 8), FAKE, FAKE, 1 << 20,
                          None) == nys.EINVAL
    assert lib.nys_test_matrix(0, 0, 3, FAKE, None) == nys.EINVAL
    assert lib.nys_test_matrix(0, 3, 3, None, None) == nys.EINVAL
    P = nys.NysPrecondC(10, 3, 0, None, None, None, 0.0)
    assert lib.nys_precond_build(FAKE, FAKE, 10, 3, 0, ctypes.byref(P), FAKE, 0, None) == nys.EINVAL
    P2 = nys.NysPrecondC(10, 4, 0, FAKE, None, FAKE, 0.0)
    assert lib.nys_precond_build(FAKE, FAKE, 10, 3, 0, ctypes.byref(P2), FAKE, 0, None) == nys.EINVAL


def test_precond_apply_argument_errors(lib):
    P = nys.NysPrecondC(10, 3, 3, FAKE, None, FAKE, 0.0)
    other = ctypes.c_void_p(8192)
    # R and Z aliasing, no columns, missing lambdas, unknown precision: rejected before any device work
    assert lib.nys_precond_apply(ctypes.byref(P), FAKE, nys.FP64, FAKE, 1, FAKE, FAKE, 1 << 20, None) == nys.EINVAL
    assert lib.nys_precond_apply(ctypes.byref(P), FAKE, nys.FP32, FAKE, 0, other, FAKE, 1 << 20, None) == nys.EINVAL
    assert lib.nys_precond_apply(ctypes.byref(P), None, nys.FP32, FAKE, 1, other, FAKE, 1 << 20, None) == nys.EINVAL
    assert lib.nys_precond_apply(ctypes.byref(P), FAKE, 7, FAKE, 1, other, FAKE, 1 << 20, None) == nys.EINVAL
    bad = nys.NysPrecondC(10, 0, 0, FAKE, None, FAKE, 0.0)
    assert lib.nys_precond_apply(ctypes.byref(bad), FAKE, nys.FP64, FAKE, 1, other, FAKE, 1 << 20, None) == nys.EINVAL


def test_build_generates_the_dispatch_sources(tmp_path):
    """The tile instantiations and their dispatch are generated at build time: the
    generator writes one source per precision family, each defining its dispatch
    function, none of them is kept under csrc/, and the build compiles them beside the
    hand-written sources."""
    from paper_2609_08136_amd import build
    gen = build.gen_dispatch
    paths = gen.write_all(str(tmp_path))
    assert [os.path.basename(p) for p in paths] == gen.GENERATED
    for p in paths:
        name = os.path.splitext(os.path.basename(p))[0].replace("kmv_", "")
        text = open(p).read()
        assert f"int32_t kmv_dispatch_{name}(" in text and "hipLaunchKernelGGL" in text
    csrc = os.path.join(ROOT, "paper_2609_08136_amd", "csrc")
    assert not any(os.path.exists(os.path.join(csrc, f)) for f in gen.GENERATED)
    assert not any(os.path.basename(s) in gen.GENERATED for s in build.SOURCES)
    assert {os.path.basename(s) for s in build.SOURCES} >= {"api.hip", "kmv_host.hip", "pcg.hip"}


def test_tile_sources_avoid_packed_fp32_ops():
    """Packed FP32 VALU instructions are disabled in the build flags and never
    written by hand."""
    from paper_2609_08136_amd import build
    assert "-packed-fp32-ops" in build.CFLAGS
    csrc = os.path.join(ROOT, "paper_2609_08136_amd", "csrc")
    for f in os.listdir(csrc):
        if not f.endswith((".hip", ".h", ".py")):
            continue
        txt = open(os.path.join(csrc, f)).read()
        assert "v_pk_fma_f32" not in txt and "v_pk_mul_f32" not in txt and "v_pk_add_f32" not in txt


def test_autotune_argument_errors(lib):
    k = nys.NysKernel(nys.RBF, 0, 1.0)
    best = nys.NysTileChoice()
    tune = lambda **kw: lib.nys_autotune(k, kw.get("prec", 0), kw.get("X", FAKE), kw.get("n", 100),
                                         kw.get("n_rows", 100), kw.get("d", 3), kw.get("m", 8), kw.get("m_lo", 1),
                                         kw.get("reps", 1), ctypes.byref(best), kw.get("ws", FAKE), 1 << 20, None)
    assert tune(prec=9) == nys.EINVAL
    assert tune(n_rows=200) == nys.EINVAL          # more rows than points
    assert tune(m_lo=9) == nys.EINVAL              # m_lo > m
    assert tune(reps=0) == nys.EINVAL
    assert tune(X=None) == nys.EINVAL
    assert tune(ws=None) == nys.EINVAL
    assert lib.nys_set_tile(nys.FP64, 1, 64, 512) == nys.EINVAL      # no 512-wide float64 tile
    assert lib.nys_set_tile(nys.F16X3_D10, 5, 4, 64) == nys.EINVAL   # empty range
    assert lib.nys_set_tile(7, 1, 4, 64) == nys.EINVAL
    assert lib.nys_set_tile(nys.F16X3_D10, 1, 64, 16) == nys.OK
    assert lib.nys_set_tile(nys.F16X3_D10, 1, 64, 0) == nys.OK       # removes it again
    lib.nys_clear_tiles()
    b = ctypes.c_size_t(0)
    assert lib.nys_workspace_bytes(6, 1000, 4000, 16, 0, 64, nys.F16X3_D10, ctypes.byref(b)) == nys.OK
    assert b.value >= (4000 + 1000) * 64 * 4


def test_library_id_is_the_content_hash_of_the_loaded_build(lib):
    import hashlib
    with open(nys.LIB_PATH, "rb") as f:
        want = hashlib.sha256(f.read()).hexdigest()[:16]
    assert nys.library_id() == want
    assert re.fullmatch(r"[0-9a-f]{16}", nys.library_id())


def test_plan_chunks_last_chunk_and_float64_costs(lib):
    """The chunk plan (host logic only): the last chunk runs at the narrowest width that
    holds the remaining columns, and the float64 planner minimises the measured chunk
    cost (widths 16..256 including 48 and 96)."""
    nys.nys_clear_tiles()
    n, d = 1_000_000, 16
    # fp16 product: 256-column chunks, the remainder in the narrowest chunk that holds it
    assert nys.nys_plan_chunks(nys.F16X3_D10, n, d, 512) == (256, 0)
    assert nys.nys_plan_chunks(nys.F16X3_D10, n, d, 320) == (256, 64)
    assert nys.nys_plan_chunks(nys.F16X3_D10, n, d, 270) == (256, 16)
    assert nys.nys_plan_chunks(nys.F16X3_D10, n, d, 1) == (16, 0)      # fp16 tile at every width
    for m, want in ((512, (256, 0)), (320, (256, 64)), (270, (256, 16)), (1, (16, 0))):
        assert nys.nys_plan_chunks(nys.F16X3_D6, n, d, m) == want        # the same tiles
    # float32: 128-column chunks, tail from its widths (32, 64, 128)
    assert nys.nys_plan_chunks(nys.FP32, n, d, 300) == (128, 64)
    assert nys.nys_plan_chunks(nys.FP32, n, d, 260) == (128, 32)
    # bf16 splits: no 16-column tile
    assert nys.nys_plan_chunks(nys.BF16X3, n, d, 270) == (256, 32)
    # float64: row-sum tile up to 4 columns, then the cheapest chunking
    assert nys.nys_plan_chunks(nys.FP64, n, d, 4) == (0, 0)
    assert nys.nys_plan_chunks(nys.FP64, n, d, 40) == (48, 0)
    assert nys.nys_plan_chunks(nys.FP64, n, d, 80) == (96, 0)
    assert nys.nys_plan_chunks(nys.FP64, n, d, 144) == (128, 16)
    assert nys.nys_plan_chunks(nys.FP64, n, d, 200) == (256, 0)
    assert nys.nys_plan_chunks(nys.FP64, n, d, 384) == (256, 128)
    assert nys.nys_plan_chunks(nys.FP64, n, d, 512) == (256, 0)
    # every plan's widths are tiles of that precision, and the chunks cover m
    for prec in (nys.FP64, nys.FP32, nys.BF16X3, nys.F16X3_D10, nys.F16X3_D6):
        for m in range(1, 600, 7):
            tm, tail = nys.nys_plan_chunks(prec, n, d, m)
            if tm == 0:
                assert prec == nys.FP64 and m <= 4 or prec != nys.FP64 and m <= 16
                continue
            full = -(-m // tm) - 1
            assert tail == 0 or (tail < tm and m - full * tm <= tail)
            assert full * tm + (tail or tm) >= m


def test_plan_ranges_bound_the_float32_accumulation(lib):
    """The low-precision products sum at most 16384 column points per float32
    accumulator where the range sums (n x m x 4 bytes per range) fit in 32 GiB, and
    fewer, longer ranges where they would not; the float64 products split only to fill
    the GPU (host logic only)."""
    n, d, cap = 1_000_000, 16, 32 << 30
    # the headline's product at n = 1e6: 16 ranges at 512 columns (capped), 62 below
    assert nys.nys_plan_ranges(nys.F16X3_D6, n, d, 512) == (16, 62528)
    assert nys.nys_plan_ranges(nys.F16X3_D6, n, d, 128) == (62, 16160)
    assert nys.nys_plan_ranges(nys.F16X3_D6, n, d, 1) == (62, 16160)
    assert nys.nys_plan_ranges(nys.FP64, n, d, 512)[0] == 1
    for prec in (nys.F16X3_D6, nys.F16X3_D10, nys.BF16X3, nys.BF16X3_D6, nys.FP32):
        for nn in (1000, 20_000, 200_000, n):
            for m in (1, 16, 64, 128, 256, 512, 2048):
                ranges, points = nys.nys_plan_ranges(prec, nn, d, m)
                assert ranges >= 1 and ranges * points >= nn and (ranges - 1) * points < nn
                wanted = -(-nn // 16384)
                if wanted * nn * m * 4 <= cap:
                    assert points <= 16384, (prec, nn, m, ranges, points)
                else:
                    assert ranges * nn * m * 4 <= cap
    rng, pts = ctypes.c_int32(), ctypes.c_int64()
    assert lib.nys_plan_ranges(9, n, d, 8, ctypes.byref(rng), ctypes.byref(pts)) == nys.EINVAL
    assert lib.nys_plan_ranges(nys.F16X3_D6, n, 42, 8, ctypes.byref(rng), ctypes.byref(pts)) == nys.EINVAL
    assert lib.nys_plan_ranges(nys.F16X3_D6, n, d, 8, None, ctypes.byref(pts)) == nys.EINVAL


def test_plan_chunks_follow_tuned_widths_and_reject_bad_arguments(lib):
    try:
        nys.nys_set_tile(nys.F16X3_D10, 257, 512, 128)
        assert nys.nys_plan_chunks(nys.F16X3_D10, 10**6, 16, 300) == (128, 64)
        assert nys.nys_plan_chunks(nys.F16X3_D6, 10**6, 16, 300) == (256, 64)    # a table of its own
        nys.nys_set_tile(nys.F16X3_D6, 257, 512, 128)
        assert nys.nys_plan_chunks(nys.F16X3_D6, 10**6, 16, 300) == (128, 64)
        # the bf16-split precisions share one table: a width tuned for BF16X3_D6 applies
        # to its own plans (and to BF16X3's and BF16X3_D10's)
        nys.nys_set_tile(nys.BF16X3_D6, 257, 512, 128)
        for prec in (nys.BF16X3_D6, nys.BF16X3, nys.BF16X3_D10):
            assert nys.nys_plan_chunks(prec, 10**6, 16, 300) == (128, 64)
    finally:
        nys.nys_clear_tiles()
    tm, tail = ctypes.c_int32(), ctypes.c_int32()
    assert lib.nys_plan_chunks(9, 1000, 16, 10, ctypes.byref(tm), ctypes.byref(tail)) == nys.EINVAL
    assert lib.nys_plan_chunks(nys.FP64, 0, 16, 10, ctypes.byref(tm), ctypes.byref(tail)) == nys.EINVAL
    assert lib.nys_plan_chunks(nys.FP64, 1000, 16, 0, ctypes.byref(tm), ctypes.byref(tail)) == nys.EINVAL
    assert lib.nys_plan_chunks(nys.F16X3_D10, 1000, 25, 10, ctypes.byref(tm), ctypes.byref(tail)) == nys.EINVAL
    assert lib.nys_plan_chunks(nys.FP64, 1000, 16, 10, None, ctypes.byref(tail)) == nys.EINVAL


def test_kernel_dot_argument_errors(lib):
    k = nys.NysKernel(nys.RBF, 0, 1.0)
    out = ctypes.c_double(0.0)
    call = lambda kern=k, deriv=0, nr=10, d=3, u=FAKE: lib.kernel_dot(kern, deriv, FAKE, nr, FAKE, 10, d, u, FAKE,
                                                                    ctypes.byref(out), FAKE, 1 << 20, None)
    assert call(kern=nys.NysKernel(nys.RBF, 0, -1.0)) == nys.EINVAL
    assert call(deriv=3) == nys.EINVAL
    assert call(nr=0) == nys.EINVAL
    assert call(d=63) == nys.EINVAL
    assert call(u=None) == nys.EINVAL
    assert lib.kernel_dot(k, 0, FAKE, 10, FAKE, 10, 3, FAKE, FAKE, ctypes.byref(out), FAKE, 0, None) == nys.ENOMEM
    assert nys.nys_workspace_bytes(nys.OP_KERNEL_DOT, 1000, 2000, 16) > 0


def test_admm_argument_errors(lib):
    """nys_admm_elastic_net rejects bad sizes, penalties, bounds and configuration
    fields before touching the device."""
    cfg = nys.NysAdmmConfig()
    info = nys.NysAdmmInfo()
    def call(n=10, p=4, lam1=0.1, lam2=0.1, lo=0.0, hi=1.0, c=None, W=FAKE):
        return lib.nys_admm_elastic_net(FAKE, n, p, FAKE, lam1, lam2, lo, hi, ctypes.byref(c or cfg), W,
                                        ctypes.byref(info), FAKE, 1 << 30, None)
    assert call(n=0) == nys.EINVAL
    assert call(W=None) == nys.EINVAL
    assert call(lam1=-1.0) == nys.EINVAL
    assert call(lam2=float("nan")) == nys.EINVAL
    assert call(lo=1.0, hi=0.0) == nys.EINVAL
    for field, bad in (("alpha", 2.0), ("alpha", -0.5), ("gamma", 1.0), ("rho", -1.0), ("rank", 5),
                       ("rho_update_factor", 0.5), ("sigma", -1e-3), ("max_iters", -1)):
        c = nys.NysAdmmConfig()
        setattr(c, field, bad)
        assert call(c=c) == nys.EINVAL, field
