"""The allocation-free kernel product (kernel_matvec_noalloc, declared in include/nys_noalloc.h)
against the allocating entry point, through the C ABI: two calls in a row, the second
with a smaller input, must give exactly the allocating call's result (same plan, same
kernels); a product too large for the fixed scratch is refused before device work."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2609_08136_amd as nys

pytestmark = pytest.mark.gpu


def _lib():
    lib = nys.load()
    f = lib.kernel_matvec_noalloc
    f.argtypes = [nys.NysKernel, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                  ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double,
                  ctypes.c_double, ctypes.c_void_p]
    f.restype = ctypes.c_int32
    lib.nys_noalloc_scratch_bytes.argtypes = []
    lib.nys_noalloc_scratch_bytes.restype = ctypes.c_size_t
    return lib


def _noalloc(lib, Xr, Xc, V, kind, sigma, prec, alpha=1.0, beta=0.0, out=None):
    nr, d = Xr.shape
    m = V.shape[1]
    O = torch.zeros((nr, m), dtype=V.dtype, device=V.device) if out is None else out.clone()
    rc = lib.kernel_matvec_noalloc(nys.NysKernel(kind, 0, float(sigma)), 0, int(prec), Xr.data_ptr(), nr,
                                   Xc.data_ptr(), Xc.shape[0], d, V.data_ptr(), m, O.data_ptr(), float(alpha),
                                   float(beta), torch.cuda.current_stream().cuda_stream)
    assert rc == nys.OK, lib.nys_last_error()
    torch.cuda.synchronize()
    return O


@pytest.mark.parametrize("prec", [nys.FP64, nys.FP32, nys.F16X3_D10, nys.BF16X3])
def test_noalloc_matches_kernel_matvec_twice(prec):
    lib = _lib()
    dev = torch.device("cuda")
    rng = np.random.default_rng(77)
    dt = torch.float64 if prec == nys.FP64 else torch.float32
    cases = [(3000, 2500, 16, 300, nys.RBF, 4.0), (700, 700, 9, 7, nys.LAPLACIAN, 2.5)]   # second: smaller
    for nr, nc, d, m, kind, sigma in cases:
        Xr = torch.from_numpy(rng.standard_normal((nr, d))).to(dev)
        Xc = Xr if nr == nc else torch.from_numpy(rng.standard_normal((nc, d))).to(dev)
        V = torch.from_numpy(rng.standard_normal((nc, m))).to(dev, dt)
        O0 = torch.from_numpy(rng.standard_normal((nr, m))).to(dev, dt)
        print(f"case noalloc prec={prec} nr={nr} nc={nc} d={d} m={m} kind={kind}", flush=True)
        got = _noalloc(lib, Xr, Xc, V, kind, sigma, prec, 0.75, -0.5, O0)
        ref = nys.kernel_matvec(Xr, Xc, V, kind, sigma, prec, 0, 0.75, -0.5, O0.clone())
        torch.cuda.synchronize()
        assert torch.equal(got, ref)


def test_noalloc_refuses_products_beyond_its_scratch():
    lib = _lib()
    cap = lib.nys_noalloc_scratch_bytes()
    assert cap == 256 << 20
    fake = ctypes.c_void_p(4096)        # never dereferenced: the size check comes first
    n = 4_000_000
    assert nys.nys_workspace_bytes(nys.OP_KERNEL_MATVEC, n, n, 16, 0, 512, nys.F16X3_D10) > cap
    rc = lib.kernel_matvec_noalloc(nys.NysKernel(nys.RBF, 0, 4.0), 0, nys.F16X3_D10, fake, n, fake, n, 16, fake, 512,
                                   fake, 1.0, 0.0, None)
    assert rc == nys.ENOMEM
    assert b"scratch" in lib.nys_last_error()
