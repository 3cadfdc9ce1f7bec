"""Python binding of libnys: Nystrom-preconditioned CG for kernel systems
(K + lambda I) x = b on an AMD Instinct MI355X.

The functions below carry the names of the C ABI (include/nys.h) and only
marshal arguments: every step runs in the HIP kernels of libnys.so.  PyTorch
supplies device memory (tensors, workspaces) and the current HIP stream.
There is no CPU fallback: if libnys.so is missing, load() raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnys.so")

RBF, LAPLACIAN = 0, 1
FP64, FP32, BF16X3, BF16X3_D6, BF16X3_D10, F16X3_D10, F16X3_D6 = 0, 1, 2, 3, 4, 5, 6
PREC_NAMES = {FP64: "fp64", FP32: "fp32", BF16X3: "bf16x3", BF16X3_D6: "bf16x3_d6", BF16X3_D10: "bf16x3_d10",
              F16X3_D10: "f16x3_d10", F16X3_D6: "f16x3_d6"}
PREC_BY_NAME = {v: k for k, v in PREC_NAMES.items()}

OK, NOT_CONVERGED, EINVAL, ENOTPD, ENUMERIC, EHIP, ENOMEM = 0, 1, -1, -2, -3, -4, -5
(OP_KERNEL_MATVEC, OP_SKETCH, OP_PRECOND_BUILD, OP_PRECOND_APPLY, OP_SOLVE, OP_BACKWARD, OP_AUTOTUNE,
 OP_KERNEL_DOT, OP_PRECOND_ADAPTIVE, OP_RIDGE_SKETCH, OP_RIDGE_SOLVE, OP_ADMM_ELASTIC_NET) = range(12)

EXPORTS = ("nys_workspace_bytes", "kernel_matvec", "kernel_dot", "nys_test_matrix", "nys_sketch", "nys_precond_build",
           "nys_precond_adaptive",
           "nys_precond_apply", "nyspcg_solve", "nyspcg_backward", "nys_autotune", "nys_set_tile",
           "nys_clear_tiles", "nys_plan_chunks", "nys_plan_ranges", "nys_peak_probe", "nys_ridge_sketch",
           "nys_ridge_solve",
           "nys_admm_elastic_net", "nys_last_error", "nys_version")

c_i32, c_i64, c_f64, c_vp, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class NysKernel(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("reserved", c_i32), ("sigma", c_f64)]


class NysPrecondC(ctypes.Structure):
    _fields_ = [("n", c_i64), ("r", c_i32), ("rank", c_i32), ("U", c_vp), ("U32", c_vp),
                ("lam_hat", c_vp), ("nu", c_f64), ("shift", c_f64)]


DAMPING_NON_ADAPTIVE, DAMPING_ADAPTIVE = 0, 1


class NysNystromConfig(ctypes.Structure):
    _fields_ = [("rank_init", c_i32), ("rank_max", c_i32), ("num_power_iters", c_i32), ("damping_mode", c_i32),
                ("error_tolerance", c_f64), ("seed", ctypes.c_uint64)]


class NysPCGOpts(ctypes.Structure):
    _fields_ = [("tol", c_f64), ("max_iters", c_i32), ("prec", c_i32), ("refine_every", c_i32),
                ("refine_mode", c_i32), ("check_true", c_i32), ("max_refinements", c_i32),
                ("refine_reduction", c_f64), ("refine_join", c_f64), ("block", c_i32), ("reserved", c_i32)]


class NysAdmmConfig(ctypes.Structure):
    """nys_admm_config (table tab:rlaopt-admm-config; zero fields take their defaults)."""
    _fields_ = [("rho", c_f64), ("rho_update_factor", c_f64), ("rho_update_threshold", c_f64),
                ("rho_update_freq", c_i32), ("precond_update_freq", c_i32), ("alpha", c_f64), ("sigma", c_f64),
                ("gamma", c_f64), ("rank", c_i32), ("max_iters", c_i32), ("eps_abs", c_f64), ("eps_rel", c_f64),
                ("seed", ctypes.c_uint64), ("pcg_max_iters", c_i32), ("reserved", c_i32)]


class NysAdmmInfo(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("converged", c_i32), ("pcg_iters", c_i64), ("r_pri", c_f64), ("r_dual", c_f64),
                ("eps_pri", c_f64), ("eps_dual", c_f64), ("rho", c_f64), ("intercept", c_f64)]


class NysColInfo(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("refinements", c_i32), ("status", c_i32), ("reserved", c_i32),
                ("relres_recursive", c_f64), ("relres_true", c_f64)]


class NysTileChoice(ctypes.Structure):
    _fields_ = [("tm", c_i32), ("reserved", c_i32), ("ms", c_f64)]


class NysError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libnys error {code}: {msg}")
        self.code = code


_lib = None
_lib_file = None
_lib_id = None


def load(path: str | None = None):
    """Load libnys.so (built by paper_2609_08136_amd.build); raises if it is absent."""
    global _lib, _lib_file
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libnys.so not found at {p}: build it with `python -m paper_2609_08136_amd.build`")
    lib = ctypes.CDLL(p)
    lib.nys_last_error.restype = ctypes.c_char_p
    lib.nys_version.restype = ctypes.c_char_p
    lib.nys_workspace_bytes.argtypes = [c_i32, c_i64, c_i64, c_i32, c_i32, c_i32, c_i32, ctypes.POINTER(c_sz)]
    lib.kernel_matvec.argtypes = [NysKernel, c_i32, c_i32, c_vp, c_i64, c_vp, c_i64, c_i32, c_vp, c_i32, c_vp,
                                  c_f64, c_f64, c_vp, c_sz, c_vp]
    lib.kernel_dot.argtypes = [NysKernel, c_i32, c_vp, c_i64, c_vp, c_i64, c_i32, c_vp, c_vp, ctypes.POINTER(c_f64),
                               c_vp, c_sz, c_vp]
    lib.nys_test_matrix.argtypes = [ctypes.c_uint64, c_i64, c_i32, c_vp, c_vp]
    lib.nys_sketch.argtypes = [NysKernel, c_i32, c_vp, c_i64, c_i32, c_vp, ctypes.c_uint64, c_i32, c_vp, c_vp, c_vp,
                               c_sz, c_vp]
    lib.nys_precond_build.argtypes = [c_vp, c_vp, c_i64, c_i32, c_i32, ctypes.POINTER(NysPrecondC), c_vp, c_sz, c_vp]
    lib.nys_precond_apply.argtypes = [ctypes.POINTER(NysPrecondC), c_vp, c_i32, c_vp, c_i32, c_vp, c_vp, c_sz, c_vp]
    lib.nys_precond_adaptive.argtypes = [NysKernel, c_i32, c_vp, c_i64, c_i32, ctypes.POINTER(NysNystromConfig),
                                         ctypes.POINTER(NysPrecondC), ctypes.POINTER(c_f64), c_vp, c_sz, c_vp]
    lib.nyspcg_solve.argtypes = [NysKernel, c_vp, c_i64, c_i32, c_vp, c_i32, ctypes.POINTER(c_f64), c_i32,
                                 ctypes.POINTER(NysPrecondC), ctypes.POINTER(NysPCGOpts), c_vp,
                                 ctypes.POINTER(NysColInfo), c_vp, c_sz, c_vp]
    lib.nyspcg_backward.argtypes = [NysKernel, c_vp, c_i64, c_i32, c_f64, c_vp, c_vp, ctypes.POINTER(NysPrecondC),
                                    ctypes.POINTER(NysPCGOpts), c_vp, ctypes.POINTER(c_f64), ctypes.POINTER(c_f64),
                                    ctypes.POINTER(NysColInfo), c_vp, c_sz, c_vp]
    lib.nys_autotune.argtypes = [NysKernel, c_i32, c_vp, c_i64, c_i64, c_i32, c_i32, c_i32, c_i32,
                                 ctypes.POINTER(NysTileChoice), c_vp, c_sz, c_vp]
    lib.nys_set_tile.argtypes = [c_i32, c_i32, c_i32, c_i32]
    lib.nys_clear_tiles.argtypes = []
    lib.nys_clear_tiles.restype = None
    lib.nys_plan_chunks.argtypes = [c_i32, c_i64, c_i32, c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]
    lib.nys_plan_ranges.argtypes = [c_i32, c_i64, c_i32, c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(c_i64)]
    lib.nys_peak_probe.argtypes = [c_i32, c_i32, ctypes.POINTER(c_f64), c_vp, c_sz, c_vp]
    lib.nys_ridge_sketch.argtypes = [c_vp, c_i64, c_i64, c_vp, ctypes.c_uint64, c_i32, c_vp, c_vp, c_vp, c_sz, c_vp]
    lib.nys_admm_elastic_net.argtypes = [c_vp, c_i64, c_i64, c_vp, c_f64, c_f64, c_f64, c_f64,
                                         ctypes.POINTER(NysAdmmConfig), c_vp, ctypes.POINTER(NysAdmmInfo), c_vp,
                                         c_sz, c_vp]
    lib.nys_ridge_solve.argtypes = [c_vp, c_i64, c_i64, c_vp, c_i32, ctypes.POINTER(c_f64), c_i32,
                                    ctypes.POINTER(NysPrecondC), ctypes.POINTER(NysPCGOpts), c_vp,
                                    ctypes.POINTER(NysColInfo), c_vp, c_sz, c_vp]
    for name in ("kernel_matvec", "kernel_dot", "nys_test_matrix", "nys_sketch", "nys_precond_adaptive", "nys_precond_build", "nys_precond_apply", "nyspcg_solve",
                 "nyspcg_backward", "nys_workspace_bytes", "nys_autotune", "nys_set_tile", "nys_plan_chunks",
                 "nys_plan_ranges", "nys_peak_probe"):
        getattr(lib, name).restype = c_i32
    _lib = lib
    _lib_file = p
    return lib


def library_id() -> str:
    """First 16 hex digits of the SHA-256 of the loaded libnys.so: tuned chunk widths
    belong to one build."""
    global _lib_id
    if _lib_id is None:
        import hashlib
        load()
        h = hashlib.sha256()
        with open(_lib_file, "rb") as f:
            for block in iter(lambda: f.read(1 << 20), b""):
                h.update(block)
        _lib_id = h.hexdigest()[:16]
    return _lib_id


def device_tag(device) -> str:
    """Name of a GPU for cache keys: its marketing name and gfx architecture (the name
    alone can be empty)."""
    props = torch.cuda.get_device_properties(device)
    return f"{props.name}|{getattr(props, 'gcnArchName', '')}"


def version() -> str:
    return load().nys_version().decode()


def _check(rc: int, allow_not_converged: bool = True) -> int:
    if rc == OK or (rc == NOT_CONVERGED and allow_not_converged):
        return rc
    raise NysError(rc, load().nys_last_error().decode())


def _need_cuda(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major)")


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def nys_workspace_bytes(op: int, n: int, n2: int = 0, d: int = 0, r: int = 0, m: int = 0, prec: int = FP64) -> int:
    b = c_sz(0)
    _check(load().nys_workspace_bytes(op, n, n2, d, r, m, prec, ctypes.byref(b)))
    return int(b.value)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _vdtype(prec: int):
    return torch.float64 if prec == FP64 else torch.float32


def kernel_matvec(Xr, Xc, V, kind: int, sigma: float, prec: int = FP64, deriv: int = 0, alpha: float = 1.0,
                  beta: float = 0.0, out=None):
    """Out = alpha K(Xr, Xc) V + beta Out  (deriv=1: dK/dsigma).  Xr, Xc float64 (n x d);
    V, Out float64 for FP64 else float32.  V may be 1-D (one column)."""
    lib = load()
    _need_cuda(Xr, torch.float64, "Xr")
    _need_cuda(Xc, torch.float64, "Xc")
    vec = V.dim() == 1
    V2 = V.reshape(-1, 1) if vec else V
    _need_cuda(V2, _vdtype(prec), "V")
    nr, d = Xr.shape
    nc = Xc.shape[0]
    if Xc.shape[1] != d or V2.shape[0] != nc:
        raise ValueError("shape mismatch")
    m = V2.shape[1]
    if out is None:
        out = torch.empty((nr, m), dtype=V2.dtype, device=V2.device)
        beta = 0.0
    out2 = out.reshape(nr, m)
    _need_cuda(out2, _vdtype(prec), "Out")
    ws = _workspace(nys_workspace_bytes(OP_KERNEL_MATVEC, nr, nc, d, 0, m, prec), Xr.device)
    rc = lib.kernel_matvec(NysKernel(kind, 0, float(sigma)), int(deriv), int(prec), Xr.data_ptr(), nr, Xc.data_ptr(),
                           nc, d, V2.data_ptr(), m, out2.data_ptr(), float(alpha), float(beta), ws.data_ptr(),
                           ws.numel(), _stream())
    _check(rc, allow_not_converged=False)
    return out.reshape(-1) if vec else out


@dataclass
class Preconditioner:
    """Nystrom preconditioner P = U diag(lam_hat) U^T + (lambda + shift) I (buffers on the
    device; shift is the adaptive damping, 0 for the non-adaptive mode)."""
    U: torch.Tensor
    U32: torch.Tensor | None
    lam_hat: torch.Tensor
    rank: int = 0
    nu: float = 0.0
    shift: float = 0.0

    @property
    def n(self) -> int:
        return self.U.shape[0]

    @property
    def r(self) -> int:
        return self.U.shape[1]

    def c_struct(self) -> NysPrecondC:
        return NysPrecondC(self.n, self.r, self.rank, self.U.data_ptr(),
                           self.U32.data_ptr() if self.U32 is not None else None,
                           self.lam_hat.data_ptr(), self.nu, self.shift)


def kernel_dot(Xr, Xc, u, v, kind: int, sigma: float, deriv: int = 0) -> float:
    """u^T K(Xr, Xc) v (deriv=1: u^T (dK/dsigma) v) in float64; u, v 1-D float64."""
    lib = load()
    _need_cuda(Xr, torch.float64, "Xr")
    _need_cuda(Xc, torch.float64, "Xc")
    u1, v1 = u.reshape(-1), v.reshape(-1)
    _need_cuda(u1, torch.float64, "u")
    _need_cuda(v1, torch.float64, "v")
    nr, d = Xr.shape
    nc = Xc.shape[0]
    if Xc.shape[1] != d or u1.numel() != nr or v1.numel() != nc:
        raise ValueError("shape mismatch")
    ws = _workspace(nys_workspace_bytes(OP_KERNEL_DOT, nr, nc, d), Xr.device)
    out = c_f64(0.0)
    _check(lib.kernel_dot(NysKernel(kind, 0, float(sigma)), int(deriv), Xr.data_ptr(), nr, Xc.data_ptr(), nc, d,
                          u1.data_ptr(), v1.data_ptr(), ctypes.byref(out), ws.data_ptr(), ws.numel(), _stream()),
           allow_not_converged=False)
    return float(out.value)


def nys_test_matrix(seed: int, n: int, r: int, device="cuda:0"):
    """Omega (n x r float64) drawn on the device from the seed (counter-based)."""
    Om = torch.empty((n, r), dtype=torch.float64, device=device)
    _check(load().nys_test_matrix(int(seed) & 0xFFFFFFFFFFFFFFFF, n, r, Om.data_ptr(), _stream()),
           allow_not_converged=False)
    return Om


def nys_sketch(X, Omega, kind: int, sigma: float, prec: int = FP64, seed: int = 0, r: int | None = None):
    """(Y, Q) of the Nystrom sketch: Q the orthonormalised test matrix, Y = K Q.
    Omega (n x r float64) is read only; with Omega None, r columns are drawn on the
    device from `seed`."""
    lib = load()
    _need_cuda(X, torch.float64, "X")
    n, d = X.shape
    if Omega is not None:
        _need_cuda(Omega, torch.float64, "Omega")
        if Omega.shape[0] != n or (r is not None and Omega.shape[1] != r):
            raise ValueError("Omega must be n x r")
        r = Omega.shape[1]
    elif r is None:
        raise ValueError("r is required when Omega is None")
    Y = torch.empty((n, r), dtype=torch.float64, device=X.device)
    Q = torch.empty((n, r), dtype=torch.float64, device=X.device)
    ws = _workspace(nys_workspace_bytes(OP_SKETCH, n, 0, d, r, 0, prec), X.device)
    rc = lib.nys_sketch(NysKernel(kind, 0, float(sigma)), int(prec), X.data_ptr(), n, d,
                        Omega.data_ptr() if Omega is not None else None, int(seed) & 0xFFFFFFFFFFFFFFFF, r,
                        Q.data_ptr(), Y.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    _check(rc, allow_not_converged=False)
    return Y, Q


def nys_precond_build(Y, Q, sketch_prec: int = FP64, with_fp32: bool = True) -> Preconditioner:
    lib = load()
    _need_cuda(Y, torch.float64, "Y")
    _need_cuda(Q, torch.float64, "Q")
    n, r = Y.shape
    P = Preconditioner(torch.empty((n, r), dtype=torch.float64, device=Y.device),
                       torch.empty((n, r), dtype=torch.float32, device=Y.device) if with_fp32 else None,
                       torch.empty(r, dtype=torch.float64, device=Y.device))
    cs = P.c_struct()
    ws = _workspace(nys_workspace_bytes(OP_PRECOND_BUILD, n, 0, 0, r, 0, FP64), Y.device)
    rc = lib.nys_precond_build(Y.data_ptr(), Q.data_ptr(), n, r, int(sketch_prec), ctypes.byref(cs), ws.data_ptr(),
                               ws.numel(), _stream())
    _check(rc, allow_not_converged=False)
    P.rank = int(cs.rank)
    P.nu = float(cs.nu)
    return P


def nys_precond_adaptive(X, kind: int, sigma: float, rank_init: int, rank_max: int | None = None,
                         num_power_iters: int = 10, error_tolerance: float = 1e-2, damping: str = "adaptive",
                         prec: int = FP64, seed: int = 0, with_fp32: bool = True):
    """Nystrom preconditioner with rank adaptation and damping mode (NystromConfig of the
    paper's table tab:rlaopt-nystrom-config).  Returns (Preconditioner, error estimate);
    the preconditioner's r is the rank the adaptation settled on."""
    lib = load()
    _need_cuda(X, torch.float64, "X")
    n, d = X.shape
    rmax = rank_init if rank_max is None else int(rank_max)
    mode = {"adaptive": DAMPING_ADAPTIVE, "non_adaptive": DAMPING_NON_ADAPTIVE}[damping]
    cfg = NysNystromConfig(int(rank_init), rmax, int(num_power_iters), mode, float(error_tolerance),
                           int(seed) & 0xFFFFFFFFFFFFFFFF)
    U = torch.empty((n, rmax), dtype=torch.float64, device=X.device)
    U32 = torch.empty((n, rmax), dtype=torch.float32, device=X.device) if with_fp32 else None
    lam = torch.empty(rmax, dtype=torch.float64, device=X.device)
    cs = NysPrecondC(n, rmax, 0, U.data_ptr(), U32.data_ptr() if U32 is not None else None, lam.data_ptr(), 0.0, 0.0)
    ws = _workspace(nys_workspace_bytes(OP_PRECOND_ADAPTIVE, n, 0, d, rmax, 0, prec), X.device)
    err = c_f64(0.0)
    rc = lib.nys_precond_adaptive(NysKernel(kind, 0, float(sigma)), int(prec), X.data_ptr(), n, d, ctypes.byref(cfg),
                                  ctypes.byref(cs), ctypes.byref(err), ws.data_ptr(), ws.numel(), _stream())
    _check(rc, allow_not_converged=False)
    r = int(cs.r)
    # U was written as n x r (row stride r) at the start of the buffer
    Ur = U.reshape(-1)[: n * r].view(n, r)
    U32r = U32.reshape(-1)[: n * r].view(n, r) if U32 is not None else None
    P = Preconditioner(Ur, U32r, lam[:r], int(cs.rank), float(cs.nu), float(cs.shift))
    return P, float(err.value)


def nys_precond_apply(P: Preconditioner, lambdas, R, prec: int = FP64):
    """Z = P_c^{-1} R column by column (lambdas: float64 CUDA tensor, one per column)."""
    lib = load()
    vec = R.dim() == 1
    R2 = R.reshape(-1, 1) if vec else R
    _need_cuda(R2, _vdtype(prec), "R")
    m = R2.shape[1]
    lam = lambdas if isinstance(lambdas, torch.Tensor) else torch.tensor(lambdas, dtype=torch.float64,
                                                                         device=R.device)
    lam = lam.reshape(-1)
    if lam.numel() == 1 and m > 1:
        lam = lam.expand(m).contiguous()
    _need_cuda(lam, torch.float64, "lambdas")
    Z = torch.empty_like(R2)
    ws = _workspace(nys_workspace_bytes(OP_PRECOND_APPLY, P.n, 0, 0, P.r, m, prec), R.device)
    cs = P.c_struct()
    rc = lib.nys_precond_apply(ctypes.byref(cs), lam.data_ptr(), int(prec), R2.data_ptr(), m, Z.data_ptr(),
                               ws.data_ptr(), ws.numel(), _stream())
    _check(rc, allow_not_converged=False)
    return Z.reshape(-1) if vec else Z


def _opts(tol, max_iters, prec, refine_every, refine_mode, check_true, max_refinements,
          refine_reduction=1e-3, refine_join=0.0, block=False) -> NysPCGOpts:
    return NysPCGOpts(float(tol), int(max_iters), int(prec), int(refine_every), int(refine_mode), int(check_true),
                      int(max_refinements), float(refine_reduction), float(refine_join), int(bool(block)), 0)


def _info_list(arr, count):
    return [dict(iters=arr[i].iters, refinements=arr[i].refinements, status=arr[i].status,
                 relres_recursive=arr[i].relres_recursive, relres_true=arr[i].relres_true) for i in range(count)]


def nyspcg_solve(X, B, lambdas, kind: int, sigma: float, P: Preconditioner | None = None, tol: float = 1e-6,
                 max_iters: int = 1000, prec: int = FP64, refine_every: int = -1, refine_mode: int = 0,
                 check_true: bool = False, max_refinements: int = 0, workspace: torch.Tensor | None = None,
                 refine_reduction: float = 1e-3, refine_join: float = 0.0, block: bool = False):
    """Solve (K + lambdas[l] I) x = B[:, j] for every (l, j); column l*nrhs + j of the result.
    block=True: block PCG, the right-hand sides of each lambda sharing one block Krylov
    space.  Returns (Xsol (n x nlam*nrhs float64), info list, status)."""
    lib = load()
    _need_cuda(X, torch.float64, "X")
    vec = B.dim() == 1
    B2 = B.reshape(-1, 1) if vec else B
    _need_cuda(B2, torch.float64, "B")
    n, d = X.shape
    nrhs = B2.shape[1]
    lams = [float(v) for v in (lambdas if hasattr(lambdas, "__len__") else [lambdas])]
    nlam = len(lams)
    m = nlam * nrhs
    Xsol = torch.empty((n, m), dtype=torch.float64, device=X.device)
    info = (NysColInfo * m)()
    lam_arr = (c_f64 * nlam)(*lams)
    need = nys_workspace_bytes(OP_SOLVE, n, 0, d, P.r if P is not None else 0, m, prec)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, X.device)
    o = _opts(tol, max_iters, prec, refine_every, refine_mode, check_true, max_refinements, refine_reduction,
              refine_join, block)
    cs = P.c_struct() if P is not None else None
    rc = lib.nyspcg_solve(NysKernel(kind, 0, float(sigma)), X.data_ptr(), n, d, B2.data_ptr(), nrhs, lam_arr, nlam,
                          ctypes.byref(cs) if cs is not None else None, ctypes.byref(o), Xsol.data_ptr(), info,
                          ws.data_ptr(), ws.numel(), _stream())
    _check(rc)
    return (Xsol.reshape(-1) if (vec and nlam == 1) else Xsol), _info_list(info, m), rc


def nyspcg_backward(X, lam: float, xsol, gx, kind: int, sigma: float, P: Preconditioner | None = None,
                    tol: float = 1e-10, max_iters: int = 1000, prec: int = FP64, refine_every: int = -1,
                    refine_mode: int = 0, check_true: bool = False, max_refinements: int = 0,
                    refine_reduction: float = 1e-3):
    """Adjoint solve (K + lam I) a = gx; returns (a, dL/dlambda, dL/dsigma, info)."""
    lib = load()
    _need_cuda(X, torch.float64, "X")
    xs = xsol.reshape(-1).contiguous()
    g = gx.reshape(-1).contiguous()
    _need_cuda(xs, torch.float64, "xsol")
    _need_cuda(g, torch.float64, "gx")
    n, d = X.shape
    adj = torch.empty(n, dtype=torch.float64, device=X.device)
    dl, ds = c_f64(0.0), c_f64(0.0)
    info = (NysColInfo * 1)()
    ws = _workspace(nys_workspace_bytes(OP_BACKWARD, n, 0, d, P.r if P is not None else 0, 1, prec), X.device)
    o = _opts(tol, max_iters, prec, refine_every, refine_mode, check_true, max_refinements, refine_reduction)
    cs = P.c_struct() if P is not None else None
    rc = lib.nyspcg_backward(NysKernel(kind, 0, float(sigma)), X.data_ptr(), n, d, float(lam), xs.data_ptr(),
                             g.data_ptr(), ctypes.byref(cs) if cs is not None else None, ctypes.byref(o),
                             adj.data_ptr(), ctypes.byref(dl), ctypes.byref(ds), info, ws.data_ptr(), ws.numel(),
                             _stream())
    _check(rc)
    return adj, float(dl.value), float(ds.value), _info_list(info, 1)[0]


def build_preconditioner(X, Omega, kind: int, sigma: float, sketch_prec: int = FP64, with_fp32: bool = True,
                         r: int | None = None, seed: int = 0):
    """Sketch then build: the Nystrom preconditioner for the test matrix Omega (read
    only), or, with Omega None, for r columns drawn on the device from `seed`."""
    Y, Q = nys_sketch(X, Omega, kind, sigma, sketch_prec, seed=seed, r=r)
    P = nys_precond_build(Y, Q, sketch_prec, with_fp32)
    del Y, Q
    return P


# ------------------------------------------------------------------------------ ridge regression

def nys_ridge_sketch(X, Omega, seed: int = 0, r: int | None = None):
    """(Y, Q) of the Nystrom sketch of the normal matrix X^T X (X: n x p float64 CUDA):
    Q the orthonormalised p x r test matrix, Y = X^T (X Q).  Omega as nys_sketch."""
    lib = load()
    _need_cuda(X, torch.float64, "X")
    n, p = X.shape
    if Omega is not None:
        _need_cuda(Omega, torch.float64, "Omega")
        if Omega.shape[0] != p or (r is not None and Omega.shape[1] != r):
            raise ValueError("Omega must be p x r")
        r = Omega.shape[1]
    elif r is None:
        raise ValueError("r is required when Omega is None")
    Y = torch.empty((p, r), dtype=torch.float64, device=X.device)
    Q = torch.empty((p, r), dtype=torch.float64, device=X.device)
    ws = _workspace(nys_workspace_bytes(OP_RIDGE_SKETCH, n, p, 0, r), X.device)
    rc = lib.nys_ridge_sketch(X.data_ptr(), n, p, Omega.data_ptr() if Omega is not None else None,
                              int(seed) & 0xFFFFFFFFFFFFFFFF, r, Q.data_ptr(), Y.data_ptr(), ws.data_ptr(),
                              ws.numel(), _stream())
    _check(rc, allow_not_converged=False)
    return Y, Q


def nys_ridge_solve(X, Y, lambdas, P: Preconditioner | None = None, tol: float = 1e-10, max_iters: int = 1000,
                    check_true: bool = False):
    """NysPCG (CG when P is None) on (X^T X + lambda I) w = X^T y for every lambda and
    every column of Y (n x nrhs, or a vector); column l*nrhs + j of the result.
    Returns (W (p x nlam*nrhs float64), info list, status)."""
    lib = load()
    _need_cuda(X, torch.float64, "X")
    vec = Y.dim() == 1
    Y2 = Y.reshape(-1, 1) if vec else Y
    _need_cuda(Y2, torch.float64, "Y")
    n, p = X.shape
    nrhs = Y2.shape[1]
    lams = [float(v) for v in (lambdas if hasattr(lambdas, "__len__") else [lambdas])]
    nlam = len(lams)
    m = nlam * nrhs
    W = torch.empty((p, m), dtype=torch.float64, device=X.device)
    info = (NysColInfo * m)()
    lam_arr = (c_f64 * nlam)(*lams)
    ws = _workspace(nys_workspace_bytes(OP_RIDGE_SOLVE, n, p, nrhs, P.r if P is not None else 0, m), X.device)
    o = _opts(tol, max_iters, FP64, 0, 0, check_true, 0)
    cs = P.c_struct() if P is not None else None
    rc = lib.nys_ridge_solve(X.data_ptr(), n, p, Y2.data_ptr(), nrhs, lam_arr, nlam,
                             ctypes.byref(cs) if cs is not None else None, ctypes.byref(o), W.data_ptr(), info,
                             ws.data_ptr(), ws.numel(), _stream())
    _check(rc)
    return (W.reshape(-1) if (vec and nlam == 1) else W), _info_list(info, m), rc


def nys_admm_elastic_net(X, y, lam1: float, lam2: float, lo: float = 0.0, hi: float = 1.0, **config):
    """NysADMM on the bounded elastic net (eq. experiment-bounded-en) with the dense data
    matrix X (n x p float64 CUDA) and targets y (n).  Keyword arguments are fields of
    nys_admm_config (rho, alpha, sigma, gamma, rank, max_iters, eps_abs, eps_rel, seed,
    ...); omitted ones take the paper's defaults.  Returns (w, info dict, status)."""
    lib = load()
    _need_cuda(X, torch.float64, "X")
    yv = y.reshape(-1)
    _need_cuda(yv, torch.float64, "y")
    n, p = X.shape
    if yv.numel() != n:
        raise ValueError("y must have one entry per row of X")
    cfg = NysAdmmConfig()
    for k, v in config.items():
        if k not in dict(NysAdmmConfig._fields_):
            raise TypeError(f"unknown nys_admm_config field {k!r}")
        setattr(cfg, k, v)
    rank = cfg.rank or min(50, p)
    W = torch.empty(p, dtype=torch.float64, device=X.device)
    info = NysAdmmInfo()
    ws = _workspace(nys_workspace_bytes(OP_ADMM_ELASTIC_NET, n, p, 0, rank), X.device)
    rc = lib.nys_admm_elastic_net(X.data_ptr(), n, p, yv.data_ptr(), float(lam1), float(lam2), float(lo), float(hi),
                                  ctypes.byref(cfg), W.data_ptr(), ctypes.byref(info), ws.data_ptr(), ws.numel(),
                                  _stream())
    _check(rc)
    return W, {f: getattr(info, f) for f, _ in NysAdmmInfo._fields_}, rc


# ------------------------------------------------------------------------------ autotuner
# Column-count buckets of the batched solve: the product is tuned at each bucket's
# upper end and the choice serves the whole bucket.
TUNE_BUCKETS = ((1, 16), (17, 32), (33, 64), (65, 128), (129, 256), (257, 512), (513, 1024))


def nys_autotune(X, kind: int, sigma: float, prec: int, m: int, m_lo: int | None = None, n_rows: int | None = None,
                 reps: int = 1) -> tuple[int, float]:
    """Time the candidate chunk widths of the product at m columns (rows X[0:n_rows]
    against all of X) and record the fastest for column counts [m_lo, m].
    Returns (width, ms); width 0 when m runs on the row-sum tile."""
    lib = load()
    _need_cuda(X, torch.float64, "X")
    n, d = X.shape
    n_rows = n if n_rows is None else int(n_rows)
    m_lo = m if m_lo is None else int(m_lo)
    ws = _workspace(nys_workspace_bytes(OP_AUTOTUNE, n_rows, n, d, 0, m, prec), X.device)
    best = NysTileChoice()
    _check(lib.nys_autotune(NysKernel(kind, 0, float(sigma)), prec, X.data_ptr(), n, n_rows, d, m, m_lo, reps,
                            ctypes.byref(best), ws.data_ptr(), ws.numel(), _stream()))
    return int(best.tm), float(best.ms)


def nys_set_tile(prec: int, m_lo: int, m_hi: int, tm: int) -> None:
    _check(load().nys_set_tile(prec, m_lo, m_hi, tm))


def nys_clear_tiles() -> None:
    load().nys_clear_tiles()


def nys_plan_chunks(prec: int, n: int, d: int, m: int) -> tuple[int, int]:
    """(chunk width, narrower last-chunk width or 0) the product would use for an
    n x n product with m columns; (0, 0) on the row-sum tile.  Host only."""
    tm, tail = c_i32(0), c_i32(0)
    _check(load().nys_plan_chunks(prec, n, d, m, ctypes.byref(tm), ctypes.byref(tail)))
    return tm.value, tail.value


def nys_plan_ranges(prec: int, n: int, d: int, m: int) -> tuple[int, int]:
    """(number of column-point ranges, points per range) of an n x n product with m
    columns: each range is summed in its own accumulator, the ranges in float64.
    Host only."""
    ranges, points = c_i32(0), c_i64(0)
    _check(load().nys_plan_ranges(prec, n, d, m, ctypes.byref(ranges), ctypes.byref(points)))
    return ranges.value, points.value


PROBE_BF16_MFMA, PROBE_F16_MFMA, PROBE_F64_MFMA, PROBE_EXP2, PROBE_COPY = range(5)


def nys_peak_probe(which: int, iters: int = 0, workspace: torch.Tensor | None = None,
                   device="cuda:0") -> float:
    """Sustained rate of one unit (flop/s, exp/s or copied bytes/s; see include/nys.h)."""
    ws = workspace if workspace is not None else _workspace(8 << 20, device)
    rate = c_f64(0.0)
    _check(load().nys_peak_probe(int(which), int(iters), ctypes.byref(rate), ws.data_ptr(), ws.numel(), _stream()),
           allow_not_converged=False)
    return float(rate.value)


def autotune_fp64_costs(X, kind: int, sigma: float, n_rows: int | None = None, reps: int = 1) -> dict:
    """Measure the float64 product's per-chunk cost of every width on X[0:n_rows] x X
    and install it as the float64 planner's cost table (the refinement residuals and
    float64 solves then size every product by measured cost).  Returns the width the
    planner takes at 256 columns and its estimated milliseconds."""
    n_rows = X.shape[0] if n_rows is None else min(int(n_rows), X.shape[0])
    tm, ms = nys_autotune(X, kind, sigma, FP64, 256, m_lo=1, n_rows=n_rows, reps=reps)
    return {"tm_at_256": tm, "ms_at_256": ms, "n_rows": n_rows}


def autotune(X, kind: int, sigma: float, prec: int, m_max: int, cache: str | None = None, reps: int = 1,
             n_rows: int | None = None) -> dict:
    """Tune every column-count bucket up to m_max (see TUNE_BUCKETS), timing rows
    X[0:n_rows] against all of X (the chunk width is a property of the tile, so a
    row subsample keeps the tuning short).  With `cache`
    (a JSON file), choices recorded for the same device, library build, precision,
    kernel and point set shape are installed instead of re-timed, and new ones are
    added to it."""
    import json
    n_rows = X.shape[0] if n_rows is None else min(int(n_rows), X.shape[0])
    key = (f"{device_tag(X.device)}|lib{library_id()}|prec{prec}|kind{kind}|n{X.shape[0]}|d{X.shape[1]}"
           f"|rows{n_rows}")
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
    entries = table.get(key, {})
    out = {}
    for lo, hi in TUNE_BUCKETS:
        if lo > m_max:
            break
        tag = f"{lo}-{hi}"
        if tag in entries:
            tm = int(entries[tag]["tm"])
            if tm:
                nys_set_tile(prec, lo, hi, tm)
            out[tag] = entries[tag]
            continue
        tm, ms = nys_autotune(X, kind, sigma, prec, min(hi, m_max), m_lo=lo, n_rows=n_rows, reps=reps)
        if tm and hi > m_max:
            nys_set_tile(prec, lo, hi, tm)
        out[tag] = entries[tag] = {"tm": tm, "ms": ms}
    if cache:
        table[key] = entries
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1)
    return out
