"""Python binding of liblrcc, the MI355X particle-particle-ladder library.

Argument marshalling only: every step of the ladder product, its adjoint and
the response solve runs in the library's HIP kernels.  PyTorch provides the
device memory and the stream.  There is no CPU fallback: if liblrcc.so is
missing or no gfx950 device is present, the calls raise.

    import paper_2604_12914_amd as lrcc
    sigma = lrcc.ppl_sigma(L, X)                 # torch complex tensors on cuda
    dX, dL = lrcc.ppl_sigma_adjoint(L, X, G)
    alpha, info = lrcc.solve(eps, L, mu, omegas)
"""
from __future__ import annotations

import ctypes
import math
import os
import re
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "liblrcc.so")
HEADER = os.path.join(ROOT, "include", "lrcc.h")

# enums of include/lrcc.h
STATUS = {0: "LRCC_OK", 1: "LRCC_ERR_ARG", 2: "LRCC_ERR_SHAPE", 3: "LRCC_ERR_DTYPE",
          4: "LRCC_ERR_DEVICE", 5: "LRCC_ERR_NOMEM", 6: "LRCC_ERR_NOT_CONVERGED",
          7: "LRCC_ERR_NONFINITE", 8: "LRCC_ERR_UNSUPPORTED"}
OK, ERR_ARG, ERR_SHAPE, ERR_DTYPE, ERR_DEVICE, ERR_NOMEM, ERR_NOT_CONVERGED, \
    ERR_NONFINITE, ERR_UNSUPPORTED = range(9)
C128, C64 = 0, 1
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
CMUL = {"4m": 0, "3m": 1}


class LrccError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("diis_dim", ctypes.c_int), ("prec", ctypes.c_int),
                ("cmul", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("deterministic", ctypes.c_int),
                ("resid_fp64_every", ctypes.c_int), ("anchor_prec", ctypes.c_int),
                ("response", ctypes.c_int), ("L_oo", ctypes.c_void_p),
                ("L_ov", ctypes.c_void_p), ("L_vo", ctypes.c_void_p),
                ("x0", ctypes.c_void_p), ("x_out", ctypes.c_void_p),
                ("metrics_path", ctypes.c_char_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters_max", ctypes.c_int), ("n_sigma_fp64", ctypes.c_int),
                ("n_sigma_lowp", ctypes.c_int), ("final_relres", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FnsInfo(ctypes.Structure):
    _fields_ = [("sweeps_density", ctypes.c_int), ("sweeps_fock", ctypes.c_int)]


class TuneResult(ctypes.Structure):
    _fields_ = [("supertile", ctypes.c_int), ("occupancy", ctypes.c_int),
                ("ms", ctypes.c_double), ("candidates", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Instance(ctypes.Structure):
    _fields_ = [("o", ctypes.c_int), ("v", ctypes.c_int), ("nchol", ctypes.c_int),
                ("eps", ctypes.c_void_p), ("L", ctypes.c_void_p), ("ncomp", ctypes.c_int),
                ("mu", ctypes.c_void_p), ("nomega", ctypes.c_int),
                ("omegas", ctypes.c_void_p), ("alpha", ctypes.c_void_p)]


_lib = None
_lock = threading.Lock()
_handles = {}


def header_symbols():
    """Names of the functions include/lrcc.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:lrcc_status|const char\*)\s+(lrcc_\w+)\s*\(",
                                 text, re.M)))


def lib() -> ctypes.CDLL:
    """Load liblrcc.so (built by paper_2604_12914_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run "
                               "'python -m paper_2604_12914_amd.build'")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        sig = {
            "lrcc_create": [ctypes.POINTER(vp), i, vp],
            "lrcc_destroy": [vp],
            "lrcc_set_stream": [vp, vp],
            "lrcc_ppl_sigma": [vp, i, i, i, i, vp, vp, vp, i, i, i],
            "lrcc_ppl_sigma_noalloc": [vp, i, i, i, i, vp, vp, vp, i, i, i],
            "lrcc_ppl_sigma_adjoint": [vp, i, i, i, i, vp, vp, vp, vp, vp, i, i, i],
            "lrcc_hhl_sigma": [vp, i, i, i, i, vp, vp, vp, i],
            "lrcc_cholesky": [vp, ctypes.c_long, vp, d, i, vp, vp, ctypes.POINTER(i)],
            "lrcc_heev": [vp, i, vp, vp, vp, ctypes.POINTER(i)],
            "lrcc_ring_sigma": [vp, i, i, i, i, vp, vp, vp, vp, vp, vp],
            "lrcc_fns_transform": [vp, i, i, i, i, i, vp, vp, vp, vp, vp],
            "lrcc_fns_plus": [vp, i, i, i, vp, vp, i, vp, vp, vp, d, d, vp, vp, vp,
                              ctypes.POINTER(i), vp, vp, ctypes.POINTER(FnsInfo)],
            "lrcc_solve": [vp, i, i, i, vp, vp, i, vp, i, vp,
                           ctypes.POINTER(SolveOpts), vp, ctypes.POINTER(SolveInfo)],
            "lrcc_solve_batched": [vp, i, ctypes.POINTER(Instance),
                                   ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo)],
            "lrcc_check_sigma_args": [i, i, i, i, vp, vp, vp, i, i, i],
            "lrcc_set_timing": [vp, i],
            "lrcc_set_deterministic": [vp, i],
            "lrcc_set_workspace_limit": [vp, ctypes.c_size_t],
            "lrcc_autotune": [vp, i, i, i, i, i, i, ctypes.c_char_p, ctypes.POINTER(TuneResult)],
            "lrcc_get_timing": [vp, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_long)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        for name in ("lrcc_status_str",):
            getattr(L, name).argtypes = [ctypes.c_int]
            getattr(L, name).restype = ctypes.c_char_p
        L.lrcc_last_error.argtypes = [vp]
        L.lrcc_last_error.restype = ctypes.c_char_p
        L.lrcc_version.argtypes = []
        L.lrcc_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status: int, h=None):
    if status != OK:
        msg = lib().lrcc_last_error(h).decode()
        raise LrccError(status, msg)


def handle(device: int):
    """Per-device library handle (created once, bound to torch's stream)."""
    import torch
    with _lock:
        h = _handles.get(device)
        if h is None:
            hp = ctypes.c_void_p()
            _check(lib().lrcc_create(ctypes.byref(hp), device, None))
            h = hp.value
            _handles[device] = h
    stream = torch.cuda.current_stream(device).cuda_stream
    _check(lib().lrcc_set_stream(h, ctypes.c_void_p(stream)), h)
    return h


def _dtype_code(t):
    import torch
    if t.dtype == torch.complex128:
        return C128
    if t.dtype == torch.complex64:
        return C64
    raise TypeError(f"expected complex64 or complex128, got {t.dtype}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


def _o_from_npo(npo: int) -> int:
    o = int(round((1 + math.sqrt(1 + 8 * npo)) / 2)) if npo else 0
    if o * (o - 1) // 2 != npo:
        raise ValueError(f"{npo} is not a pair count o(o-1)/2")
    return o


def _geometry(L, X, o):
    if L.dim() != 3 or L.shape[1] != L.shape[2]:
        raise ValueError("L must be [nchol, v, v]")
    if X.dim() != 3:
        raise ValueError("X must be [nrhs, o(o-1)/2, v(v-1)/2]")
    nchol, v = L.shape[0], L.shape[1]
    if X.shape[2] != v * (v - 1) // 2:
        raise ValueError("X's last extent must be v(v-1)/2")
    o = _o_from_npo(X.shape[1]) if o is None else o
    if X.shape[1] != o * (o - 1) // 2:
        raise ValueError("X's middle extent must be o(o-1)/2")
    if not (L.is_cuda and X.is_cuda and L.device == X.device):
        raise ValueError("L and X must be on the same GPU")
    if L.dtype != X.dtype:
        raise TypeError("L and X must have the same dtype")
    return nchol, v, o, X.shape[0], X.device.index


def ppl_sigma(L, X, o=None, prec="fp64", cmul="4m", out=None):
    """sigma = PPL(L, X) on the GPU; returns a new tensor (or fills ``out``)."""
    import torch
    L, X = L.contiguous(), X.contiguous()
    nchol, v, o, nrhs, dev = _geometry(L, X, o)
    out = torch.empty_like(X) if out is None else out
    h = handle(dev)
    _check(lib().lrcc_ppl_sigma(h, o, v, nchol, nrhs, _ptr(L), _ptr(X), _ptr(out),
                                _dtype_code(X), PREC[prec], CMUL[cmul]), h)
    return out


def ppl_sigma_noalloc(L, X, out, o=None, prec="fp64", cmul="4m"):
    """sigma = PPL(L, X) into the caller's ``out`` through the allocation-free
    entry point (the library allocates nothing; FP64 or FP32 ladder)."""
    L, X = L.contiguous(), X.contiguous()
    nchol, v, o, nrhs, dev = _geometry(L, X, o)
    if out.shape != X.shape or out.dtype != X.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous tensor shaped like X")
    h = handle(dev)
    _check(lib().lrcc_ppl_sigma_noalloc(h, o, v, nchol, nrhs, _ptr(L), _ptr(X), _ptr(out),
                                        _dtype_code(X), PREC[prec], CMUL[cmul]), h)
    return out


def hhl_sigma(Loo, X, v=None, out=None):
    """Hole-hole ladder sigma_ij^ab = sum_kl <kl||ij> X_kl^ab on the GPU (FP64
    arithmetic); Loo [nchol, o, o], X packed [nrhs, o(o-1)/2, v(v-1)/2]."""
    import torch
    Loo, X = Loo.contiguous(), X.contiguous()
    if Loo.dim() != 3 or Loo.shape[1] != Loo.shape[2] or X.dim() != 3:
        raise ValueError("Loo must be [nchol, o, o] and X [nrhs, npo, npv]")
    if Loo.dtype != X.dtype or X.dtype not in (torch.complex128, torch.complex64):
        raise TypeError("Loo and X must share a complex dtype")
    nchol, o = Loo.shape[0], Loo.shape[1]
    nrhs, npo, npv = X.shape
    if npo != o * (o - 1) // 2:
        raise ValueError("X's occupied-pair count does not match Loo")
    if v is None:
        v = int(round((1 + (1 + 8 * npv) ** 0.5) / 2))
    if npv != v * (v - 1) // 2:
        raise ValueError("X's virtual-pair count does not match v")
    out = torch.empty_like(X) if out is None else out
    h = handle(X.device.index)
    _check(lib().lrcc_hhl_sigma(h, o, v, nchol, nrhs, _ptr(Loo), _ptr(X), _ptr(out),
                                _dtype_code(X)), h)
    return out


def cholesky(M, tau=1e-5, max_vectors=None):
    """Pivoted Cholesky decomposition of a Hermitian PSD matrix M [n, n]
    (complex128, on the GPU): returns (L [k, n] tensor, pivots [k] numpy) with
    M ~= sum_q L_q L_q^H and every remaining diagonal element <= tau."""
    import numpy as np
    import torch
    M = M.contiguous()
    if M.dim() != 2 or M.shape[0] != M.shape[1] or M.dtype != torch.complex128:
        raise ValueError("M must be a square complex128 matrix")
    n = M.shape[0]
    kmax = n if max_vectors is None else min(int(max_vectors), n)
    L = torch.empty((kmax, n), dtype=torch.complex128, device=M.device)
    piv = torch.empty((kmax,), dtype=torch.int32, device=M.device)
    cnt = ctypes.c_int(0)
    h = handle(M.device.index)
    _check(lib().lrcc_cholesky(h, n, _ptr(M), float(tau), kmax, _ptr(L),
                               piv.data_ptr() if kmax else None, ctypes.byref(cnt)), h)
    k = cnt.value
    return L[:k], piv[:k].cpu().numpy().astype(np.int64)


def ring_sigma(Loo, Lov, Lvo, Lvv, X, o=None, out=None):
    """Ring term P(ij)P(ab) sum_kc <kb||cj> X_ik^ac on packed complex128
    doubles X [nrhs, npo, npv]; the four Cholesky blocks [nchol, ., .]."""
    import torch
    Loo, Lov, Lvo, Lvv, X = (t.contiguous() for t in (Loo, Lov, Lvo, Lvv, X))
    nchol, v = Lvv.shape[0], Lvv.shape[1]
    o = Lov.shape[1] if o is None else o
    for t, shp in ((Loo, (nchol, o, o)), (Lov, (nchol, o, v)), (Lvo, (nchol, v, o)),
                   (Lvv, (nchol, v, v))):
        if tuple(t.shape) != shp or t.dtype != torch.complex128:
            raise ValueError(f"expected complex128 {shp}, got {t.dtype} {tuple(t.shape)}")
    if X.dim() != 3 or X.shape[1:] != (o * (o - 1) // 2, v * (v - 1) // 2) or \
            X.dtype != torch.complex128:
        raise ValueError("X must be complex128 [nrhs, o(o-1)/2, v(v-1)/2]")
    S = torch.empty_like(X) if out is None else out
    h = handle(X.device.index)
    _check(lib().lrcc_ring_sigma(h, o, v, nchol, X.shape[0], _ptr(Loo), _ptr(Lov), _ptr(Lvo),
                                 _ptr(Lvv), _ptr(X), _ptr(S)), h)
    return S


def fns_transform(B, L=None, mu=None):
    """(Lt, mu_t): Cholesky vectors L [nchol, v, v] and dipole block
    mu [ncomp, o, v] in the kept FNS++ basis B [v, k] (complex128, GPU):
    Lt^P = B^H L^P B, mu_t = mu conj(B)."""
    import torch
    B = B.contiguous()
    v, k = B.shape
    Lt = mt = None
    nchol = ncomp = o = 0
    if L is not None:
        L = L.contiguous()
        nchol = L.shape[0]
        if tuple(L.shape) != (nchol, v, v) or L.dtype != torch.complex128:
            raise ValueError("L must be complex128 [nchol, v, v]")
        Lt = torch.empty((nchol, k, k), dtype=torch.complex128, device=B.device)
    if mu is not None:
        mu = mu.contiguous()
        ncomp, o = mu.shape[0], mu.shape[1]
        if tuple(mu.shape) != (ncomp, o, v) or mu.dtype != torch.complex128:
            raise ValueError("mu must be complex128 [ncomp, o, v]")
        mt = torch.empty((ncomp, o, k), dtype=torch.complex128, device=B.device)
    h = handle(B.device.index)
    _check(lib().lrcc_fns_transform(h, v, k, nchol, ncomp, o, _ptr(B), _ptr(L), _ptr(mu),
                                    _ptr(Lt), _ptr(mt)), h)
    return Lt, mt


def heev(A, vectors=True):
    """Eigen-decomposition of a Hermitian complex128 matrix on the GPU by
    Jacobi rotations: returns (w ascending, V with eigenvectors as columns or
    None, sweeps)."""
    import torch
    A = A.contiguous()
    if A.dim() != 2 or A.shape[0] != A.shape[1] or A.dtype != torch.complex128:
        raise ValueError("A must be a square complex128 matrix")
    n = A.shape[0]
    w = torch.empty((n,), dtype=torch.float64, device=A.device)
    V = torch.empty((n, n), dtype=torch.complex128, device=A.device) if vectors else None
    sw = ctypes.c_int(0)
    h = handle(A.device.index)
    _check(lib().lrcc_heev(h, n, _ptr(A), _ptr(w), _ptr(V), ctypes.byref(sw)), h)
    return w, V, sw.value


def fns_plus(eps, Lov, A_ov, A_vv, A_oo, omega=0.0, threshold=1e-5):
    """FNS++ virtual basis on the GPU (all inputs complex128/float64 device
    tensors; eps [o+v], Lov [nchol, o, v], A_ov [ncomp, o, v],
    A_vv [ncomp, v, v], A_oo [ncomp, o, o]).  Returns a dict with occ [v]
    (|n| descending), keep, B [v, keep], eps_new [keep], gamma [v, v],
    hbar [o+v] and the Jacobi sweep counts."""
    import torch
    eps, Lov = eps.contiguous(), Lov.contiguous()
    A_ov, A_vv, A_oo = A_ov.contiguous(), A_vv.contiguous(), A_oo.contiguous()
    nchol, o, v = Lov.shape
    ncomp = A_vv.shape[0]
    if eps.shape != (o + v,) or eps.dtype != torch.float64:
        raise ValueError("eps must be float64 [o+v]")
    for t, shp in ((Lov, (nchol, o, v)), (A_ov, (ncomp, o, v)), (A_vv, (ncomp, v, v)),
                   (A_oo, (ncomp, o, o))):
        if tuple(t.shape) != shp or t.dtype != torch.complex128:
            raise ValueError(f"expected complex128 {shp}, got {t.dtype} {tuple(t.shape)}")
    dev = Lov.device
    occ = torch.empty((v,), dtype=torch.float64, device=dev)
    B = torch.empty((v * v,), dtype=torch.complex128, device=dev)
    en = torch.empty((v,), dtype=torch.float64, device=dev)
    gamma = torch.empty((v, v), dtype=torch.complex128, device=dev)
    hbar = torch.empty((o + v,), dtype=torch.float64, device=dev)
    keep = ctypes.c_int(0)
    info = FnsInfo()
    h = handle(dev.index)
    _check(lib().lrcc_fns_plus(h, o, v, nchol, _ptr(eps), _ptr(Lov), ncomp, _ptr(A_ov),
                               _ptr(A_vv), _ptr(A_oo), float(omega), float(threshold),
                               _ptr(occ), _ptr(B), _ptr(en), ctypes.byref(keep), _ptr(gamma),
                               _ptr(hbar), ctypes.byref(info)), h)
    k = keep.value
    return {"occ": occ, "keep": k, "B": B[:v * k].view(v, k), "eps_new": en[:k],
            "gamma": gamma, "hbar": hbar, "sweeps_density": info.sweeps_density,
            "sweeps_fock": info.sweeps_fock}


def ppl_sigma_adjoint(L, X, G, o=None, want_dX=True, want_dL=True, prec="fp64", cmul="4m"):
    """(dX, dL) for upstream gradient G of sigma = PPL(L, X)."""
    import torch
    L, X, G = L.contiguous(), X.contiguous(), G.contiguous()
    nchol, v, o, nrhs, dev = _geometry(L, X, o)
    if G.shape != X.shape or G.dtype != X.dtype:
        raise ValueError("G must match X")
    dX = torch.empty_like(X) if want_dX else None
    dL = torch.empty_like(L) if want_dL else None
    h = handle(dev)
    _check(lib().lrcc_ppl_sigma_adjoint(h, o, v, nchol, nrhs, _ptr(L), _ptr(X), _ptr(G),
                                        _ptr(dX), _ptr(dL), _dtype_code(X), PREC[prec],
                                        CMUL[cmul]), h)
    return dX, dL


def autotune(o, v, nchol, nrhs, prec="fp64", cmul="4m", cache_path=None, device=0):
    """Time the ladder's launch variants for this shape and keep the fastest
    in the device's handle; returns the choice as a dict."""
    h = handle(device)
    res = TuneResult()
    cp = cache_path.encode() if cache_path else None
    _check(lib().lrcc_autotune(h, o, v, nchol, nrhs, PREC[prec], CMUL[cmul], cp,
                               ctypes.byref(res)), h)
    return res.as_dict()


def set_timing(enable: bool, device: int = 0):
    """Start (clearing totals) or stop HIP-event timing of ladder kernels."""
    h = handle(device)
    _check(lib().lrcc_set_timing(h, 1 if enable else 0), h)


def set_deterministic(enable: bool, device: int = 0):
    """Deterministic (atomic-free, bit-reproducible) ladders on this device's handle."""
    h = handle(device)
    _check(lib().lrcc_set_deterministic(h, int(bool(enable))), h)


def set_workspace_limit(nbytes: int, device: int = 0):
    """Cap the bf16x3 ladder's integral-panel workspace (0 = default)."""
    h = handle(device)
    _check(lib().lrcc_set_workspace_limit(h, int(nbytes)), h)


def get_timing(device: int = 0):
    """(summed ladder-kernel milliseconds, launches) since timing was enabled."""
    h = handle(device)
    ms, n = ctypes.c_double(), ctypes.c_long()
    _check(lib().lrcc_get_timing(h, ctypes.byref(ms), ctypes.byref(n)), h)
    return ms.value, n.value


def _autograd_function():
    import torch

    class PPLSigma(torch.autograd.Function):
        """sigma = PPL(L, X) with a hand-written backward (adjoint ladder and
        dL kernels; integral tiles recomputed, never stored)."""

        @staticmethod
        def forward(ctx, L, X, prec="fp64", cmul="4m"):
            ctx.save_for_backward(L, X)
            ctx.prec, ctx.cmul = prec, cmul
            return ppl_sigma(L, X, prec=prec, cmul=cmul)

        @staticmethod
        def backward(ctx, G):
            L, X = ctx.saved_tensors
            dX, dL = ppl_sigma_adjoint(L, X, G, want_dX=ctx.needs_input_grad[1],
                                       want_dL=ctx.needs_input_grad[0],
                                       prec=ctx.prec, cmul=ctx.cmul)
            return dL, dX, None, None

    return PPLSigma


_PPLSigma = None


def PPLSigma():
    """The torch.autograd.Function class (created on first use)."""
    global _PPLSigma
    if _PPLSigma is None:
        _PPLSigma = _autograd_function()
    return _PPLSigma


def ppl(L, X, prec="fp64", cmul="4m"):
    """Differentiable sigma = PPL(L, X)."""
    return PPLSigma().apply(L, X, prec, cmul)


RESPONSE = {"right": 0, "full": 1}


def solve(eps, L, mu, omegas, tol=1e-8, max_iter=100, diis_dim=8, prec="fp64",
          cmul="4m", inner_tol=1e-5, max_outer=6, check=True, resid_fp64_every=0,
          anchor_prec="fp64", response="right", Loo=None, Lov=None, Lvo=None,
          deterministic=False, x0=None, x_out=None, metrics_path=None):
    """Model response solve; returns (alpha [nomega, ncomp, ncomp] complex128 numpy,
    info dict).  response="right": alpha from the right-hand amplitudes;
    "full": the full response function (right- and left-hand solves).
    Loo: occupied-occupied Cholesky vectors [nchol, o, o] (complex128) to
    include the hole-hole ladder in the model Jacobian; with it, Lov
    [nchol, o, v] and Lvo [nchol, v, o] add the ring term.
    x0 / x_out: initial / final right-hand amplitudes, complex128 tensors
    [nomega, ncomp, o(o-1)/2, v(v-1)/2] on the GPU (warm start, checkpoint);
    metrics_path: a file that receives one JSON line per iteration;
    deterministic: atomic-free, bit-reproducible ladders."""
    import numpy as np
    import torch
    L, mu, eps = L.contiguous(), mu.contiguous(), eps.contiguous()
    if L.dtype != torch.complex128 or mu.dtype != torch.complex128 or eps.dtype != torch.float64:
        raise TypeError("solve takes complex128 L and mu and float64 eps")
    nchol, v = L.shape[0], L.shape[1]
    ncomp, o = mu.shape[0], mu.shape[1]
    om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
    alpha = np.zeros((len(om), ncomp, ncomp), dtype=np.complex128)
    if Loo is not None:
        Loo = Loo.contiguous()
        if Loo.dtype != torch.complex128 or tuple(Loo.shape) != (nchol, o, o):
            raise ValueError("Loo must be complex128 [nchol, o, o]")
    if (Lov is None) != (Lvo is None):
        raise ValueError("Lov and Lvo come together")
    if Lov is not None:
        Lov, Lvo = Lov.contiguous(), Lvo.contiguous()
        if Lov.dtype != torch.complex128 or tuple(Lov.shape) != (nchol, o, v) or \
                Lvo.dtype != torch.complex128 or tuple(Lvo.shape) != (nchol, v, o):
            raise ValueError("Lov must be complex128 [nchol, o, v] and Lvo [nchol, v, o]")
    shape = (len(om), ncomp, o * (o - 1) // 2, v * (v - 1) // 2)
    for name, t in (("x0", x0), ("x_out", x_out)):
        if t is not None and (t.dtype != torch.complex128 or tuple(t.shape) != shape
                              or not t.is_contiguous() or not t.is_cuda):
            raise ValueError(f"{name} must be a contiguous complex128 GPU tensor {shape}")
    opts = SolveOpts(tol, max_iter, diis_dim, PREC[prec], CMUL[cmul], inner_tol, max_outer,
                     int(bool(deterministic)), resid_fp64_every, PREC[anchor_prec],
                     RESPONSE[response],
                     Loo.data_ptr() if Loo is not None else None,
                     Lov.data_ptr() if Lov is not None else None,
                     Lvo.data_ptr() if Lvo is not None else None,
                     x0.data_ptr() if x0 is not None and x0.numel() else None,
                     x_out.data_ptr() if x_out is not None and x_out.numel() else None,
                     metrics_path.encode() if metrics_path else None)
    info = SolveInfo()
    h = handle(L.device.index)
    st = lib().lrcc_solve(h, o, v, nchol, _ptr(eps), _ptr(L), ncomp, _ptr(mu), len(om),
                          om.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts),
                          alpha.ctypes.data_as(ctypes.c_void_p), ctypes.byref(info))
    if st != OK and (check or st != ERR_NOT_CONVERGED):
        _check(st, h)
    return alpha, dict(info.as_dict(), status=STATUS[st])


def solve_batched(instances, tol=1e-8, max_iter=100, diis_dim=8, prec="fp64", cmul="4m",
                  inner_tol=1e-5, max_outer=6, check=True, resid_fp64_every=0,
                  deterministic=False):
    """Batched solve of several instances: each a dict(eps, L, mu, omegas)."""
    import numpy as np
    import torch
    keep, arr = [], (Instance * len(instances))()
    alphas = []
    dev = None
    for k, inst in enumerate(instances):
        L, mu, eps = (inst["L"].contiguous(), inst["mu"].contiguous(),
                      inst["eps"].contiguous())
        if L.dtype != torch.complex128 or mu.dtype != torch.complex128:
            raise TypeError("solve_batched takes complex128 L and mu")
        om = np.ascontiguousarray(np.asarray(inst["omegas"], dtype=np.float64))
        al = np.zeros((len(om), mu.shape[0], mu.shape[0]), dtype=np.complex128)
        keep += [L, mu, eps, om]
        alphas.append(al)
        dev = L.device.index
        arr[k] = Instance(mu.shape[1], L.shape[1], L.shape[0], eps.data_ptr(), L.data_ptr(),
                          mu.shape[0], mu.data_ptr(), len(om), om.ctypes.data, al.ctypes.data)
    opts = SolveOpts(tol, max_iter, diis_dim, PREC[prec], CMUL[cmul], inner_tol, max_outer,
                     int(bool(deterministic)), resid_fp64_every, 0, 0)
    info = SolveInfo()
    h = handle(dev)
    st = lib().lrcc_solve_batched(h, len(instances), arr, ctypes.byref(opts), ctypes.byref(info))
    if st != OK and (check or st != ERR_NOT_CONVERGED):
        _check(st, h)
    return alphas, dict(info.as_dict(), status=STATUS[st])
