"""Python binding of libbsparareal.so: Parareal for the Black-Scholes equation
on an AMD Instinct MI355X (gfx950).

Argument marshalling only: every computation runs in the HIP kernels behind
the C ABI declared in ``include/bsparareal.h``.  torch tensors provide device
memory, ``torch.cuda.current_stream()`` provides the HIP stream.  There is no
CPU fallback: if the library is not built, or no GPU is present, the calls
raise.

Names follow the C ABI one to one:
``bs_initial``, ``bs_fine_propagate_batch``, ``bs_coarse_numeric``,
``pinn_forward``, ``pinn_residual_fwd_bwd``, ``parareal_start``,
``parareal_iterate``, ``parareal_solve``.
"""
from __future__ import annotations

import atexit
import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsparareal.so")

BS_OK, BS_NOT_CONVERGED = 0, 1
BS_ERR_ARG, BS_ERR_HIP, BS_ERR_NONFINITE, BS_ERR_DIVERGED, BS_ERR_WORKSPACE = -1, -2, -3, -4, -5
BS_DIVERGENCE_GROWTH = 1.0e3
COARSE_IE, COARSE_PINN, COARSE_PINN_IE, COARSE_FLOWMAP = 0, 1, 2, 3
PREC_FP32, PREC_BF16 = 0, 1

EXPORTS = ("bs_last_error", "bs_initial", "bs_fine_propagate_batch", "bs_coarse_numeric",
           "pinn_forward", "pinn_residual_workspace_size", "pinn_residual_fwd_bwd",
           "parareal_workspace_size", "parareal_start", "parareal_iterate", "parareal_solve",
           "parareal_batch_workspace_size", "parareal_solve_batch",
           "bs_tune_set_shape", "bs_tune_reset", "bs_profile_enable", "bs_profile_read",
           "bs_set_divergence_growth", "bs_divergence_growth", "bs_release_resources",
           "parareal_solve_noalloc")
BS_NOALLOC_SCRATCH_BYTES = 8 << 20


class BsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bsparareal error {code}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("K", ctypes.c_double), ("r", ctypes.c_double), ("sigma", ctypes.c_double),
                ("T", ctypes.c_double), ("s_max", ctypes.c_double), ("is_put", ctypes.c_int)]


class _Grid(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("payoff_mode", ctypes.c_int)]


class _Slices(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("fine_steps", ctypes.c_int), ("coarse_steps", ctypes.c_int)]


class _Net(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int), ("depth", ctypes.c_int), ("width", ctypes.c_int),
                ("precision", ctypes.c_int), ("params", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libbsparareal.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2303_03848_amd.build`")
    lib = ctypes.CDLL(path)
    P, G, S, N = (ctypes.POINTER(c) for c in (_Params, _Grid, _Slices, _Net))
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    ip, dp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    szp = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "bs_last_error": (ctypes.c_char_p, []),
        "bs_initial": (i, [P, G, vp, vp]),
        "bs_fine_propagate_batch": (i, [P, G, i, vp, d, i, vp, vp, vp]),
        "bs_coarse_numeric": (i, [P, G, i, vp, d, i, vp, vp, vp]),
        "pinn_forward": (i, [N, i, vp, vp, vp]),
        "pinn_residual_workspace_size": (i, [N, i, i, i, szp]),
        "pinn_residual_fwd_bwd": (i, [N, P, i, vp, i, vp, vp, i, vp, vp, vp, vp, vp, sz, vp]),
        "parareal_workspace_size": (i, [G, S, i, szp]),
        "parareal_start": (i, [P, G, S, i, N, vp, sz, vp, vp]),
        "parareal_iterate": (i, [P, G, S, i, N, vp, sz, vp, i, dp, ip, vp]),
        "parareal_solve": (i, [P, G, S, i, d, N, i, vp, sz, vp, ip, dp, vp]),
        "parareal_solve_noalloc": (i, [P, G, S, i, d, N, i, vp, ip, dp, vp]),
        "parareal_batch_workspace_size": (i, [i, P, G, S, i, szp]),
        "parareal_solve_batch": (i, [i, P, G, S, i, d, N, i, vp, sz, vp,
                                     ctypes.POINTER(ctypes.c_long), ip, dp, i, vp]),
        "bs_tune_set_shape": (i, [i, i, i, i, i]),
        "bs_tune_reset": (i, []),
        "bs_profile_enable": (i, [i]),
        "bs_profile_read": (i, [dp]),
        "bs_set_divergence_growth": (i, [d]),
        "bs_divergence_growth": (d, []),
        "bs_release_resources": (i, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    # the library's pinned buffers, streams and tables go before the HIP
    # runtime shuts down
    atexit.register(_release_at_exit)
    return lib


def _release_at_exit():
    if _lib is not None:
        try:
            import torch as _t
            if _t.cuda.is_initialized():
                _t.cuda.synchronize()
                _lib.bs_release_resources()
        except Exception:  # interpreter shutdown: nothing left to report to
            pass


def _check(rc: int) -> int:
    if rc < 0:
        msg = load_library().bs_last_error().decode(errors="replace")
        raise BsError(rc, msg)
    return rc


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str) -> int:
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    return t.data_ptr()


def _params(p: dict) -> _Params:
    return _Params(float(p["K"]), float(p["r"]), float(p["sigma"]), float(p["T"]),
                   float(p["s_max"]), int(bool(p.get("is_put", False))))


@dataclass
class PinnNet:
    """A tanh network (tau, S/K[, sigma, r]) -> V/K with flat float32 params on the GPU."""
    params: torch.Tensor
    n_in: int = 2
    depth: int = 4
    width: int = 64
    precision: int = PREC_FP32

    def c(self) -> _Net:
        return _Net(self.n_in, self.depth, self.width, self.precision,
                    _dev(self.params, torch.float32, "net.params"))

    @staticmethod
    def n_params(n_in: int, depth: int, width: int) -> int:
        return width * n_in + width + (depth - 1) * (width * width + width) + width + 1


def bs_initial(p: dict, M: int, payoff_mode: int = 1, out: torch.Tensor | None = None):
    out = torch.empty(M, dtype=torch.float64, device="cuda") if out is None else out
    _check(load_library().bs_initial(ctypes.byref(_params(p)), ctypes.byref(_Grid(M, payoff_mode)),
                                     _dev(out, torch.float64, "out"), _stream()))
    return out


def _propagate(fn, p, M, tau0, dtau, steps, u_in, u_out):
    nsys = u_in.shape[0] if u_in.dim() == 2 else 1
    if u_out is None:
        u_out = torch.empty_like(u_in)
    if u_in.numel() != nsys * M or u_out.numel() != nsys * M or tau0.numel() != nsys:
        raise ValueError("shape mismatch: u_in/u_out must be [nsys, M], tau0 [nsys]")
    _check(fn(ctypes.byref(_params(p)), ctypes.byref(_Grid(M, 1)), nsys,
              _dev(tau0, torch.float64, "tau0"), float(dtau), int(steps),
              _dev(u_in, torch.float64, "u_in"), _dev(u_out, torch.float64, "u_out"), _stream()))
    return u_out


def bs_fine_propagate_batch(p, M, tau0, dtau, steps, u_in, u_out=None):
    """F: `steps` Crank-Nicolson steps on each row of u_in [nsys, M] from tau0[s]."""
    return _propagate(load_library().bs_fine_propagate_batch, p, M, tau0, dtau, steps, u_in, u_out)


def bs_coarse_numeric(p, M, tau0, dtau, steps, u_in, u_out=None):
    """Numerical G: `steps` implicit-Euler steps on each row of u_in."""
    return _propagate(load_library().bs_coarse_numeric, p, M, tau0, dtau, steps, u_in, u_out)


def pinn_forward(net: PinnNet, X: torch.Tensor, out: torch.Tensor | None = None):
    n = X.shape[0]
    out = torch.empty(n, dtype=torch.float32, device="cuda") if out is None else out
    _check(load_library().pinn_forward(ctypes.byref(net.c()), n, _dev(X, torch.float32, "X"),
                                       _dev(out, torch.float32, "out"), _stream()))
    return out


def pinn_residual_workspace_size(net: PinnNet, n_f: int, n_e: int, n_b: int) -> int:
    b = ctypes.c_size_t()
    _check(load_library().pinn_residual_workspace_size(ctypes.byref(net.c()), n_f, n_e, n_b,
                                                       ctypes.byref(b)))
    return b.value


def pinn_residual_fwd_bwd(net: PinnNet, p: dict, X_f, X_e, X_b, ws=None, loss3=None, grad=None,
                          y_e=None, y_b=None):
    """(loss3 [3] = MSE_f, MSE_exp, MSE_b; grad [n_params]) on the GPU.  y_e / y_b:
    value targets of the terminal / boundary sets (None: eqs. (2)-(4))."""
    n_f, n_e, n_b = X_f.shape[0], X_e.shape[0], X_b.shape[0]
    need = pinn_residual_workspace_size(net, n_f, n_e, n_b)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    loss3 = torch.empty(3, dtype=torch.float32, device="cuda") if loss3 is None else loss3
    grad = torch.empty_like(net.params) if grad is None else grad
    ptr = lambda t: _dev(t, torch.float32, "X") if t.shape[0] else None  # noqa: E731

    def target(y, n, name):
        if y is None or n == 0:
            return None
        if y.numel() != n:
            raise ValueError(f"{name} must hold one target per point")
        return _dev(y, torch.float32, name)
    _check(load_library().pinn_residual_fwd_bwd(
        ctypes.byref(net.c()), ctypes.byref(_params(p)), n_f, ptr(X_f), n_e, ptr(X_e),
        target(y_e, n_e, "y_e"), n_b, ptr(X_b), target(y_b, n_b, "y_b"),
        _dev(loss3, torch.float32, "loss3"), _dev(grad, torch.float32, "grad"),
        ws.data_ptr(), ws.numel(), _stream()))
    return loss3, grad


class Parareal:
    """One Parareal problem: option `p`, grid M, N slices; owns its workspace and U."""

    def __init__(self, p: dict, M: int, N: int, fine_steps: int, coarse_steps: int = 1,
                 coarse_kind: int = COARSE_IE, net: PinnNet | None = None, payoff_mode: int = 1):
        self.p, self.M, self.N = dict(p), M, N
        self.kind, self.net = coarse_kind, net
        self._p = _params(p)
        self._g = _Grid(M, payoff_mode)
        self._s = _Slices(N, fine_steps, coarse_steps)
        lib = load_library()
        b = ctypes.c_size_t()
        _check(lib.parareal_workspace_size(ctypes.byref(self._g), ctypes.byref(self._s),
                                           coarse_kind, ctypes.byref(b)))
        self.ws_bytes = b.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.U = torch.empty((N + 1, M), dtype=torch.float64, device="cuda")

    def _net(self):
        return ctypes.byref(self.net.c()) if self.net is not None else None

    def start(self):
        _check(load_library().parareal_start(
            ctypes.byref(self._p), ctypes.byref(self._g), ctypes.byref(self._s), self.kind,
            self._net(), self.ws.data_ptr(), self.ws_bytes, self.U.data_ptr(), _stream()))
        return self.U

    def iterate(self, k: int):
        d, bad = ctypes.c_double(), ctypes.c_int()
        _check(load_library().parareal_iterate(
            ctypes.byref(self._p), ctypes.byref(self._g), ctypes.byref(self._s), self.kind,
            self._net(), self.ws.data_ptr(), self.ws_bytes, self.U.data_ptr(), int(k),
            ctypes.byref(d), ctypes.byref(bad), _stream()))
        return d.value

    def solve(self, tol: float, max_iter: int | None = None):
        """Returns (iters, defects list, status) with U holding the solution."""
        max_iter = self.N if max_iter is None else max_iter
        it = ctypes.c_int()
        hist = (ctypes.c_double * max_iter)()
        rc = _check(load_library().parareal_solve(
            ctypes.byref(self._p), ctypes.byref(self._g), ctypes.byref(self._s), self.kind,
            float(tol), self._net(), int(max_iter), self.ws.data_ptr(), self.ws_bytes,
            self.U.data_ptr(), ctypes.byref(it), hist, _stream()))
        return it.value, list(hist)[: it.value], rc


def bs_tune_set_shape(kernel: int, M_lo: int, M_hi: int, threads: int, nodes_per_thread: int):
    """Use (threads, nodes_per_thread) blocks for M in [M_lo, M_hi]; kernel 0 = F/G batch, 1 = sweep."""
    _check(load_library().bs_tune_set_shape(kernel, M_lo, M_hi, threads, nodes_per_thread))


def bs_tune_reset():
    _check(load_library().bs_tune_reset())


def bs_set_divergence_growth(growth: float = BS_DIVERGENCE_GROWTH):
    """Divergence guard of the solves: stop with BS_ERR_DIVERGED once an
    iteration's defect exceeds `growth` x the first one (process-wide)."""
    _check(load_library().bs_set_divergence_growth(float(growth)))


def bs_divergence_growth() -> float:
    return load_library().bs_divergence_growth()


def bs_release_resources():
    """Free the library's per-thread pinned buffers, streams and tables."""
    _check(load_library().bs_release_resources())


def bs_profile_enable(on: bool = True):
    _check(load_library().bs_profile_enable(int(bool(on))))


def bs_profile_read() -> dict:
    out = (ctypes.c_double * 8)()
    _check(load_library().bs_profile_read(out))
    return {"fine_ms": out[0], "fine_launches": int(out[1]), "fine_cells": out[2],
            "sweep_ms": out[3], "sweep_launches": int(out[4]), "solve_ms": out[5],
            "solve_launches": int(out[6]), "solve_cells": out[7]}


def parareal_solve_noalloc(p: dict, M: int, N: int, fine_steps: int, coarse_steps: int = 1,
                           coarse_kind: int = COARSE_IE, tol: float = 1e-8,
                           net: PinnNet | None = None, max_iter: int | None = None,
                           payoff_mode: int = 1, U: torch.Tensor | None = None):
    """parareal_solve without a workspace (the library's fixed device scratch
    array).  U: caller's [N+1, M] float64 CUDA tensor (allocated here if
    None).  Returns (U, iters, defects, status)."""
    if U is None:
        U = torch.empty((N + 1, M), dtype=torch.float64, device="cuda")
    if U.numel() != (N + 1) * M:
        raise ValueError("U must hold (N+1)*M values")
    max_iter = N if max_iter is None else max_iter
    it = ctypes.c_int()
    hist = (ctypes.c_double * max_iter)()
    rc = _check(load_library().parareal_solve_noalloc(
        ctypes.byref(_params(p)), ctypes.byref(_Grid(M, payoff_mode)),
        ctypes.byref(_Slices(N, fine_steps, coarse_steps)), coarse_kind, float(tol),
        ctypes.byref(net.c()) if net is not None else None, int(max_iter),
        _dev(U, torch.float64, "U"), ctypes.byref(it), hist, _stream()))
    return U, it.value, list(hist)[: it.value], rc


def parareal_solve(p: dict, M: int, N: int, fine_steps: int, coarse_steps: int = 1,
                   coarse_kind: int = COARSE_IE, tol: float = 1e-8, net: PinnNet | None = None,
                   max_iter: int | None = None, payoff_mode: int = 1):
    """Convenience wrapper: returns (U [N+1, M] cuda float64, iters, defects)."""
    pr = Parareal(p, M, N, fine_steps, coarse_steps, coarse_kind, net, payoff_mode)
    iters, defects, _ = pr.solve(tol, max_iter)
    return pr.U, iters, defects


def parareal_solve_batch(options, coarse_kind: int = COARSE_IE, tol: float = 1e-8,
                         net: PinnNet | None = None, max_iter: int | None = None,
                         payoff_mode: int = 1, lookahead: int = 0):
    """Solve many options together.  `options`: dicts with K, r, sigma, T, s_max,
    is_put, M, N, fine_steps, coarse_steps.  Returns (U_packed [cuda float64],
    offsets, iters, defects, status); option o's state is
    U_packed[offsets[o]: offsets[o] + (N+1)*M].reshape(N+1, M)."""
    n = len(options)
    Pa = (_Params * n)(*[_params(o) for o in options])
    Ga = (_Grid * n)(*[_Grid(o["M"], payoff_mode) for o in options])
    Sa = (_Slices * n)(*[_Slices(o["N"], o["fine_steps"], o.get("coarse_steps", 1))
                         for o in options])
    offs, tot = [], 0
    for o in options:
        offs.append(tot)
        tot += (o["N"] + 1) * o["M"]
    Oa = (ctypes.c_long * n)(*offs)
    lib = load_library()
    b = ctypes.c_size_t()
    _check(lib.parareal_batch_workspace_size(n, Pa, Ga, Sa, coarse_kind, ctypes.byref(b)))
    wsb = b.value
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    U = torch.empty(tot, dtype=torch.float64, device="cuda")
    it = (ctypes.c_int * n)()
    de = (ctypes.c_double * n)()
    if max_iter is None:
        max_iter = max(o["N"] for o in options)
    rc = _check(lib.parareal_solve_batch(
        n, Pa, Ga, Sa, coarse_kind, float(tol), ctypes.byref(net.c()) if net is not None else None,
        int(max_iter), ws.data_ptr(), wsb, U.data_ptr(), Oa, it, de, int(lookahead),
        _stream()))
    return U, offs, list(it), list(de), rc
