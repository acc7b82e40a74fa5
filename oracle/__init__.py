"""Plain FP64 CPU oracle for Parareal on the Black-Scholes equation.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The HIP library never
calls it, and it never calls the HIP library; the two share no code.

* ``bs_oracle.c`` (built into ``libbsoracle.so`` by :func:`build`) holds the
  mesh, payoff, boundary data, Thomas solver, theta-method propagators,
  serial fine integration, Parareal and the closed-form price.
* ``mlp.py`` holds the network, its input-derivative streams, the PINN loss
  and its hand-written gradient, in numpy float64.
* ``flowmap.py`` holds Parareal with a flow-map network coarse (the network
  sees the state), in plain Python loops over the C oracle's fine propagator.

Parity status of each function is recorded in the module docstrings and in
the tests that pin it (``tests/test_oracle_*.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bs_oracle.c")
_LIB = os.path.join(_HERE, "libbsoracle.so")

COARSE_IE, COARSE_PINN, COARSE_PINN_IE, COARSE_CN = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile bs_oracle.c with gcc: -O2, no FMA contraction, OpenMP."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("K", ctypes.c_double), ("r", ctypes.c_double), ("sigma", ctypes.c_double),
                ("T", ctypes.c_double), ("s_max", ctypes.c_double), ("is_put", ctypes.c_int)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Params)
        i, d = ctypes.c_int, ctypes.c_double
        sig = {
            "or_initial": (None, [P, i, i, _dp]),
            "or_boundary": (None, [P, d, _dp, _dp]),
            "or_thomas": (None, [i, _dp, _dp, _dp, _dp, _dp, _dp]),
            "or_propagate": (None, [P, i, d, d, d, i, _dp, _dp]),
            "or_propagate_bc": (None, [P, i, d, d, i, _dp, _dp, _dp, _dp]),
            "or_fine": (None, [P, i, d, d, i, _dp, _dp]),
            "or_coarse_ie": (None, [P, i, d, d, i, _dp, _dp]),
            "or_serial_fine": (None, [P, i, i, i, _dp]),
            "or_parareal": (i, [P, i, i, i, i, i, i, _dp, d, i, i, _dp,
                                ctypes.POINTER(ctypes.c_int), _dp, _dp]),
            "or_bs_price": (d, [d, d, d, d, d, i]),
            "or_max_threads": (i, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def params(K, r, sigma, T, s_max, is_put=False) -> _Params:
    return _Params(float(K), float(r), float(sigma), float(T), float(s_max), int(bool(is_put)))


def params_from(d: dict) -> _Params:
    return params(d["K"], d["r"], d["sigma"], d["T"], d["s_max"], d.get("is_put", False))


def grid(p: _Params, M: int) -> np.ndarray:
    """Interior nodes S_j = j dS, j = 1..M, dS = S_max/(M+1)."""
    dS = p.s_max / (M + 1)
    return np.arange(1, M + 1, dtype=np.float64) * dS


def initial(p, M, payoff_mode=1):
    u = np.empty(M)
    _load().or_initial(ctypes.byref(p), M, payoff_mode, _ptr(u))
    return u


def boundary(p, tau):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _load().or_boundary(ctypes.byref(p), float(tau), ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def thomas(a, b, c, d):
    a, b, c, d = map(_f64, (a, b, c, d))
    n = len(b)
    x, cp = np.empty(n), np.empty(n)
    _load().or_thomas(n, _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(x), _ptr(cp))
    return x


def propagate(p, M, theta, tau0, dtau, steps, u):
    u = _f64(u)
    out = np.empty(M)
    _load().or_propagate(ctypes.byref(p), M, float(theta), float(tau0), float(dtau), int(steps),
                         _ptr(u), _ptr(out))
    return out


def propagate_bc(p, M, theta, dt, steps, g_lo, g_hi, u):
    u, g_lo, g_hi = _f64(u), _f64(g_lo), _f64(g_hi)
    assert len(g_lo) == steps + 1 and len(g_hi) == steps + 1
    out = np.empty(M)
    _load().or_propagate_bc(ctypes.byref(p), M, float(theta), float(dt), int(steps), _ptr(g_lo),
                            _ptr(g_hi), _ptr(u), _ptr(out))
    return out


def fine(p, M, tau0, dtau, steps, u):
    """F: `steps` Crank-Nicolson steps from tau0 over dtau."""
    u = _f64(u)
    out = np.empty(M)
    _load().or_fine(ctypes.byref(p), M, float(tau0), float(dtau), int(steps), _ptr(u), _ptr(out))
    return out


def coarse_ie(p, M, tau0, dtau, steps, u):
    """Numerical G: `steps` implicit-Euler steps from tau0 over dtau."""
    u = _f64(u)
    out = np.empty(M)
    _load().or_coarse_ie(ctypes.byref(p), M, float(tau0), float(dtau), int(steps), _ptr(u),
                         _ptr(out))
    return out


def serial_fine(p, M, N, fine_steps, payoff_mode=1, U0=None):
    """U_{n+1} = F(U_n), n = 0..N-1; returns (N+1, M)."""
    U = np.empty((N + 1, M))
    U[0] = initial(p, M, payoff_mode) if U0 is None else _f64(U0)
    _load().or_serial_fine(ctypes.byref(p), M, N, fine_steps, _ptr(U))
    return U


def parareal(p, M, N, fine_steps, coarse_steps=1, coarse_kind=COARSE_IE, Vt=None, tol=1e-8,
             max_iter=None, payoff_mode=1, nthreads=None, keep_iterates=False):
    """Parareal in plain loops.  Returns dict(U, iters, defects, status[, iterates])."""
    if max_iter is None:
        max_iter = N
    if nthreads is None:
        nthreads = 1
    if coarse_kind in (COARSE_PINN, COARSE_PINN_IE):
        Vt = _f64(Vt)
        assert Vt.shape == (N + 1, M)
    else:
        Vt = None
    U = np.empty((N + 1, M))
    defects = np.full(max(max_iter, 1), np.nan)
    it = ctypes.c_int(0)
    iterates = np.empty((max_iter + 1, N + 1, M)) if keep_iterates else None
    st = _load().or_parareal(ctypes.byref(p), M, payoff_mode, N, fine_steps, coarse_steps,
                             coarse_kind, _ptr(Vt), float(tol), int(max_iter), int(nthreads),
                             _ptr(U), ctypes.byref(it), _ptr(defects), _ptr(iterates))
    out = {"U": U, "iters": it.value, "defects": defects[: it.value], "status": st}
    if keep_iterates:
        out["iterates"] = iterates[: it.value + 1]
    return out


def bs_price(S, K, r, sigma, tau, is_put=False):
    """Closed-form European price (scalar or array S)."""
    lib = _load()
    S = np.atleast_1d(np.asarray(S, dtype=np.float64))
    out = np.array([lib.or_bs_price(float(s), float(K), float(r), float(sigma), float(tau),
                                    int(bool(is_put))) for s in S])
    return out


def max_threads() -> int:
    return _load().or_max_threads()
