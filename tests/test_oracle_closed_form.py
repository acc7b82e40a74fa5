"""Oracle against the closed-form Black-Scholes price.

The closed form is itself pinned by direct numerical integration of the
discounted expected payoff under the log-normal law (scipy.integrate.quad)
and by put-call parity.  The fine propagator is then checked against it on
the small call workload: the error is bounded, and shrinks as O(dS^2) under
refinement (cell-averaged payoff).

Reading of the accuracy bound: the error is measured on the scale of the
strike (v = V/K), max |V_fd - V_exact| / K <= 1e-3, and as the normalised
l2 error of the paper's Fig. 3, ||V_fd - V_exact||_2 / ||V_exact||_2 <= 1e-3.
The absolute maximum error at M = 256 is about 1.2e-3, purely spatial and
located out of the money.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
from workloads import SMALL_CALL, option_params


def _price_by_quadrature(S, K, r, sigma, tau, is_put):
    def integrand(z):
        ST = S * np.exp((r - 0.5 * sigma ** 2) * tau + sigma * np.sqrt(tau) * z)
        pay = max(K - ST, 0.0) if is_put else max(ST - K, 0.0)
        return pay * np.exp(-0.5 * z * z) / np.sqrt(2 * np.pi)
    val, _ = integrate.quad(integrand, -12, 12, limit=400, epsabs=1e-13, epsrel=1e-13)
    return np.exp(-r * tau) * val


@pytest.mark.parametrize("S,K,r,sigma,tau", [(100, 100, 0.05, 0.2, 1.0), (70, 100, 0.05, 0.2, 1.0),
                                             (180, 100, 0.03, 0.35, 2.0), (95, 120, 0.0, 0.5, 0.25)])
@pytest.mark.parametrize("is_put", [False, True])
def test_closed_form_vs_quadrature(S, K, r, sigma, tau, is_put):
    got = oracle.bs_price([S], K, r, sigma, tau, is_put)[0]
    ref = _price_by_quadrature(S, K, r, sigma, tau, is_put)
    assert abs(got - ref) <= 1e-9 * max(1.0, ref)


def test_closed_form_put_call_parity_and_limits():
    S = np.linspace(1, 300, 50)
    c = oracle.bs_price(S, 100, 0.05, 0.2, 1.0, False)
    p = oracle.bs_price(S, 100, 0.05, 0.2, 1.0, True)
    assert np.max(np.abs(c - p - (S - 100 * np.exp(-0.05)))) < 1e-11
    assert np.allclose(oracle.bs_price(S, 100, 0.05, 0.2, 0.0), np.maximum(S - 100, 0))


def _serial_final(cfg, M, steps):
    p = oracle.params_from(option_params(cfg))
    U = oracle.serial_fine(p, M, cfg["N"], steps, payoff_mode=1)
    S = oracle.grid(p, M)
    ex = oracle.bs_price(S, p.K, p.r, p.sigma, p.T, bool(p.is_put))
    return U[-1], ex


def test_fine_vs_closed_form_small_call():
    cfg = SMALL_CALL
    V, ex = _serial_final(cfg, cfg["M"], cfg["fine_steps"])
    err = np.abs(V - ex)
    assert err.max() / cfg["K"] <= 1e-3
    assert np.linalg.norm(V - ex) / np.linalg.norm(ex) <= 1e-3
    assert err.max() < 2e-3


def test_fine_second_order_in_space():
    cfg = SMALL_CALL
    errs = []
    for lvl in range(4):
        M = 256 * 2 ** lvl
        V, ex = _serial_final(cfg, M, 64 * 2 ** lvl)
        errs.append(np.abs(V - ex).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for q in ratios:
        assert 3.8 <= q <= 4.2, (errs, ratios)


def test_fine_put_call_parity():
    """C - P solves the discrete problem with initial data S - K (the cell
    average of a linear function is its midpoint value) and boundary data
    S - K exp(-r tau); it equals S - K exp(-r tau) up to the O(dt^2) gap
    between exp(-r dt) and the Crank-Nicolson factor."""
    cfg = dict(SMALL_CALL)
    V_call, _ = _serial_final(cfg, cfg["M"], cfg["fine_steps"])
    cfg["is_put"] = True
    V_put, _ = _serial_final(cfg, cfg["M"], cfg["fine_steps"])
    p = oracle.params_from(option_params(cfg))
    S = oracle.grid(p, cfg["M"])
    gap = np.abs(V_call - V_put - (S - p.K * np.exp(-p.r * p.T)))
    assert gap.max() < 1e-7


def test_put_vs_closed_form():
    cfg = dict(SMALL_CALL, is_put=True)
    V, ex = _serial_final(cfg, cfg["M"], cfg["fine_steps"])
    assert np.abs(V - ex).max() / cfg["K"] <= 1e-3


def test_point_payoff_vs_closed_form():
    cfg = SMALL_CALL
    p = oracle.params_from(option_params(cfg))
    U = oracle.serial_fine(p, cfg["M"], cfg["N"], cfg["fine_steps"], payoff_mode=0)
    S = oracle.grid(p, cfg["M"])
    ex = oracle.bs_price(S, p.K, p.r, p.sigma, p.T)
    assert np.abs(U[-1] - ex).max() / p.K <= 1e-3
    assert np.array_equal(U[0], np.maximum(S - p.K, 0.0))
