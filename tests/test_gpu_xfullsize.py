"""Full-size parity: the workloads exactly as configured, on the GPU, against
the FP64 oracle's serial fine solution (the fixed point of eq. (7), Sec. 3.1).

Bar: normwise max |U_gpu - U_fine| / max |U_fine| <= 1e-10 over every time
level n = 0..N and node.  A converged Parareal iterate differs from the
fixed point by about the last defect or less (the iteration contracts fast
near convergence: measured with the oracle at 0.1-0.3 x the last defect),
so at tol 1e-8 (price units; solutions of 50..400) the gap is ~1e-11 and at
tol 1e-10 ~1e-13, well inside the bar; rounding adds ~1e-12 (propagator
tests).  The 16384-node put's serial fine solution takes about 20 minutes
of one CPU core (257 levels of 2048 CN steps, each level needing the one
before), so the oracle's values at 12 levels are stored
(tests/golden/large_put_reference.py writes them); the 512 options' serial
fine solutions take minutes of CPU time in all and run in background
processes started when the tests are collected (tests/oracle_jobs.py).

* The 16384-node put (256 slices, 2048 CN steps per slice, tol 1e-10) with
  the 6 x 256 network coarse in BF16 (seeded weights) and with the numerical
  coarse.
* The 1024-node call (32 slices, 512 CN steps per slice, tol 1e-8) with a
  TRAINED 4 x 64 network (weights trained by the oracle alone,
  tests/golden/train_call_network.py) evaluated in BF16 and FP32: the
  solution against serial fine, the iteration count against the oracle's
  Parareal on its own FP64 network grid of the same weights (within one),
  and the network's own error against serial fine reported per precision.
* All 512 options of the batched workload (numerical and network coarse),
  every option against its serial fine solution; the numerical coarse's
  iteration counts against the oracle's Parareal on sampled options.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2303_03848_amd as bsp
from oracle import mlp
from tests.gpu_util import cuda, network_grid, normwise, say, to_dev
from tests.oracle_jobs import oracle_result
from workloads import (LARGE_PUT, OPTION_BATCH, PINN_CALL, option_batch, option_params,
                       perturbed, xavier_normal)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _large_put_reference():
    path = os.path.join(GOLDEN, "large_put_levels.npz")
    if not os.path.exists(path):
        pytest.skip("fixture tests/golden/large_put_levels.npz not written yet "
                    "(python -m tests.golden.large_put_reference)")
    with np.load(path) as z:
        return z["levels"], z["U"]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("kind", [bsp.COARSE_PINN_IE, bsp.COARSE_IE])
def test_large_put_full_size(kind):
    cuda()
    levels, ref = _large_put_reference()
    cfg = LARGE_PUT
    M, N, Sf = cfg["M"], cfg["N"], cfg["fine_steps"]
    net = None
    if kind == bsp.COARSE_PINN_IE:
        th = perturbed(xavier_normal(2, cfg["depth"], cfg["width"], seed=7), 0.02, 8)
        net = bsp.PinnNet(to_dev(th, torch.float32), 2, cfg["depth"], cfg["width"], bsp.PREC_BF16)
    say(f"large put full size, kind {kind}: M={M} N={N} Sf={Sf} tol={cfg['tol']}")
    U, iters, defects = bsp.parareal_solve(option_params(cfg), M, N, Sf, 1, kind,
                                           tol=cfg["tol"], net=net)
    U = U.cpu().numpy()
    say(f"large put: {iters} iterations, last defect {defects[-1]:.2e}")
    assert ref.shape == (len(levels), M)
    got = U[levels]
    per_level = np.max(np.abs(got - ref), axis=1) / np.max(np.abs(ref))
    err = float(per_level.max())
    say(f"large put: normwise error vs serial fine {err:.3e} at levels {levels.tolist()} "
        f"(worst level {int(levels[per_level.argmax()])})")
    assert np.array_equal(got[0], ref[0])
    assert err <= 1e-10


def _golden_call_net():
    path = os.path.join(GOLDEN, "pinn_call_4x64.npy")
    if not os.path.exists(path):
        pytest.skip("trained fixture tests/golden/pinn_call_4x64.npy not written yet "
                    "(python -m tests.golden.train_call_network)")
    return np.load(path)


@pytest.mark.parametrize("prec", [bsp.PREC_BF16, bsp.PREC_FP32])
def test_call_trained_network(prec):
    cuda()
    cfg = PINN_CALL
    M, N, Sf, tol = cfg["M"], cfg["N"], cfg["fine_steps"], cfg["tol"]
    th = _golden_call_net()
    po = oracle.params_from(option_params(cfg))
    ser = oracle.serial_fine(po, M, N, Sf)
    S = oracle.grid(po, M)
    taus = np.arange(N + 1) * (po.T / N)
    Vt = mlp.grid_values(th.astype(np.float64), 2, cfg["depth"], cfg["width"], po.K, taus, S)
    net = bsp.PinnNet(to_dev(th, torch.float32), 2, cfg["depth"], cfg["width"], prec)
    U, iters, defects = bsp.parareal_solve(option_params(cfg), M, N, Sf, 1, bsp.COARSE_PINN_IE,
                                           tol=tol, net=net)
    U = U.cpu().numpy()
    ref = oracle.parareal(po, M, N, Sf, 1, oracle.COARSE_PINN_IE, Vt=Vt, tol=tol, nthreads=8)
    ie = oracle.parareal(po, M, N, Sf, 1, oracle.COARSE_IE, tol=tol, nthreads=8)
    # the network's own error on the Parareal grid, price units (levels n >= 1)
    vt_gpu = network_grid(bsp, net, option_params(cfg), M, N) * po.K
    err_gpu = float(np.max(np.abs(vt_gpu[1:] - ser[1:])))
    err_ora = float(np.max(np.abs(Vt[1:] - ser[1:])))
    name = "bf16" if prec == bsp.PREC_BF16 else "fp32"
    say(f"trained 4x64 network ({name}): gpu {iters} iterations, oracle (fp64 network) "
        f"{ref['iters']}, numeric coarse {ie['iters']}; network max error vs serial fine: "
        f"{name} {err_gpu:.3e}, fp64 {err_ora:.3e} price units")
    assert abs(iters - ref["iters"]) <= 1
    assert normwise(U, ser) <= 1e-10
    assert normwise(ref["U"], ser) <= 1e-10


def _batch_opts():
    cfg = OPTION_BATCH
    return [dict(o, fine_steps=cfg["fine_steps"], coarse_steps=cfg["coarse_steps"])
            for o in option_batch(cfg)]


@pytest.mark.oracle_job("option_batch")
@pytest.mark.timeout(900)
@pytest.mark.parametrize("kind", [bsp.COARSE_IE, bsp.COARSE_PINN_IE])
def test_option_batch_all_options(kind):
    cuda()
    cfg = OPTION_BATCH
    opts = _batch_opts()
    net = None
    if kind != bsp.COARSE_IE:
        th = perturbed(xavier_normal(4, cfg["depth"], cfg["width"], seed=5), 0.02, 6)
        net = bsp.PinnNet(to_dev(th, torch.float32), 4, cfg["depth"], cfg["width"], bsp.PREC_BF16)
    say(f"512-option batch, kind {kind}: all options against serial fine")
    U, offs, iters, defects, rc = bsp.parareal_solve_batch(opts, kind, cfg["tol"], net=net)
    assert rc == bsp.BS_OK
    U = U.cpu().numpy()
    ref = oracle_result("option_batch")
    assert ref.size == U.size
    worst, worst_i = 0.0, -1
    for i, o in enumerate(opts):
        n = (o["N"] + 1) * o["M"]
        got, r = U[offs[i]: offs[i] + n], ref[offs[i]: offs[i] + n]
        e = normwise(got, r)
        if e > worst:
            worst, worst_i = e, i
    say(f"iterations min {min(iters)} max {max(iters)} mean {np.mean(iters):.2f}; worst "
        f"normwise error vs serial fine {worst:.3e} (option {worst_i})")
    assert worst <= 1e-10
    if kind == bsp.COARSE_IE:
        for i in range(0, 512, 64):
            o = opts[i]
            r = oracle.parareal(oracle.params_from(o), o["M"], o["N"], o["fine_steps"], 1,
                                oracle.COARSE_IE, tol=cfg["tol"], nthreads=8)
            assert iters[i] == r["iters"], (i, iters[i], r["iters"])
