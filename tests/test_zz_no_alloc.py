"""parareal_solve_noalloc (the solve without a caller workspace, for callers
that cannot allocate device memory) against parareal_solve, through the C
ABI: same iterates, defects and iteration counts (the same kernels run, so
bitwise), on two calls in a row where the second is smaller (the library's
scratch array keeps the first call's contents), on both of its paths (the
one-launch solve and the iterations one after the other), and the size
limit as an argument error.
"""
import numpy as np
import pytest
import torch

import paper_2303_03848_amd as bsp
from tests.gpu_util import cuda, say, to_dev
from workloads import SMALL_CALL, option_params, perturbed, xavier_normal

pytestmark = pytest.mark.gpu


def _pair(p, M, N, Sf, kind=bsp.COARSE_IE, net=None, tol=1e-8):
    say(f"no-alloc vs parareal_solve: M={M} N={N} Sf={Sf} kind={kind}")
    U0, it0, d0 = bsp.parareal_solve(p, M, N, Sf, 1, kind, tol=tol, net=net)
    U1, it1, d1, rc = bsp.parareal_solve_noalloc(p, M, N, Sf, 1, kind, tol=tol, net=net)
    torch.cuda.synchronize()
    assert rc in (bsp.BS_OK, bsp.BS_NOT_CONVERGED)
    assert it1 == it0, (it1, it0)
    assert d1 == d0
    assert torch.equal(U1, U0)
    return it1


@pytest.mark.parametrize("sizes", [((1024, 32, 64), (256, 8, 16)),    # one-launch solve
                                   ((2048, 16, 32), (1500, 8, 24))])  # one iteration at a time
def test_noalloc_matches_solve_twice(sizes):
    cuda()
    p = option_params(SMALL_CALL)
    for M, N, Sf in sizes:
        it = _pair(p, M, N, Sf)
        assert it >= 2


def test_noalloc_network_coarse():
    cuda()
    p = option_params(SMALL_CALL)
    th = perturbed(xavier_normal(2, 2, 16, seed=1), 0.05, 2)
    net = bsp.PinnNet(to_dev(th, torch.float32), 2, 2, 16, bsp.PREC_FP32)
    _pair(p, 512, 16, 32, bsp.COARSE_PINN_IE, net)
    _pair(p, 3000, 8, 16, bsp.COARSE_PINN_IE, net)


def test_noalloc_size_limits():
    cuda()
    p = option_params(SMALL_CALL)
    for M, N in ((4097, 4), (4096, 200), (64, 513)):
        with pytest.raises(bsp.BsError) as e:
            bsp.parareal_solve_noalloc(p, M, N, 4, 1, bsp.COARSE_IE, tol=1e-8)
        assert e.value.code == bsp.BS_ERR_ARG
    # a valid call afterwards is unaffected
    _pair(p, 256, 8, 16)
