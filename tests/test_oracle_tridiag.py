"""Oracle Thomas solver against LAPACK's banded solver (scipy.linalg.solve_banded)
and a dense solve, on random strictly diagonally dominant systems."""
import numpy as np
import pytest
import scipy.linalg

import oracle


@pytest.mark.parametrize("n", [1, 2, 3, 17, 256, 1000])
def test_thomas_vs_banded(n):
    rng = np.random.default_rng(n)
    a = rng.uniform(-1, 1, n)
    c = rng.uniform(-1, 1, n)
    b = np.abs(a) + np.abs(c) + rng.uniform(0.5, 2.0, n)
    b *= rng.choice([-1.0, 1.0], n)
    d = rng.normal(size=n)
    x = oracle.thomas(a, b, c, d)
    ab = np.zeros((3, n))
    ab[0, 1:] = c[:-1]
    ab[1] = b
    ab[2, :-1] = a[1:]
    ref = scipy.linalg.solve_banded((1, 1), ab, d)
    assert np.max(np.abs(x - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    A = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    assert np.max(np.abs(A @ x - d)) <= 1e-12 * max(1.0, np.max(np.abs(d)))
