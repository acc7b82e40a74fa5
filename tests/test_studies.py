"""Host logic of the studies (bench_studies.py): the speedup bound of
eq. (8), the fixed-work split of the N-sweep and iteration counting."""
import math

import pytest

from bench_studies import eq8_bound, iterations_to, nsweep_splits


def test_eq8_bound_limits():
    # free coarse propagator: the bound is N / K
    assert eq8_bound(3, 48, 0.0, 1.0) == pytest.approx(16.0)
    # K = N with free coarse: no speedup
    assert eq8_bound(8, 8, 0.0, 1.0) == pytest.approx(1.0)
    # coarse as expensive as fine: 1 / (1 + 2 K / N)
    assert eq8_bound(2, 8, 1.0, 1.0) == pytest.approx(1.0 / (1.25 + 0.25))
    # grows with N towards c_f / c_c
    vals = [eq8_bound(4, N, 1e-3, 1.0) for N in (8, 64, 512, 4096, 1 << 20)]
    assert all(a < b for a, b in zip(vals, vals[1:]))
    assert vals[-1] == pytest.approx(1e3, rel=1e-2)


def test_nsweep_splits_keep_total_work():
    total = 256 * 2048
    splits = nsweep_splits(total, [1, 2, 3, 4, 64, 256, 1000])
    assert [N for N, _ in splits] == [2, 4, 64, 256]
    assert all(N * s == total for N, s in splits)


def test_iterations_to():
    d = [1.0, 1e-3, 1e-9, 1e-11]
    assert iterations_to(d, 1e-8) == 3
    assert iterations_to(d, 1e-10) == 4
    assert iterations_to(d, 1e-12) is None
    assert iterations_to([], 1.0) is None
    assert not math.isnan(eq8_bound(1, 2, 0.5, 1.0))
