"""CPU checks of the simulated cameras' arrival schedule (no GPU)."""
import numpy as np

from paper_2310_09467_amd import cameras


def test_poisson_arrivals_rate_and_gaps():
    ts = cameras.arrivals(50.0, 200.0, seed=7)
    n = len(ts)
    # count ~ Poisson(10000): within 5 sigma
    assert abs(n - 10000) < 5 * np.sqrt(10000)
    gaps = np.diff(np.concatenate([[0.0], ts]))
    assert np.all(gaps > 0) and ts[-1] < 200.0
    # exponential gaps: mean 1/rate, coefficient of variation 1
    assert abs(gaps.mean() - 0.02) < 5 * 0.02 / np.sqrt(n)
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05


def test_schedule_is_ordered_and_reproducible():
    a = cameras.schedule(4, 50.0, 5.0)
    b = cameras.schedule(4, 50.0, 5.0)
    assert a == b
    assert [e[0] for e in a] == sorted(e[0] for e in a)
    cams = {e[1] for e in a}
    assert cams == {0, 1, 2, 3}
    sizes = np.bincount([e[2] for e in a], minlength=3)
    assert np.all(sizes > 0.2 * len(a))
