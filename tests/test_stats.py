"""Repeat statistics (Sec. II.B) on synthetic traces with known answers."""
import numpy as np
import pytest

from paper_1703_01545_amd import stats


def test_mean_and_se_definition():
    x = np.array([[1.0, 2.0], [3.0, 6.0], [5.0, 10.0]])
    m, se = stats.per_time(x)
    assert np.allclose(m, [3.0, 6.0])
    # std with N - 1 over sqrt(N): sqrt(4) / sqrt(3) and sqrt(16) / sqrt(3)
    assert np.allclose(se, [2.0 / np.sqrt(3), 4.0 / np.sqrt(3)])
    with pytest.raises(ValueError):
        stats.mean_and_se(np.ones((1, 3)))


def test_cumulative_averages_after_equilibration():
    tr = np.array([[9.0, 9.0, 1.0, 2.0, 3.0], [9.0, 9.0, 3.0, 4.0, 5.0]])
    c = stats.cumulative_averages(tr, 2)
    assert np.allclose(c, [[1.0, 1.5, 2.0], [3.0, 3.5, 4.0]])
    with pytest.raises(ValueError):
        stats.cumulative_averages(tr, 5)


def test_final_estimate_earliest_minimum_and_target():
    # repeats that agree more and more, then spread again: the minimum of the
    # standard error of the cumulative averages is taken, the earliest of ties
    rng = np.random.default_rng(0)
    base = rng.standard_normal((11, 1))
    tr = np.concatenate([base * 5, base * 0 + 1.0, base * 0 + 1.0, base * 0 + 1.0], axis=1)
    tr[:, 0] += 100.0  # equilibration segment, excluded
    est = stats.final_estimate(tr, 1)
    assert est.j == 1 and est.se == 0.0 and est.value == 1.0 and not est.reached_target
    noisy = rng.standard_normal((11, 50)) * 0.1 + 2.0
    e1 = stats.final_estimate(noisy, 0, target=0.05)
    assert e1.reached_target and e1.se < 0.05
    # before the returned index no cumulative-average error was below target
    m, se = stats.mean_and_se(stats.cumulative_averages(noisy, 0), axis=0)
    assert np.all(se[: e1.j] >= 0.05)
    assert stats.first_below(se, 0.05) == e1.j


def test_reblocking_recovers_the_error_of_an_ar1_series():
    """x_t = rho x_{t-1} + e_t, e ~ N(0, 1): the variance of the mean of n
    values tends to 1 / (n (1 - rho)^2); the naive error underestimates it
    by sqrt((1 + rho) / (1 - rho)) = 3 at rho = 0.8."""
    rho, n = 0.8, 2 ** 17
    rng = np.random.default_rng(5)
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0] / np.sqrt(1 - rho ** 2)
    for t in range(1, n):
        x[t] = rho * x[t - 1] + e[t]
    rb = stats.reblock(x)
    exact = 1.0 / (np.sqrt(n) * (1 - rho))
    assert rb.level > 0
    assert abs(rb.value - exact) < 0.15 * exact
    assert rb.se[0] < 0.5 * exact  # the unblocked error is far too small
    # uncorrelated data: the plateau starts at once
    white = stats.reblock(rng.standard_normal(n))
    assert abs(white.value - 1 / np.sqrt(n)) < 0.1 / np.sqrt(n)


def test_speedup_is_ratio_of_walkers_times_time():
    # the K-atom figures of Sec. III.C: 1056 walkers to tau = 10 against 24 to tau = 7
    assert abs(stats.speedup(1056, 10.0, 24, 7.0) - 62.857) < 1e-3
