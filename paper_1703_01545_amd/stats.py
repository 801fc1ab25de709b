"""Repeat statistics of correlated-sampling energy differences (Sec. II.B).

The protocol: a correlated pair is propagated N_r times with different
random-number seeds.  At every measured imaginary time the mean of the energy
difference over the repeats and its standard error (the standard deviation
over the repeats divided by sqrt(N_r)) are formed.  After an equilibration
time chosen where the difference has stabilised, each repeat's measurements
are averaged cumulatively (the running average of the measurements taken
after the equilibration up to each time); the final estimate is the mean of
these cumulative averages over the repeats, with their standard error, at the
time where that error reaches its minimum (the earliest of equal minima) or
first falls below a target.  A single long run's standard error is corrected
for autocorrelation by reblocking (Flyvbjerg and Petersen, J. Chem. Phys. 91,
461 (1989)).  The cost of reaching a target error is proportional to the
number of walkers times the propagation time (Sec. III.C), which gives the
speed-up of correlated over uncorrelated sampling.

Host-side arithmetic on energy traces only (numpy); the traces come from the
library's GPU path (``repeats.py``).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np


def mean_and_se(samples: np.ndarray, axis: int = 0):
    """Mean and standard error (std with N - 1 over sqrt(N)) along `axis`."""
    x = np.asarray(samples, dtype=np.float64)
    n = x.shape[axis]
    if n < 2:
        raise ValueError("a standard error needs at least two repeats")
    return x.mean(axis=axis), x.std(axis=axis, ddof=1) / np.sqrt(n)


def per_time(traces: np.ndarray):
    """traces[r, j] (repeat r, measurement j) -> mean and standard error over
    the repeats at every measurement."""
    return mean_and_se(traces, axis=0)


def cumulative_averages(traces: np.ndarray, j_eq: int) -> np.ndarray:
    """Running average of each repeat's measurements j_eq..j, for j >= j_eq;
    shape (N_r, n_meas - j_eq)."""
    x = np.asarray(traces, dtype=np.float64)[:, j_eq:]
    if x.shape[1] == 0:
        raise ValueError("equilibration index at or past the last measurement")
    return np.cumsum(x, axis=1) / np.arange(1, x.shape[1] + 1)[None, :]


@dataclass
class Estimate:
    value: float        # mean of the cumulative averages over the repeats
    se: float           # its standard error
    j: int              # measurement index at which it is taken
    reached_target: bool


def final_estimate(traces: np.ndarray, j_eq: int, target: Optional[float] = None) -> Estimate:
    """The estimate at the first measurement where the standard error of the
    cumulative averages falls below `target`, else at the earliest minimum of
    that error."""
    cum = cumulative_averages(traces, j_eq)
    m, se = mean_and_se(cum, axis=0)
    if target is not None:
        below = np.nonzero(se < target)[0]
        if below.size:
            k = int(below[0])
            return Estimate(float(m[k]), float(se[k]), j_eq + k, True)
    k = int(np.argmin(se))  # argmin returns the earliest of equal minima
    return Estimate(float(m[k]), float(se[k]), j_eq + k, False)


def first_below(se_curve: np.ndarray, target: float) -> Optional[int]:
    """Index of the first entry of a standard-error curve below target."""
    idx = np.nonzero(np.asarray(se_curve) < target)[0]
    return int(idx[0]) if idx.size else None


@dataclass
class Reblocking:
    se: np.ndarray       # standard error of the mean at each blocking level
    se_err: np.ndarray   # its own statistical error
    n_blocks: np.ndarray
    level: int           # chosen level (start of the plateau)

    @property
    def value(self) -> float:
        return float(self.se[self.level])


def reblock(x: Sequence[float], min_blocks: int = 16) -> Reblocking:
    """Flyvbjerg-Petersen blocking of a correlated series: at each level
    neighbouring values are averaged in pairs; the naive standard error of
    the mean grows with the level until the blocks are longer than the
    autocorrelation time and then stays constant.  The chosen level is the
    first whose estimate plus its error bar is not exceeded by any later
    level's estimate (the start of the plateau)."""
    y = np.asarray(x, dtype=np.float64)
    se, err, nb = [], [], []
    while y.size >= min_blocks:
        n = y.size
        v = np.var(y)  # population variance of the block means
        s = np.sqrt(v / (n - 1))
        se.append(s)
        err.append(s / np.sqrt(2.0 * (n - 1)))
        nb.append(n)
        y = 0.5 * (y[: n // 2 * 2: 2] + y[1: n // 2 * 2: 2])
    if not se:
        raise ValueError("series too short to reblock")
    se_a, err_a = np.array(se), np.array(err)
    level = len(se_a) - 1
    for lv in range(len(se_a)):
        if np.all(se_a[lv + 1:] <= se_a[lv] + err_a[lv]):
            level = lv
            break
    return Reblocking(se_a, err_a, np.array(nb), level)


def speedup(walkers_uncorrelated: int, tau_uncorrelated: float, walkers_correlated: int,
            tau_correlated: float) -> float:
    """CPU-time ratio of two ways of reaching the same target error: the cost
    of a run is proportional to walkers x propagation time (Sec. III.C)."""
    return (walkers_uncorrelated * tau_uncorrelated) / (walkers_correlated * tau_correlated)
