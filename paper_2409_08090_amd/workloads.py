"""Seeded synthetic light curves shaped like the nifty-ls paper's workloads.

The paper times FP64 series with N_d in [1e2, 1e6] and N_f ~ 12 N_d frequencies
(Sec. 2) but does not supply its data, so these generators stand in for it.
This module draws random inputs only; it holds none of the periodogram's
arithmetic and is shared, unchanged, by the oracle tests and the GPU tests.

Every generator returns plain numpy float64 arrays plus the frequency grid
(f0, df, nf) on which the periodogram is evaluated.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Curve:
    t: np.ndarray
    y: np.ndarray
    dy: np.ndarray
    f0: float
    df: float
    nf: int

    @property
    def nd(self) -> int:
        return int(self.t.size)


def single_small(seed: int = 0, nd: int = 1000, nf: int = 12000,
                 noiseless: bool = False) -> Curve:
    """Single FP64 light curve: N_d times uniform on [0, 100] (sorted), a
    sinusoid at 0.37 plus N(0, 0.1^2) noise, dy = 0.1; f_k = 0.002 + 0.002 k.
    With ``noiseless`` the series is an exact sinusoid plus offset, at a
    frequency that lies on the grid (k = 184)."""
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0.0, 100.0, nd))
    f0 = df = 0.002
    if noiseless:
        fs = f0 + 184 * df
        y = 0.7 * np.cos(2 * np.pi * fs * t) - 0.4 * np.sin(2 * np.pi * fs * t) + 3.0
    else:
        y = np.sin(2 * np.pi * 0.37 * t) + rng.normal(0.0, 0.1, nd)
    dy = np.full(nd, 0.1)
    return Curve(t, y, dy, f0, df, nf)


def gapped_times(rng, nd: int, years: int = 10, season: float = 245.0,
                 year: float = 365.0) -> np.ndarray:
    """Times uniform on the observing seasons [365 y, 365 y + 245), y = 0..years-1
    (120-day gaps every 365 days), sorted."""
    season_idx = rng.integers(0, years, nd)
    t = season_idx * year + rng.uniform(0.0, season, nd)
    return np.sort(t)


def single_large(seed: int = 1, nd: int = 1_000_000, span_years: int = 10,
                 nf: int | None = None) -> Curve:
    """Single large light curve: N_d times over [0, 3650] with 120-day gaps every
    365 days, y = three sinusoids (f ~ U[0.01, 5], amplitude ~ U[0.1, 1]) plus
    N(0, 0.2^2), dy ~ U(0.1, 0.3); df = 1/(5 * span), f0 = df, N_f = 12 N_d.
    ``nd`` and ``span_years`` shrink the same recipe for smaller test cases."""
    rng = np.random.default_rng(seed)
    t = gapped_times(rng, nd, years=span_years)
    fs = rng.uniform(0.01, 5.0, 3)
    amp = rng.uniform(0.1, 1.0, 3)
    ph = rng.uniform(0.0, 2 * np.pi, 3)
    y = np.zeros(nd)
    for f, a, p in zip(fs, amp, ph):
        y += a * np.sin(2 * np.pi * f * t + p)
    y += rng.normal(0.0, 0.2, nd)
    dy = rng.uniform(0.1, 0.3, nd)
    span = 365.0 * span_years
    df = 1.0 / (5.0 * span)
    return Curve(t, y, dy, df, df, int(nf if nf is not None else 12 * nd))


def batch_curve(rng, nd: int) -> Curve:
    """One curve of the batched workload: span log-uniform in [10, 1000] days,
    sorted uniform times, one sinusoid + N(0, 0.5^2), dy = 0.5,
    N_f = 12 N_d, df = 1/(5 span), f0 = df, signal frequency in
    [20 df, 0.8 f_max]."""
    span = float(np.exp(rng.uniform(np.log(10.0), np.log(1000.0))))
    t = np.sort(rng.uniform(0.0, span, nd))
    nf = 12 * nd
    df = 1.0 / (5.0 * span)
    fmax = df + (nf - 1) * df
    fsig = rng.uniform(20 * df, 0.8 * fmax)
    y = np.sin(2 * np.pi * fsig * t + rng.uniform(0, 2 * np.pi)) + rng.normal(0.0, 0.5, nd)
    dy = np.full(nd, 0.5)
    return Curve(t, y, dy, df, df, nf)


def batch(seed: int = 3, ncurves: int = 10_000, nd_min: int = 100,
          nd_max: int = 10_000) -> list[Curve]:
    """The batched workload: ``ncurves`` curves with N_d log-uniform in
    [nd_min, nd_max]."""
    rng = np.random.default_rng(seed)
    nds = np.floor(np.exp(rng.uniform(np.log(nd_min), np.log(nd_max), ncurves))).astype(np.int64)
    return [batch_curve(rng, int(n)) for n in nds]


def serving_requests(seed: int = 4, nreq: int = 20_000, rate: float = 2000.0,
                     nd_min: int = 50, nd_max: int = 200_000):
    """Open-loop Poisson request stream: (arrival_time_s, Curve, precision) with
    N_d log-uniform in [nd_min, nd_max] and FP32 / FP64 chosen by a fair coin."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, nreq)
    arrivals = np.cumsum(gaps)
    out = []
    for i in range(nreq):
        nd = int(np.floor(np.exp(rng.uniform(np.log(nd_min), np.log(nd_max)))))
        c = batch_curve(rng, nd)
        prec = "fp32" if rng.random() < 0.5 else "fp64"
        out.append((float(arrivals[i]), c, prec))
    return out


@dataclass
class SharedTimes:
    """Series observed at the same times: y and dy are nseries x nd (dy rows
    are identical when the series share their weights)."""
    t: np.ndarray
    y: np.ndarray
    dy: np.ndarray
    f0: float
    df: float
    nf: int

    @property
    def nd(self) -> int:
        return int(self.t.size)

    @property
    def nseries(self) -> int:
        return int(self.y.shape[0])

    def curve(self, i: int) -> Curve:
        return Curve(self.t, self.y[i], self.dy[i], self.f0, self.df, self.nf)


def shared_times(seed: int = 5, nd: int = 1_000_000, nseries: int = 8, span_years: int = 10,
                 nf: int | None = None, shared_dy: bool = True,
                 sorted_t: bool = True) -> SharedTimes:
    """Several series on the times of the single large curve (10 years with
    120-day gaps): each row of y is its own mix of three sinusoids
    (f ~ U[0.01, 5], amplitude ~ U[0.1, 1]) plus N(0, 0.2^2); dy ~ U(0.1, 0.3),
    one row for every series or (shared_dy False) a row per series;
    df = 1/(5 span), f0 = df, N_f = 12 N_d.  ``sorted_t`` False returns the
    same times (and the matching y, dy columns) in a random order."""
    rng = np.random.default_rng(seed)
    t = gapped_times(rng, nd, years=span_years)
    y = np.empty((nseries, nd))
    for i in range(nseries):
        fs = rng.uniform(0.01, 5.0, 3)
        amp = rng.uniform(0.1, 1.0, 3)
        ph = rng.uniform(0.0, 2 * np.pi, 3)
        y[i] = rng.normal(0.0, 0.2, nd)
        for f, a, p in zip(fs, amp, ph):
            y[i] += a * np.sin(2 * np.pi * f * t + p)
    if shared_dy:
        dy = np.broadcast_to(rng.uniform(0.1, 0.3, nd), (nseries, nd)).copy()
    else:
        dy = rng.uniform(0.1, 0.3, (nseries, nd))
    if not sorted_t:
        perm = rng.permutation(nd)
        t, y, dy = t[perm], y[:, perm], dy[:, perm]
    span = 365.0 * span_years
    df = 1.0 / (5.0 * span)
    return SharedTimes(t, y, dy, df, df, int(nf if nf is not None else 12 * nd))


def uniform_series(seed: int, nd: int, nf: int, span: float = 1.0, sorted_t: bool = True,
                   hetero_dy: bool = True) -> Curve:
    """Generic random series for edge-case tests: uniform times on [0, span],
    Gaussian values, dy ~ U(0.5, 1.5) (or 1), frequency grid f0 = df = 1/(5 span)."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, span, nd)
    if sorted_t:
        t = np.sort(t)
    y = rng.normal(0.0, 1.0, nd) + np.sin(2 * np.pi * 3.3 / span * t)
    dy = rng.uniform(0.5, 1.5, nd) if hetero_dy else np.ones(nd)
    df = 1.0 / (5.0 * span)
    return Curve(t, y, dy, df, df, nf)
