"""Observer statistics beyond one probe (oracle; test infrastructure only).

* Several observer points per observer location (the probes spread along the span): the
  time-averaged pressure and the RMS of the pressure perturbation are computed per point and
  then averaged over the points, and the OASPL of Eq. (9) is taken of the averaged RMS.
* Power spectral density of the pressure perturbation by Welch's method of averaged
  periodograms (the spectra section of each case: a number of windows with 50 % overlap).
  Readings where the paper is silent: periodic Hann window, each segment demeaned, one-sided
  density scaling (integral over frequency = variance), segment length the largest even L with
  n_windows segments of length L at a hop of L/2 inside the series.
"""
from __future__ import annotations

import numpy as np

from .fr import cumulative_prms


def observer_oaspl(series: np.ndarray, group: np.ndarray, n_group: int, p_ref: float):
    """series[a, n] per probe, group[a] its observer: (mean p_RMS per observer, OASPL per observer)."""
    series = np.atleast_2d(np.asarray(series, float))
    prms = np.array([cumulative_prms(series[a])[-1] for a in range(series.shape[0])])
    avg = np.array([prms[np.asarray(group) == g].mean() for g in range(n_group)])
    with np.errstate(divide="ignore"):
        return avg, 20.0 * np.log10(avg / p_ref)


def welch_psd(p: np.ndarray, n_windows: int, sample_dt: float):
    """Welch PSD of the pressure perturbation: n_windows demeaned, Hann-windowed segments of
    length L = 2 floor(n / (n_windows + 1)) at a hop of L/2; periodogram |DFT|^2 / (fs sum w^2),
    averaged over segments, doubled at every frequency but 0 and fs/2 (one-sided)."""
    p = np.asarray(p, float)
    L = 2 * (len(p) // (n_windows + 1))
    hop = L // 2
    fs = 1.0 / sample_dt
    t = np.arange(L)
    w = 0.5 - 0.5 * np.cos(2.0 * np.pi * t / L)
    acc = np.zeros(L // 2 + 1)
    for k in range(n_windows):
        seg = p[k * hop:k * hop + L]
        X = np.fft.rfft((seg - seg.mean()) * w)
        acc += np.abs(X) ** 2
    psd = acc / n_windows / (fs * (w ** 2).sum())
    psd[1:L // 2] *= 2.0
    if L % 2:
        psd[L // 2] *= 2.0
    return np.arange(L // 2 + 1) * fs / L, psd
