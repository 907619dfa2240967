"""Transmitted pulse and its windowed, tabulated impulse response (Eqs. (8)-(10)).

Readings (the paper gives no pulse shape, window length or tabulation rule):
  * s(t) is a Gaussian-windowed sinusoid centred at t_c = t_0 / 2:
        s(t) = sin(2 pi f_c (t - t_c)) * exp(-(t - t_c)^2 / (2 sigma_t^2)).
  * With gamma = 0, Eq. (9) gives h = F^-1{S} = s (tau is carried by the
    voxel weight, not by the template).
  * Eq. (10) keeps h on the open interval 0 < t < t_0 (rect(u) is 1 only for
    |u| < 1/2), t_0 = L_h / fs with an integer window length L_h.
  * The template is computed once (Sec. 3, last paragraph) on a grid Q times
    finer than the sampling grid, b[n] = h~(n / (Q fs)), n = 0 .. Q L_h, so
    b[0] = b[Q L_h] = 0; between grid points it is interpolated linearly.
"""
from __future__ import annotations

import numpy as np


def window_samples(acq) -> int:
    """L_h = t_0 * fs; the window must hold a whole number of samples."""
    lh = acq.t_win * acq.fs
    n = int(round(lh))
    if abs(lh - n) > 1e-9 * max(1.0, lh):
        raise ValueError("t_win * fs must be an integer")
    return n


def pulse(t, acq):
    """s(t), the transmitted signal."""
    tc = 0.5 * acq.t_win
    u = np.asarray(t, float) - tc
    return np.sin(2 * np.pi * acq.f_c * u) * np.exp(-u * u / (2 * acq.sigma_t ** 2))


def windowed_response(t, acq):
    """h~(0, t) of Eq. (10) for gamma = 0: s(t) on 0 < t < t_0, zero elsewhere."""
    t = np.asarray(t, float)
    inside = (t > 0) & (t < acq.t_win)
    return np.where(inside, pulse(t, acq), 0.0)


def template(acq) -> np.ndarray:
    """Tabulated template b[n] = h~(0, n / (Q fs)), n = 0 .. Q L_h."""
    lh = window_samples(acq)
    q = acq.oversample
    n = np.arange(q * lh + 1)
    b = windowed_response(n / (q * acq.fs), acq)
    b[0] = 0.0
    b[-1] = 0.0
    return b


def interp(b: np.ndarray, zf):
    """Linear interpolation of b at fine-grid position zf; zero outside (0, len(b)-1)."""
    zf = np.asarray(zf, float)
    last = len(b) - 1
    inside = (zf > 0) & (zf < last)
    zc = np.where(inside, zf, 0.0)
    n = np.floor(zc).astype(np.int64)
    f = zc - n
    n1 = np.minimum(n + 1, last)
    val = (1.0 - f) * b[n] + f * b[n1]
    return np.where(inside, val, 0.0)
