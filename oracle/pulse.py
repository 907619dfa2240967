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


def interp(b: np.ndarray, zf, rows=None):
    """Linear interpolation of b at fine-grid position zf; zero outside (0, len(b)-1).

    With `rows`, b is a bank [G][len] and rows[k] picks the template of zf[k, ...].
    """
    zf = np.asarray(zf, float)
    last = b.shape[-1] - 1
    inside = (zf > 0) & (zf < last)
    zc = np.where(inside, zf, 0.0)
    n = np.floor(zc).astype(np.int64)
    f = zc - n
    n1 = np.minimum(n + 1, last)
    if rows is None:
        val = (1.0 - f) * b[n] + f * b[n1]
    else:
        r = np.asarray(rows, np.int64).reshape(np.asarray(rows).shape + (1,) * (zf.ndim - np.ndim(rows)))
        val = (1.0 - f) * b[r, n] + f * b[r, n1]
    return np.where(inside, val, 0.0)


# ---------------------------------------------------------------------------
# Attenuated response, Eq. (9) with gamma > 0.
#
# With S(f) the Fourier transform of s (convention S(f) = int s(t) e^{-2 pi i f t} dt),
# a Gaussian-windowed sine centred at t_c has
#     S(f) = [G(f - f_c) - G(f + f_c)] e^{-2 pi i f t_c} / (2i),
#     G(f) = sigma_t sqrt(2 pi) exp(-2 pi^2 sigma_t^2 f^2).
# s is real, so the inverse transform of S(f) e^{-gamma |f|} folds onto f > 0:
#     h(gamma, t) = int_0^inf [G(f - f_c) - G(f + f_c)] e^{-gamma f} sin(2 pi f (t - t_c)) df.
# (At gamma = 0 this is s(t) itself.)  The integral is evaluated by composite
# Gauss-Legendre quadrature in float64 over [0, f_c + 6 / (pi sigma_t)], past
# which the Gaussian factor is below e^-72 of its peak; panels are short
# against the period of the sine over the window, so the rule converges to
# rounding.  tau of Eq. (9) is carried by the voxel weight, as for gamma = 0.
# ---------------------------------------------------------------------------

_GL_NODES = 20


def spectrum_band(acq) -> float:
    """Upper end of the frequency range that the quadrature covers [Hz]."""
    return acq.f_c + 6.0 / (np.pi * acq.sigma_t)


def _quadrature(acq, t):
    """Nodes and weights on [0, spectrum_band] for times t (enough panels that
    each spans at most 1/8 of a period of sin(2 pi f (t - t_c)))."""
    fmax = spectrum_band(acq)
    umax = float(np.max(np.abs(np.asarray(t, float) - 0.5 * acq.t_win), initial=0.0))
    panels = max(16, int(np.ceil(8.0 * fmax * umax)))
    x, w = np.polynomial.legendre.leggauss(_GL_NODES)
    edges = np.linspace(0.0, fmax, panels + 1)
    half = 0.5 * (edges[1:] - edges[:-1])
    mid = 0.5 * (edges[1:] + edges[:-1])
    f = (mid[:, None] + half[:, None] * x[None, :]).reshape(-1)
    wf = (half[:, None] * w[None, :]).reshape(-1)
    return f, wf


def spectrum_weight(f, acq):
    """G(f - f_c) - G(f + f_c): the magnitude factor of S on f >= 0."""
    f = np.asarray(f, float)
    s = acq.sigma_t
    c = s * np.sqrt(2.0 * np.pi)
    return c * (np.exp(-2.0 * (np.pi * s * (f - acq.f_c)) ** 2) - np.exp(-2.0 * (np.pi * s * (f + acq.f_c)) ** 2))


def attenuated_response(gamma: float, t, acq):
    """h(gamma, t) of Eq. (9) (tau excluded) by quadrature of the spectrum."""
    t = np.asarray(t, float)
    f, wf = _quadrature(acq, t)
    amp = wf * spectrum_weight(f, acq) * np.exp(-gamma * f)
    u = t.reshape(-1) - 0.5 * acq.t_win
    out = np.sin(2.0 * np.pi * u[:, None] * f[None, :]) @ amp
    return out.reshape(t.shape)


def attenuated_template(acq, gamma: float) -> np.ndarray:
    """b_gamma[n] = h~(gamma, n / (Q fs)), n = 0 .. Q L_h (Eq. (10)): zero at
    both ends of the open window.  gamma = 0 gives the closed-form template."""
    if gamma == 0.0:
        return template(acq)
    lh = window_samples(acq)
    q = acq.oversample
    n = np.arange(q * lh + 1)
    b = attenuated_response(gamma, n / (q * acq.fs), acq)
    b[0] = 0.0
    b[-1] = 0.0
    return b
