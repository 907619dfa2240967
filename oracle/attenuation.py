"""Attenuation bins: the windowed responses of Eqs. (9)-(10) for gamma > 0.

Test infrastructure (part of the oracle): a plain float64 statement of what
the attenuated operator computes, for checking the device library.

Eq. (13) uses h~(gamma(v), .) with each voxel's own total attenuation
gamma(v) = sum_l gamma_l(v), gamma_l = c_l alpha_l T_l = alpha_l x (path length
in layer l) (Eq. (3)), while Sec. 3 computes the windowed response once.
Readings (the paper gives no binning rule):
  * With every alpha_l = 0 there is one template (gamma = 0) and nothing here
    changes the operator.
  * Otherwise G = acq.n_gamma templates (default 16) are tabulated at
    gamma_g = g * dgamma, g = 0 .. G-1, with dgamma = 2 Gamma_max / (G - 1);
    Gamma_max is the largest one-way path attenuation over the problem's legs
    (voxel centres at the largest lateral distance from any transducer, every
    row).  2 Gamma_max bounds gamma(v) = Gamma_tx + Gamma_rx of every trace.
  * A (trace, voxel) pair uses the template nearest its gamma:
    bin = floor(gamma / dgamma + 1/2) in float64, gamma = Gamma_tx + Gamma_rx,
    capped at G - 1.  So |gamma - gamma_bin| <= dgamma / 2.  A pair whose
    gamma / dgamma lies within a hair of a half-integer has two equally near
    templates; near_ties() names such pairs so that a comparison can set them
    aside.
  * If Gamma_max = 0 (attenuating layers lie below every voxel) G is 1.
"""
from __future__ import annotations

import numpy as np

from . import geometry, pulse

MAX_BINS = 64


def attenuating(card) -> bool:
    return any(a != 0.0 for a in (card.medium.atten or ()))


def max_lateral(card) -> float:
    """Largest lateral distance from a transducer to a voxel centre [m]."""
    a, g = card.array, card.grid
    xs = list(a.tx_x) + [geometry.receiver_x(card, i, j) for i in range(a.n_scans) for j in range(a.n_rx)]
    xv = geometry.voxel_laterals(g)[[0, -1]]
    return float(max(abs(v - x) for x in xs for v in xv))


def max_leg(card) -> float:
    """Gamma_max: the largest one-way path attenuation over the legs.  At a
    fixed depth it grows with the lateral distance (every angle grows), so
    the rows are scanned at the largest lateral distance."""
    z = geometry.voxel_depths(card.grid)
    _, _, att = geometry.leg(card.medium, z, np.full_like(z, max_lateral(card)))
    return float(np.max(att))


def n_bins(card) -> int:
    if not attenuating(card):
        return 1
    g = int(getattr(card.acq, "n_gamma", 16))
    if not 2 <= g <= MAX_BINS:
        raise ValueError("n_gamma must be in 2..64")
    return 1 if max_leg(card) == 0.0 else g


def step(card) -> float:
    """dgamma [s]; 0 with a single bin."""
    g = n_bins(card)
    return 0.0 if g == 1 else 2.0 * max_leg(card) / (g - 1)


def gammas(card) -> np.ndarray:
    return step(card) * np.arange(n_bins(card))


def bank(card, absolute: bool = False) -> np.ndarray:
    """Templates b_g[n] = h~(gamma_g, n / (Q fs)) as an array [G][Q L_h + 1]
    (|b_g| with absolute=True, for the surrogate's curvature)."""
    b = np.stack([pulse.attenuated_template(card.acq, float(gm)) for gm in gammas(card)])
    return np.abs(b) if absolute else b


def bins_of(legs, dgamma: float, g: int) -> np.ndarray:
    """Template index per voxel: the bin nearest gamma = Gamma_tx + Gamma_rx."""
    if g == 1:
        return np.zeros(np.shape(legs[0]), np.int64)
    gamma = np.asarray(legs[0], float) + np.asarray(legs[1], float)
    return np.minimum(np.floor(gamma / dgamma + 0.5), g - 1).astype(np.int64)


def tie_distance(legs, dgamma: float) -> np.ndarray:
    """Distance of gamma / dgamma from the nearest half-integer, in bins: the
    margin by which a pair's nearest template is decided."""
    u = (np.asarray(legs[0], float) + np.asarray(legs[1], float)) / dgamma
    return np.abs(u - np.floor(u) - 0.5)


def near_ties(card, tol: float = 1e-9):
    """(i, j, v) of every (trace, voxel) pair whose gamma / dgamma lies within
    `tol` of a half-integer below the last bin: two templates are nearly as
    near, and an independent computation of gamma may pick the other."""
    g = n_bins(card)
    out = []
    if g == 1:
        return out
    dgamma = step(card)
    for i in range(card.array.n_scans):
        for j in range(card.array.n_rx):
            _, _, legs = geometry.trace_geometry(card, i, j, legs=True)
            u = (legs[0] + legs[1]) / dgamma
            hit = (tie_distance(legs, dgamma) < tol) & (u < g - 1)
            out.extend((i, j, int(v)) for v in np.nonzero(hit)[0])
    return out


def trace_bins(card, i: int, j: int, vox) -> np.ndarray:
    """Template index of every voxel in `vox` for trace (i, j)."""
    g = n_bins(card)
    if g == 1:
        return np.zeros(len(vox), np.int64)
    _, _, legs = geometry.trace_geometry(card, i, j, vox, legs=True)
    return bins_of(legs, step(card), g)
