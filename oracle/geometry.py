"""Ray geometry in a stack of planar layers (Sec. 2, "Multi-layered structures").

Frame: x is the lateral coordinate along the array, z the depth below the
array face (z = 0 is the top of layer 1, Fig. 1).  Layer l has speed c_l; its
top lies at the sum of the thicknesses above it; the last layer is unbounded.

A "leg" is the one-way path from a point on the array face to a voxel centre.
For a leg reaching depth z_v at lateral distance X, layer l is crossed over a
vertical extent eta_l (the full thickness for layers above the voxel's layer,
the remaining depth in the voxel's own layer, zero below it).  Snell's law
(Eq. (6)) keeps sin(theta_l)/c_l equal to one ray parameter kappa on every
layer, so the lateral offset of Eq. (5) is

    X(kappa) = sum_l eta_l * tan(theta_l),   sin(theta_l) = kappa * c_l,

which increases with kappa.  The paper finds the matching incidence angle by
binary search (text after Eq. (6)); the oracle solves the same equation for
kappa with its own safeguarded Newton iteration, to full float64 precision.
Reading: the search variable is kappa in [0, 1/c_max), c_max the fastest
traversed layer, because the paper's range theta_1 in [0, pi/2] passes the
critical angle wherever a deeper layer is faster and Eq. (6) is then undefined.

From kappa follow the travel time of Eq. (4), the angle sum that enters the
apodization of Eq. (12), and the path length that multiplies alpha_l in
gamma_l = c_l * alpha_l * T_l (Eq. (3)).
"""
from __future__ import annotations

import numpy as np


def layer_tops(medium) -> np.ndarray:
    """Depth of the top of every layer; layer 1 starts at the array face."""
    return np.concatenate([[0.0], np.cumsum(np.asarray(medium.thickness, float))])


def voxel_depths(grid) -> np.ndarray:
    """Depths of the voxel centres of rows 0..nz-1."""
    return grid.z0 + (np.arange(grid.nz) + 0.5) * grid.dz


def voxel_laterals(grid) -> np.ndarray:
    """Lateral positions of the voxel centres of columns 0..nx-1."""
    return grid.x0 + (np.arange(grid.nx) + 0.5) * grid.dx


def path_thicknesses(medium, depth) -> np.ndarray:
    """eta[..., l]: vertical extent of layer l on the way from z = 0 to `depth`."""
    tops = layer_tops(medium)
    n_lay = medium.n_layers
    depth = np.asarray(depth, float)
    eta = np.zeros(depth.shape + (n_lay,))
    for l in range(n_lay):
        bottom = tops[l + 1] if l + 1 < n_lay else np.inf
        eta[..., l] = np.clip(np.minimum(depth, bottom) - tops[l], 0.0, None)
    return eta


def voxel_layer(medium, depth) -> np.ndarray:
    """Index (0-based) of the deepest layer with a positive crossing extent."""
    eta = path_thicknesses(medium, depth)
    return np.sum(eta > 0, axis=-1) - 1


def transmittance(medium, depth) -> np.ndarray:
    """tau of Eq. (7): product over the interfaces above the voxel.

    Reading: each interface between layers a and b (impedance Z = rho * c)
    contributes its two-way normal-incidence pressure transmission
    (2 Z_b / (Z_a + Z_b)) * (2 Z_a / (Z_a + Z_b)); layer 1 contributes 1.
    """
    lay = np.atleast_1d(voxel_layer(medium, depth))
    z = np.asarray(medium.density, float) * np.asarray(medium.speed, float)
    out = np.ones(lay.shape)
    for k in range(medium.n_layers - 1):
        t2 = 4.0 * z[k] * z[k + 1] / (z[k] + z[k + 1]) ** 2
        out = np.where(lay > k, out * t2, out)
    return out.reshape(np.shape(depth))


def _offset(kappa, eta, c):
    # layers the leg does not reach (eta = 0) take no part; their sine is set to 0
    s = np.where(eta > 0, kappa[:, None] * c[None, :], 0.0)
    cosv = np.sqrt((1.0 - s) * (1.0 + s))
    x = np.sum(eta * s / cosv, axis=1)
    dx = np.sum(eta * c[None, :] / cosv ** 3, axis=1)
    return x, dx


def solve_kappa(eta, c, X, n_iter: int = 200) -> np.ndarray:
    """Ray parameter kappa with X(kappa) = X for every row of `eta`.

    eta: (n, L) crossing extents; c: (L,) speeds; X: (n,) lateral distances >= 0.
    Safeguarded Newton on the increasing function X(kappa) - X: each step keeps
    a bracket [lo, hi] of the root and falls back to its midpoint whenever the
    Newton point leaves it.
    """
    eta = np.atleast_2d(np.asarray(eta, float))
    c = np.asarray(c, float)
    X = np.broadcast_to(np.asarray(X, float), (eta.shape[0],)).copy()
    cmax = np.max(np.where(eta > 0, c[None, :], 0.0), axis=1)
    lo = np.zeros_like(X)
    hi = 1.0 / cmax
    k = 0.5 * (lo + hi)
    done = X == 0.0
    for _ in range(n_iter):
        xk, dxk = _offset(k, eta, c)
        f = xk - X
        lo = np.where(f < 0, k, lo)
        hi = np.where(f > 0, k, hi)
        kn = k - f / dxk
        bad = ~((kn > lo) & (kn < hi))
        kn = np.where(bad, 0.5 * (lo + hi), kn)
        step = np.abs(kn - k)
        k = np.where(done, 0.0, kn)
        if np.all(done | (step <= 2 * np.finfo(float).eps * np.abs(k))):
            break
    return np.where(done, 0.0, k)


def leg(medium, depth, X):
    """One-way legs from the array face to voxel centres.

    depth, X: broadcastable arrays (voxel-centre depth, lateral distance).
    Returns (T, theta_sum, path_atten):
      T           travel time [s], sum_l eta_l / (c_l cos theta_l)          (Eq. (4))
      theta_sum   sum over traversed layers of theta_l                      (Eq. (12))
      path_atten  sum_l alpha_l * eta_l / cos theta_l  (= sum of gamma_l, Eq. (3))
    """
    depth, X = np.broadcast_arrays(np.asarray(depth, float), np.abs(np.asarray(X, float)))
    shape = depth.shape
    eta = path_thicknesses(medium, depth.ravel())
    c = np.asarray(medium.speed, float)
    alpha = np.asarray(medium.atten, float)
    kappa = solve_kappa(eta, c, X.ravel())
    used = eta > 0
    s = np.where(used, kappa[:, None] * c[None, :], 0.0)
    cosv = np.sqrt((1.0 - s) * (1.0 + s))
    T = np.sum(eta / (c[None, :] * cosv), axis=1)
    theta = np.sum(np.arcsin(s), axis=1)
    att = np.sum(alpha[None, :] * eta / cosv, axis=1)
    return T.reshape(shape), theta.reshape(shape), att.reshape(shape)


def apodization(theta_tx, theta_rx, beta: int):
    """phi^(beta) of Eq. (12): cos^beta of each leg's angle sum, multiplied."""
    return np.cos(theta_tx) ** beta * np.cos(theta_rx) ** beta


def receiver_x(card, i: int, j: int) -> float:
    """Absolute lateral position of receiver j during scan i."""
    return card.array.tx_x[i] + card.array.rx_offset[j]


def trace_geometry(card, i: int, j: int, vox=None, legs: bool = False):
    """Per-voxel delay, weight and attenuation for trace (scan i, receiver j).

    vox: optional flat voxel indices (v = row * nx + col); default all voxels.
    Returns flat arrays over those voxels:
      delay   fs * (T_tx + T_rx), the echo's start in samples after firing
      weight  tau(v) * phi^(beta)(v)   (tau of Eq. (7), phi of Eq. (12))
      gamma   total attenuation exponent gamma(v) of Eq. (7)
    With legs=True the attenuation comes as its two one-way parts
    (gamma_tx, gamma_rx) instead of their sum.
    """
    g = card.grid
    if vox is None:
        vox = np.arange(g.nx * g.nz)
    vox = np.asarray(vox, np.int64)
    z = voxel_depths(g)[vox // g.nx]
    xv = voxel_laterals(g)[vox % g.nx]
    xs = card.array.tx_x[i]
    xr = receiver_x(card, i, j)
    t_tx, th_tx, a_tx = leg(card.medium, z, xv - xs)
    t_rx, th_rx, a_rx = leg(card.medium, z, xv - xr)
    delay = card.acq.fs * (t_tx + t_rx)
    weight = transmittance(card.medium, z) * apodization(th_tx, th_rx, card.array.beta)
    if legs:
        return delay, weight, (a_tx, a_rx)
    return delay, weight, a_tx + a_rx


def direct_delay(card, i: int, j: int) -> float:
    """Start (samples) of the direct arrival of trace (i, j).

    Reading: the direct-arrival signal of Eq. (1) travels along the array face
    in layer 1, so it starts |x_rx - x_tx| / c_1 after firing.
    """
    return card.acq.fs * abs(receiver_x(card, i, j) - card.array.tx_x[i]) / card.medium.speed[0]
