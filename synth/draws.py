"""Seeded random draws: phantoms, unit-variance noise and random test vectors.

All generators use numpy's PCG64 bit generator with an explicit seed, so the
same seed gives the same array on every machine.  Nothing here evaluates the
reconstruction method; scaling noise to a target SNR needs the noise-free data
and is left to the caller.
"""
from __future__ import annotations

import numpy as np

from .cards import Card


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def phantom(card: Card) -> np.ndarray:
    """Reflectivity image x_true, shape (nz, nx), float64.

    Full-width interface rows take the card's reflectivities.  An optional
    debonding gap replaces the interface at its row over a seeded lateral span
    with a top face and a bottom face a seeded thickness lower.  Point reflectors
    of seeded sign and amplitude are then placed in the card's row/column band,
    at least `min_spacing` voxels (Chebyshev) apart and off the interface rows.
    """
    g, ph = card.grid, card.phantom
    rng = _rng(ph.seed)
    x = np.zeros((g.nz, g.nx), dtype=np.float64)
    for row, refl in ph.interfaces:
        if 0 <= row < g.nz:
            x[row, :] = refl
    blocked = {row for row, _ in ph.interfaces}
    if ph.gap is not None:
        row, t_lo, t_hi, s_lo, s_hi, r_top, r_bot, r_out = ph.gap
        thick = rng.uniform(t_lo, t_hi)
        n_rows = max(1, int(round(thick / g.dz)))
        span = int(round(rng.uniform(s_lo, s_hi) * g.nx))
        start = int(rng.integers(0, g.nx - span + 1))
        x[row, :] = r_out
        x[row, start:start + span] = r_top
        bottom = row + n_rows
        if bottom < g.nz:
            x[bottom, start:start + span] = r_bot
            blocked.add(bottom)
        blocked.add(row)
    placed = []
    r_lo, r_hi = ph.rows
    c_lo, c_hi = ph.cols
    tries = 0
    while len(placed) < ph.n_reflectors:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place reflectors with the requested spacing")
        r = int(rng.integers(r_lo, r_hi))
        c = int(rng.integers(c_lo, c_hi))
        if any(abs(r - b) < 2 for b in blocked):
            continue
        if any(max(abs(r - pr), abs(c - pc)) < ph.min_spacing for pr, pc in placed):
            continue
        amp = rng.uniform(ph.amp_lo, ph.amp_hi) * (1.0 if rng.random() < 0.5 else -1.0)
        x[r, c] = amp
        placed.append((r, c))
    return x


def noise(card: Card) -> np.ndarray:
    """Unit-variance Gaussian noise, shape (P, K, M), float64."""
    a = card.array
    return _rng(card.noise_seed).standard_normal((a.n_scans, a.n_rx, card.acq.n_samples))


def random_vector(shape, seed: int, kind: str = "normal") -> np.ndarray:
    """A seeded float64 test vector: 'normal' N(0,1), 'uniform' U[-1,1] or 'sparse'
    (N(0,1) on a seeded 2 % of entries, zero elsewhere)."""
    rng = _rng(seed)
    if kind == "normal":
        return rng.standard_normal(shape)
    if kind == "uniform":
        return rng.uniform(-1.0, 1.0, shape)
    if kind == "sparse":
        v = rng.standard_normal(shape)
        keep = rng.random(shape) < 0.02
        return np.where(keep, v, 0.0)
    raise ValueError(kind)
