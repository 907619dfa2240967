"""Synthetic measurements for Eq. (1): y = A x_true + D g + w, w ~ N(0, sigma^2 I).

Reading: the SNR of a workload is the mean power of the noise-free data over
all P K M samples (zeros included) divided by sigma^2; the synthetic data hold
no direct arrivals (g = 0).  The phantom and the unit-variance noise come from
the seeded generators shared with the GPU path; only the scaling and the
operator are computed here.
"""
from __future__ import annotations

import numpy as np

from synth import phantom, noise

from . import operator


def noise_sigma(clean, snr_db: float) -> float:
    return float(np.sqrt(np.mean(np.asarray(clean) ** 2) / 10.0 ** (snr_db / 10.0)))


def synthesize(card):
    """Returns (x_true, y, sigma) with y of shape (P, K, M)."""
    x_true = phantom(card)
    clean = operator.forward(card, x_true)
    sigma = noise_sigma(clean, card.snr_db)
    return x_true, clean + sigma * noise(card), sigma
