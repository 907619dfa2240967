"""The system matrix A applied matrix-free, its transpose, and the basis D.

Eq. (13) gives trace (i, j) as a sum over voxels of the windowed response,
delayed by the voxel's travel time and weighted by its apodization:

    y_ij(t) = sum_v h~(t - T_ij(v)) * phi_ij(v) * x(v).

Sampling t at t_m = m / fs (reading: sample 0 at firing), using the tabulated
template b of Eq. (10) with linear interpolation, and carrying tau of Eq. (7)
in the voxel weight:

    y[i, j, m] = sum_v W_ij(v) x(v) I_b((m - D_ij(v)) Q),   D = fs T,  W = tau phi,

with I_b the interpolant of b (zero outside the open window).  Reading: the
scan positions of the array are separate firings, so their traces are stacked
as rows [P][K][M] of one measurement vector rather than summed (the paper's
"summing over all transmitters" applies to transmitters firing together, which
no workload here has).  Echoes that start at or after the last sample are
dropped.  The transpose is written out from the same sum.

D (Eq. (1)) has one column per trace: the template placed at the direct-arrival
delay of that trace, in that trace's rows only.

forward() and adjoint_voxels() take `workers`: with more than one, the traces
are split into that many contiguous runs, each run is evaluated by the same
per-trace code in its own process (a spawned pool), and the runs' results are
put together in run order (the adjoint's partial sums are added in that
order).  workers=None uses all host cores, at most 16.

With attenuation (some alpha_l > 0) the template is chosen per (trace, voxel)
from the bank of attenuation.py; `b` may be a single template [len] or such a
bank [G][len].  Reading: the direct arrival keeps the gamma = 0 template.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from . import attenuation, geometry, pulse

_CHUNK = 8192


def default_bank(card, absolute: bool = False) -> np.ndarray:
    """The templates the operator uses: [1][len] without attenuation."""
    if attenuation.n_bins(card) == 1:
        b = pulse.template(card.acq)[None, :]
        return np.abs(b) if absolute else b
    return attenuation.bank(card, absolute)


def _bank(card, b):
    return default_bank(card) if b is None else np.atleast_2d(np.asarray(b, float))


def _rows(card, bank, legs):
    """Template index per voxel from its legs' attenuations (all zero for a
    single template)."""
    if bank.shape[0] == 1:
        return np.zeros(np.shape(legs[0]), np.int64)
    if bank.shape[0] != attenuation.n_bins(card):
        raise ValueError("template bank does not match the card's attenuation bins")
    return attenuation.bins_of(legs, attenuation.step(card), bank.shape[0])


def _taps(delay, acq, bank, rows):
    """Sample indices and values of every voxel's interpolated template."""
    lh = pulse.window_samples(acq)
    m0 = np.floor(delay).astype(np.int64)
    k = np.arange(lh + 2)
    m = m0[:, None] + k[None, :]
    val = pulse.interp(bank, (m - delay[:, None]) * acq.oversample, rows)
    return m, val


def forward_trace(card, i, j, x_flat, b=None, weight_abs=False):
    """Trace (i, j) of A x, shape (M,).  x_flat: image in raster order (nz * nx)."""
    acq = card.acq
    bank = _bank(card, b)
    n_vox = card.grid.nx * card.grid.nz
    y = np.zeros(acq.n_samples)
    for s in range(0, n_vox, _CHUNK):
        vox = np.arange(s, min(s + _CHUNK, n_vox))
        delay, w, legs = geometry.trace_geometry(card, i, j, vox, legs=True)
        if weight_abs:
            w = np.abs(w)
        m, val = _taps(delay, acq, bank, _rows(card, bank, legs))
        contrib = val * (w * x_flat[vox])[:, None]
        keep = (m >= 0) & (m < acq.n_samples)
        y += np.bincount(m[keep], weights=contrib[keep], minlength=acq.n_samples)
    return y


def host_workers(workers=None) -> int:
    """Processes for the multi-core path: `workers`, or all host cores (at most 16)."""
    if workers is not None:
        return max(1, int(workers))
    return max(1, min(16, os.cpu_count() or 1))


def _runs(items, n):
    """`items` split into at most n contiguous, non-empty runs, in order."""
    n = max(1, min(n, len(items)))
    bounds = np.linspace(0, len(items), n + 1).round().astype(int)
    return [items[bounds[k]:bounds[k + 1]] for k in range(n)]


def _pool(n):
    return mp.get_context("spawn").Pool(n)


def _forward_run(args):
    card, traces, x_flat, bank, weight_abs = args
    return [forward_trace(card, i, j, x_flat, bank, weight_abs) for i, j in traces]


def forward(card, x, traces=None, b=None, weight_abs=False, workers=1):
    """A x as an array (P, K, M); `traces` restricts to a list of (i, j)."""
    a = card.array
    y = np.zeros((a.n_scans, a.n_rx, card.acq.n_samples))
    x_flat = np.asarray(x, float).reshape(-1)
    if traces is None:
        traces = [(i, j) for i in range(a.n_scans) for j in range(a.n_rx)]
    bank = _bank(card, b)
    n = host_workers(workers)
    if n > 1 and len(traces) > 1:
        runs = _runs(list(traces), n)
        with _pool(len(runs)) as pool:
            parts = pool.map(_forward_run, [(card, run, x_flat, bank, weight_abs) for run in runs])
        for run, part in zip(runs, parts):
            for (i, j), yt in zip(run, part):
                y[i, j] = yt
        return y
    for i, j in traces:
        y[i, j] = forward_trace(card, i, j, x_flat, bank, weight_abs)
    return y


def forward_columns(card, vox, coef, b=None, weight_abs=False):
    """sum over v in vox of coef[v] A[:, v], as traces (P, K, M): A x for an x
    that is zero outside the voxels `vox`."""
    acq, a = card.acq, card.array
    bank = _bank(card, b)
    vox = np.asarray(vox, np.int64)
    coef = np.asarray(coef, float)
    y = np.zeros((a.n_scans, a.n_rx, acq.n_samples))
    for i in range(a.n_scans):
        for j in range(a.n_rx):
            delay, w, legs = geometry.trace_geometry(card, i, j, vox, legs=True)
            if weight_abs:
                w = np.abs(w)
            m, val = _taps(delay, acq, bank, _rows(card, bank, legs))
            contrib = val * (w * coef)[:, None]
            keep = (m >= 0) & (m < acq.n_samples)
            y[i, j] = np.bincount(m[keep], weights=contrib[keep], minlength=acq.n_samples)
    return y


def _adjoint_traces(card, traces, rows, vox, bank, weight_abs):
    """sum over the listed traces (i, j) of their part of A^T r at `vox`;
    rows[k] is trace k's samples."""
    acq = card.acq
    out = np.zeros(len(vox))
    for (i, j), rij in zip(traces, rows):
        for s in range(0, len(vox), _CHUNK):
            sl = slice(s, s + _CHUNK)
            delay, w, legs = geometry.trace_geometry(card, i, j, vox[sl], legs=True)
            if weight_abs:
                w = np.abs(w)
            m, val = _taps(delay, acq, bank, _rows(card, bank, legs))
            keep = (m >= 0) & (m < acq.n_samples)
            rv = np.where(keep, rij[np.clip(m, 0, acq.n_samples - 1)], 0.0)
            out[sl] += w * np.sum(rv * val, axis=1)
    return out


def _adjoint_run(args):
    return _adjoint_traces(*args)


def adjoint_voxels(card, r, vox, b=None, weight_abs=False, workers=1):
    """(A^T r) at the flat voxel indices `vox`; r has shape (P, K, M)."""
    bank = _bank(card, b)
    vox = np.asarray(vox, np.int64)
    a = card.array
    traces = [(i, j) for i in range(a.n_scans) for j in range(a.n_rx)]
    n = host_workers(workers)
    if n > 1 and len(traces) > 1:
        runs = _runs(traces, n)
        with _pool(len(runs)) as pool:
            parts = pool.map(_adjoint_run, [(card, run, [r[i, j] for i, j in run], vox, bank, weight_abs)
                                            for run in runs])
        out = np.zeros(len(vox))
        for part in parts:
            out += part
        return out
    return _adjoint_traces(card, traces, [r[i, j] for i, j in traces], vox, bank, weight_abs)


def adjoint(card, r, b=None, weight_abs=False):
    """A^T r as an image (nz, nx)."""
    g = card.grid
    vox = np.arange(g.nx * g.nz)
    return adjoint_voxels(card, r, vox, b, weight_abs).reshape(g.nz, g.nx)


def dense(card, b=None) -> np.ndarray:
    """A as a dense (P K M, N) matrix, column v = trace response of voxel v."""
    g, a, acq = card.grid, card.array, card.acq
    bank = _bank(card, b)
    n_vox = g.nx * g.nz
    mat = np.zeros((a.n_scans * a.n_rx * acq.n_samples, n_vox))
    vox = np.arange(n_vox)
    for i in range(a.n_scans):
        for j in range(a.n_rx):
            row0 = (i * a.n_rx + j) * acq.n_samples
            delay, w, legs = geometry.trace_geometry(card, i, j, vox, legs=True)
            m, val = _taps(delay, acq, bank, _rows(card, bank, legs))
            keep = (m >= 0) & (m < acq.n_samples)
            cols = np.broadcast_to(vox[:, None], m.shape)
            np.add.at(mat, (row0 + m[keep], cols[keep]), (val * w[:, None])[keep])
    return mat


def direct_basis(card, b=None) -> np.ndarray:
    """Columns of D as traces d[i, j, :] (P, K, M)."""
    a, acq = card.array, card.acq
    b = pulse.template(acq) if b is None else np.atleast_2d(np.asarray(b, float))[0]
    m = np.arange(acq.n_samples)
    d = np.zeros((a.n_scans, a.n_rx, acq.n_samples))
    for i in range(a.n_scans):
        for j in range(a.n_rx):
            d[i, j] = pulse.interp(b, (m - geometry.direct_delay(card, i, j)) * acq.oversample)
    return d


def apply_direct(card, g, b=None) -> np.ndarray:
    """D g as traces (P, K, M)."""
    return direct_basis(card, b) * np.asarray(g, float)[:, :, None]


def abs_template(acq) -> np.ndarray:
    """|b|: its interpolant bounds |I_b| from above, since |(1-f)u + f v| <= (1-f)|u| + f|v|."""
    return np.abs(pulse.template(acq))
