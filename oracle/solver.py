"""MAP cost of Eq. (18) and two minimisers of it.

    C(x, g) = ||y - A x - D g||^2 / (2 sigma^2) + sum_{s,r} b_sr rho(x_s - x_r).

sqs():  the parity solver.  Reading: the paper minimises with ICD, whose
        pseudocode lives in a cited work; the iteration here instead updates
        every voxel at once from one A x and one A^T e per iteration.  Each
        iteration
          1. forms e = y - A x - D g and records C(x, g);
          2. sets each g_ij to its exact minimiser for fixed x (the columns of
             D have disjoint rows, so this is one division per trace);
          3. takes the separable-surrogate step
               x_s -= (-(A^T e)_s / sigma^2 + slope_s) / (d_s + curv_s),
             with (slope, curv) from the prior surrogate at x and
             d = Abar^T Abar 1 / sigma^2, Abar the operator built from |W| and
             the template |b| (elementwise Abar >= |A|, so diag(d) >= A^T A / sigma^2).
        Start x = 0, g = 0 unless given; no positivity constraint (the image is
        a signed reflection coefficient).  After the last iteration the cost
        of the final (x, g) is appended, so the history has n_iter + 1 entries.
icd():  the paper's solver (Sec. 2, "Optimization"), in raster voxel order, on
        a dense A; one g update per sweep.  Used only on tiny problems.
icd_grouped():
        ICD over a lattice of voxel groups: group (a, b) holds the voxels with
        row % R == a and column % S == b (R, S >= 2, so no two members are
        8-neighbours), visited in the order a = 0..R-1, b = 0..S-1.  The
        members of a group move together, each by its one-voxel ICD step with
        the prior's neighbours held fixed and the data curvature
        d^G_v = (Abar^T Abar 1_G)_v / sigma^2 in place of ||A_v||^2 / sigma^2
        (Abar as for sqs; 1_G the group's indicator).  diag(Abar^T Abar 1_G)
        bounds A_G^T A_G, so every group step lowers the cost; members whose
        columns share no sample move exactly as sequential ICD with the
        curvature ||Abar_v||^2 would.  Reading: the paper's ICD runs one
        voxel at a time (its pseudocode is in a cited work); this is the
        grouped form a parallel device runs.
Both decrease C monotonically and, the cost being strictly convex, share its
minimiser.
"""
from __future__ import annotations

import numpy as np

from . import operator, prior as qprior


def data_cost(e, sigma) -> float:
    return float(np.sum(np.asarray(e, float) ** 2) / (2.0 * sigma ** 2))


def map_cost(card, y, x, g, sigma, pr) -> float:
    e = y - operator.forward(card, x) - operator.apply_direct(card, g)
    return data_cost(e, sigma) + qprior.cost(x, card.grid, pr)


def sqs_denominator(card, sigma) -> np.ndarray:
    """d = Abar^T (Abar 1) / sigma^2, image-shaped."""
    babs = operator.default_bank(card, absolute=True)
    ones = np.ones((card.grid.nz, card.grid.nx))
    col = operator.forward(card, ones, b=babs, weight_abs=True)
    return operator.adjoint(card, col, b=babs, weight_abs=True) / sigma ** 2


def sqs_denominator_voxels(card, sigma, vox, workers=1) -> np.ndarray:
    """d at the flat voxel indices `vox`: Abar 1 over every trace, then
    Abar^T of it at those voxels (on `workers` processes, see operator)."""
    babs = operator.default_bank(card, absolute=True)
    ones = np.ones((card.grid.nz, card.grid.nx))
    col = operator.forward(card, ones, b=babs, weight_abs=True, workers=workers)
    return operator.adjoint_voxels(card, col, vox, b=babs, weight_abs=True, workers=workers) / sigma ** 2


def first_step_voxels(card, y, sigma, pr, vox, den_vox, estimate_direct=None, workers=1):
    """The first surrogate iteration from x = 0, g = 0 at the voxels `vox`
    (x^1 there, g^1 and the cost C(0, 0)), given d at those voxels: e = y,
    the exact g step, then x^1_s = -(-(A^T e)_s / sigma^2 + slope_s) /
    (d_s + curv_s) with the prior surrogate at x = 0."""
    grid, a = card.grid, card.array
    if estimate_direct is None:
        estimate_direct = bool(getattr(pr, "estimate_direct", True))
    x0 = np.zeros((grid.nz, grid.nx))
    g = np.zeros((a.n_scans, a.n_rx))
    dbasis = operator.direct_basis(card)
    e = np.array(y, float)
    cost0 = data_cost(e, sigma) + qprior.cost(x0, grid, pr)
    if estimate_direct:
        g = direct_step(dbasis, e)
        e = e - dbasis * g[:, :, None]
    u = operator.adjoint_voxels(card, e, vox, workers=workers)
    slope, curv = qprior.surrogate(x0, grid, pr)
    vox = np.asarray(vox, np.int64)
    x1 = -(-u / sigma ** 2 + slope.reshape(-1)[vox]) / (np.asarray(den_vox, float) + curv.reshape(-1)[vox])
    return x1, g, cost0


def direct_step(dbasis, e):
    """Per-trace exact g increment: <d_ij, e_ij> / ||d_ij||^2 (zero where d_ij = 0)."""
    nrm = np.sum(dbasis ** 2, axis=2)
    num = np.sum(dbasis * e, axis=2)
    return np.where(nrm > 0, num / np.where(nrm > 0, nrm, 1.0), 0.0)


def sqs(card, y, sigma, pr, n_iter, x0=None, g0=None, estimate_direct=True, den=None,
        history=False):
    """Run n_iter surrogate iterations; returns (x, g, cost[n_iter + 1]) (+ iterates)."""
    grid, a = card.grid, card.array
    x = np.zeros((grid.nz, grid.nx)) if x0 is None else np.array(x0, float)
    g = np.zeros((a.n_scans, a.n_rx)) if g0 is None else np.array(g0, float)
    b = operator.default_bank(card)
    dbasis = operator.direct_basis(card, b)
    if den is None:
        den = sqs_denominator(card, sigma)
    costs, iterates = [], []
    for _ in range(n_iter):
        e = y - operator.forward(card, x, b=b) - dbasis * g[:, :, None]
        costs.append(data_cost(e, sigma) + qprior.cost(x, grid, pr))
        if estimate_direct:
            dg = direct_step(dbasis, e)
            g = g + dg
            e = e - dbasis * dg[:, :, None]
        grad_data = -operator.adjoint(card, e, b=b) / sigma ** 2
        slope, curv = qprior.surrogate(x, grid, pr)
        x = x - (grad_data + slope) / (den + curv)
        iterates.append((x.copy(), g.copy()))
    e = y - operator.forward(card, x, b=b) - dbasis * g[:, :, None]
    costs.append(data_cost(e, sigma) + qprior.cost(x, grid, pr))
    if history:
        return x, g, np.array(costs), iterates
    return x, g, np.array(costs)


def icd(card, y, sigma, pr, n_sweeps, x0=None, g0=None, estimate_direct=True, amat=None):
    """ICD sweeps in raster order on a dense A; returns (x, g, cost[n_sweeps + 1])."""
    grid, a, acq = card.grid, card.array, card.acq
    if amat is None:
        amat = operator.dense(card)
    x = np.zeros(grid.nz * grid.nx) if x0 is None else np.array(x0, float).reshape(-1)
    g = np.zeros((a.n_scans, a.n_rx)) if g0 is None else np.array(g0, float)
    dbasis = operator.direct_basis(card)
    col_sq = np.sum(amat ** 2, axis=0)
    e = (y - dbasis * g[:, :, None]).reshape(-1) - amat @ x
    costs = []
    for _ in range(n_sweeps):
        costs.append(data_cost(e, sigma) + qprior.cost(x, grid, pr))
        if estimate_direct:
            e3 = e.reshape(a.n_scans, a.n_rx, acq.n_samples)
            dg = direct_step(dbasis, e3)
            g = g + dg
            e = (e3 - dbasis * dg[:, :, None]).reshape(-1)
        for v in range(x.size):
            theta1 = -(amat[:, v] @ e) / sigma ** 2
            theta2 = col_sq[v] / sigma ** 2
            slope, curv = qprior.icd_terms(x, grid, pr, v)
            if theta2 + curv <= 0:
                continue
            step = -(theta1 + slope) / (theta2 + curv)
            x[v] += step
            e -= amat[:, v] * step
    costs.append(data_cost(e, sigma) + qprior.cost(x, grid, pr))
    return x.reshape(grid.nz, grid.nx), g, np.array(costs)


def icd_groups(grid, rows: int, cols: int):
    """Flat voxel indices of each lattice group, in visiting order."""
    if rows < 2 or cols < 2:
        raise ValueError("group lattice must be at least 2 x 2")
    idx = np.arange(grid.nz * grid.nx).reshape(grid.nz, grid.nx)
    return [idx[a::rows, b::cols].reshape(-1) for a in range(rows) for b in range(cols)]


def group_denominator(card, groups) -> np.ndarray:
    """d^G_v = (Abar^T Abar 1_G)_v for every voxel v of every group G (not yet
    divided by sigma^2), as a flat array."""
    babs = operator.default_bank(card, absolute=True)
    d = np.zeros(card.grid.nz * card.grid.nx)
    for grp in groups:
        col = operator.forward_columns(card, grp, np.ones(len(grp)), b=babs, weight_abs=True)
        d[grp] = operator.adjoint_voxels(card, col, grp, b=babs, weight_abs=True)
    return d


def icd_grouped(card, y, sigma, pr, n_sweeps, rows: int = 8, cols: int = 8, x0=None, g0=None,
                estimate_direct=True, den=None, history=False):
    """Grouped ICD sweeps; returns (x, g, cost[n_sweeps + 1]) (+ iterate after
    each sweep).  Each sweep records the cost, takes the exact g step, then
    visits the groups in order."""
    grid, a = card.grid, card.array
    groups = icd_groups(grid, rows, cols)
    if den is None:
        den = group_denominator(card, groups)
    bank = operator.default_bank(card)
    dbasis = operator.direct_basis(card, bank)
    x = np.zeros(grid.nz * grid.nx) if x0 is None else np.array(x0, float).reshape(-1)
    g = np.zeros((a.n_scans, a.n_rx)) if g0 is None else np.array(g0, float)
    e = y - operator.forward(card, x.reshape(grid.nz, grid.nx), b=bank) - dbasis * g[:, :, None]
    costs, iterates = [], []
    for _ in range(n_sweeps):
        costs.append(data_cost(e, sigma) + qprior.cost(x, grid, pr))
        if estimate_direct:
            dg = direct_step(dbasis, e)
            g = g + dg
            e = e - dbasis * dg[:, :, None]
        for grp in groups:
            theta1 = -operator.adjoint_voxels(card, e, grp, b=bank) / sigma ** 2
            theta2 = den[grp] / sigma ** 2
            step = np.zeros(len(grp))
            for k, v in enumerate(grp):
                slope, curv = qprior.icd_terms(x, grid, pr, int(v))
                if theta2[k] + curv > 0:
                    step[k] = -(theta1[k] + slope) / (theta2[k] + curv)
            x[grp] += step
            e = e - operator.forward_columns(card, grp, step, b=bank)
        iterates.append((x.reshape(grid.nz, grid.nx).copy(), g.copy()))
    costs.append(data_cost(e, sigma) + qprior.cost(x, grid, pr))
    if history:
        return x.reshape(grid.nz, grid.nx), g, np.array(costs), iterates
    return x.reshape(grid.nz, grid.nx), g, np.array(costs)
