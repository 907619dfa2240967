"""Pins of the oracle's grouped ICD (Sec. 2, "Optimization", run over a
lattice of voxel groups): the group curvature against a dense Abar, the
majorizer inequality on random group steps, monotone cost, and the minimiser
against a dense linear solve (quadratic prior) and against sequential ICD."""
import numpy as np
import pytest

from synth import tiny_card, random_vector
from synth.cards import Prior
from oracle import operator, solver, data, prior as qp


def _problem(n_layers=2, seed=7, **kw):
    card = tiny_card(n_layers=n_layers, nx=8, nz=7, n_scans=1, n_rx=3, n_samples=160, seed=seed, **kw)
    x_true, y, sigma = data.synthesize(card)
    return card, x_true, y, sigma


def test_groups_partition_the_image():
    card, _, _, _ = _problem()
    groups = solver.icd_groups(card.grid, 3, 2)
    allv = np.sort(np.concatenate(groups))
    np.testing.assert_array_equal(allv, np.arange(card.grid.nz * card.grid.nx))
    nx = card.grid.nx
    for grp in groups:  # no two members are 8-neighbours
        r, c = np.divmod(grp, nx)
        dr = np.abs(r[:, None] - r[None, :])
        dc = np.abs(c[:, None] - c[None, :])
        near = (dr <= 1) & (dc <= 1)
        assert np.count_nonzero(near) == len(grp)
    with pytest.raises(ValueError):
        solver.icd_groups(card.grid, 1, 4)


@pytest.mark.parametrize("rows,cols", [(2, 2), (3, 4)])
def test_group_curvature_is_a_majorizer(rows, cols):
    """d^G from the matrix-free sums equals (Abar^T Abar 1_G)_G from a dense
    Abar (beta even, so every weight is >= 0 and Abar is the dense matrix of
    the |b| template), is at least ||A_v||^2, and bounds delta^T A_G^T A_G
    delta by sum_v d^G_v delta_v^2 for random group steps."""
    card, _, _, _ = _problem(n_layers=3)
    groups = solver.icd_groups(card.grid, rows, cols)
    den = solver.group_denominator(card, groups)
    amat = operator.dense(card)
    abar = operator.dense(card, b=operator.default_bank(card, absolute=True))
    assert np.all(abar >= 0)
    rng = np.random.default_rng(5)
    for grp in groups:
        ref = abar[:, grp].T @ abar[:, grp].sum(axis=1)
        np.testing.assert_allclose(den[grp], ref, rtol=1e-12, atol=1e-14 * ref.max())
        assert np.all(den[grp] >= np.sum(amat[:, grp] ** 2, axis=0) * (1 - 1e-12))
        for _ in range(5):
            d = rng.standard_normal(len(grp))
            quad = float(np.sum((amat[:, grp] @ d) ** 2))
            assert quad <= float(np.sum(den[grp] * d * d)) * (1 + 1e-12)


def test_forward_columns_is_a_restricted_forward():
    card, _, _, _ = _problem(n_layers=3)
    g = card.grid
    x = random_vector((g.nz, g.nx), seed=4)
    vox = np.arange(0, g.nz * g.nx, 5)
    xs = np.zeros(g.nz * g.nx)
    xs[vox] = x.reshape(-1)[vox]
    np.testing.assert_allclose(operator.forward_columns(card, vox, xs[vox]),
                               operator.forward(card, xs.reshape(g.nz, g.nx)), rtol=0, atol=1e-13)


def test_grouped_icd_monotone():
    card, _, y, sigma = _problem(n_layers=3)
    _, _, cost = solver.icd_grouped(card, y, sigma, Prior(), 8, rows=2, cols=2)
    assert np.all(np.diff(cost) <= 1e-14 * cost[:-1])
    _, _, cs = solver.sqs(card, y, sigma, Prior(), 8)
    # each sweep does at least as well as a surrogate iteration here
    assert cost[-1] < cs[-1]


def test_grouped_icd_reaches_the_quadratic_minimiser():
    """p = q = 2: the minimiser solves the normal equations (dense solve)."""
    card, _, y, sigma = _problem(n_layers=2)
    pr = Prior(p=2.0, q=2.0, sigma0=0.05)
    g = card.grid
    n = g.nz * g.nx
    amat = operator.dense(card)
    dbasis = operator.direct_basis(card)
    P, K, M = dbasis.shape
    dmat = np.zeros((P * K * M, P * K))
    for t in range(P * K):
        dmat[t * M:(t + 1) * M, t] = dbasis.reshape(P * K, M)[t]
    full = np.hstack([amat, dmat])
    s, r, bw, sg = qp.cliques(g, pr)
    H = np.zeros((n + P * K, n + P * K))
    w = bw / (2 * sg ** 2)
    np.add.at(H, (s, s), w)
    np.add.at(H, (r, r), w)
    np.add.at(H, (s, r), -w)
    np.add.at(H, (r, s), -w)
    sol = np.linalg.solve(full.T @ full / sigma ** 2 + H, full.T @ y.reshape(-1) / sigma ** 2)
    x_opt, g_opt = sol[:n].reshape(g.nz, g.nx), sol[n:].reshape(P, K)
    # the minimiser is a fixed point of a grouped sweep
    x1, g1, _ = solver.icd_grouped(card, y, sigma, pr, 1, rows=2, cols=2, x0=x_opt, g0=g_opt)
    np.testing.assert_allclose(x1, x_opt, rtol=0, atol=1e-10 * np.max(np.abs(x_opt)))
    np.testing.assert_allclose(g1, g_opt, rtol=0, atol=1e-10 * np.max(np.abs(g_opt)))
    # and sweeps from zero approach it
    errs = [np.max(np.abs(solver.icd_grouped(card, y, sigma, pr, k, rows=2, cols=2)[0] - x_opt)) for k in (5, 40)]
    assert errs[1] < 0.5 * errs[0]


def test_grouped_and_sequential_icd_share_the_minimiser():
    card, _, y, sigma = _problem(n_layers=2)
    pr = Prior(p=1.2, T=0.5, sigma0=0.5)
    x_s, g_s, c_s = solver.icd(card, y, sigma, pr, 400)
    # sequential ICD's limit is (to its own convergence) a fixed point of the
    # grouped sweep, and the grouped sweeps from zero descend toward its cost
    x_g, g_g, c_1 = solver.icd_grouped(card, y, sigma, pr, 1, rows=3, cols=2, x0=x_s, g0=g_s)
    np.testing.assert_allclose(x_g, x_s, rtol=0, atol=1e-6 * np.max(np.abs(x_s)))
    assert abs(c_1[-1] - c_s[-1]) <= 1e-12 * c_s[-1]
    _, _, c_g = solver.icd_grouped(card, y, sigma, pr, 30, rows=3, cols=2)
    assert np.all(np.diff(c_g) <= 1e-14 * c_g[:-1])
    assert c_s[-1] * (1 - 1e-12) <= c_g[-1]
    assert c_g[-1] - c_s[-1] < 0.01 * (c_g[0] - c_s[-1])
