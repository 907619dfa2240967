"""Pins of the oracle's MAP cost (Eqs. (2), (18)) and its two minimisers: cost
at zero, gradient by finite differences, monotone decrease, agreement of SQS
and ICD at convergence, the quadratic case against a dense linear solve, and
warm-start resume."""
import numpy as np
import pytest

from synth import tiny_card, card_c1, random_vector
from synth.cards import Prior
from oracle import operator, solver, data, prior as qp


def _problem(n_layers=2, seed=7, **kw):
    card = tiny_card(n_layers=n_layers, nx=8, nz=7, n_scans=1, n_rx=3, n_samples=160, seed=seed, **kw)
    x_true, y, sigma = data.synthesize(card)
    return card, x_true, y, sigma


def test_cost_at_zero():
    card, _, y, sigma = _problem()
    g = card.grid
    c0 = solver.map_cost(card, y, np.zeros((g.nz, g.nx)), np.zeros((1, 3)), sigma, Prior())
    assert abs(c0 - np.sum(y ** 2) / (2 * sigma ** 2)) <= 1e-12 * c0


def test_cost_gradient_by_finite_differences():
    card, _, y, sigma = _problem()
    pr = Prior()
    g = card.grid
    x = 0.1 * random_vector((g.nz, g.nx), seed=3)
    gg = np.zeros((1, 3))
    e = y - operator.forward(card, x) - operator.apply_direct(card, gg)
    grad = -operator.adjoint(card, e) / sigma ** 2 + qp.gradient(x, g, pr)
    h = 1e-6
    for v in (0, 13, 40):
        d = np.zeros(g.nz * g.nx)
        d[v] = h
        d = d.reshape(x.shape)
        num = (solver.map_cost(card, y, x + d, gg, sigma, pr)
               - solver.map_cost(card, y, x - d, gg, sigma, pr)) / (2 * h)
        assert abs(grad.reshape(-1)[v] - num) <= 1e-5 * (abs(num) + 1.0)


def test_snr_of_synthetic_data():
    card = card_c1()
    x_true, y, sigma = data.synthesize(card)
    clean = operator.forward(card, x_true)
    snr = 10 * np.log10(np.mean(clean ** 2) / np.mean((y - clean) ** 2))
    assert abs(snr - card.snr_db) < 0.6  # 2048 noise samples: +-0.5 dB sampling spread
    assert abs(10 * np.log10(np.mean(clean ** 2) / sigma ** 2) - card.snr_db) < 1e-9


def test_sqs_monotone():
    card, _, y, sigma = _problem(n_layers=3)
    _, _, cost = solver.sqs(card, y, sigma, Prior(), 25)
    assert np.all(np.diff(cost) <= 1e-14 * cost[:-1])
    assert cost[-1] < 0.5 * cost[0]


def _sqs_step(card, y, sigma, pr, x, g, den):
    """One surrogate iteration from (x, g); returns the new (x, g)."""
    x1, g1, _ = solver.sqs(card, y, sigma, pr, 1, x0=x, g0=g, den=den)
    return x1, g1


def test_sqs_and_icd_share_the_minimiser():
    """Strict convexity (Sec. 2, "Optimization") gives one minimiser.  ICD
    converges to a point where the cost gradient vanishes, and that point is a
    fixed point of the simultaneous surrogate iteration."""
    card, _, y, sigma = _problem(n_layers=2)
    pr = Prior(p=1.2, T=0.5, sigma0=0.5)
    amat = operator.dense(card)
    x_i, g_i, c_i = solver.icd(card, y, sigma, pr, 400, amat=amat)
    assert np.all(np.diff(c_i) <= 1e-13 * c_i[:-1])
    e = y - operator.forward(card, x_i) - operator.apply_direct(card, g_i)
    grad = -operator.adjoint(card, e) / sigma ** 2 + qp.gradient(x_i, card.grid, pr)
    grad0 = -operator.adjoint(card, y) / sigma ** 2
    assert np.max(np.abs(grad)) <= 1e-7 * np.max(np.abs(grad0))
    den = solver.sqs_denominator(card, sigma)
    x_s, g_s = _sqs_step(card, y, sigma, pr, x_i, g_i, den)
    np.testing.assert_allclose(x_s, x_i, rtol=0, atol=1e-8 * np.max(np.abs(x_i)))
    # and surrogate steps from zero move toward it with decreasing cost
    _, _, c_s = solver.sqs(card, y, sigma, pr, 30, den=den)
    assert np.all(np.diff(c_s) <= 1e-14 * c_s[:-1])
    assert c_s[-1] >= c_i[-1] * (1 - 1e-12)


def test_quadratic_prior_matches_dense_solve():
    """p = q = 2 makes the cost quadratic in (x, g); its minimiser solves the
    normal equations, computed with a dense numpy solve.  ICD reaches it, and
    it is a fixed point of the surrogate iteration."""
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
    # prior Hessian: each pair contributes b (x_s - x_r)^2 / (4 sg^2)
    s, r, bw, sg = qp.cliques(g, pr)
    H = np.zeros((n + P * K, n + P * K))
    w = bw / (2 * sg ** 2)  # second derivative of b D^2/(4 sg^2)
    np.add.at(H, (s, s), w)
    np.add.at(H, (r, r), w)
    np.add.at(H, (s, r), -w)
    np.add.at(H, (r, s), -w)
    lhs = full.T @ full / sigma ** 2 + H
    rhs = full.T @ y.reshape(-1) / sigma ** 2
    sol = np.linalg.solve(lhs, rhs)
    x_opt, g_opt = sol[:n].reshape(g.nz, g.nx), sol[n:].reshape(P, K)
    x_i, g_i, _ = solver.icd(card, y, sigma, pr, 600, amat=amat)
    np.testing.assert_allclose(x_i, x_opt, rtol=0, atol=1e-7 * np.max(np.abs(x_opt)))
    den = solver.sqs_denominator(card, sigma)
    x_s, g_s = _sqs_step(card, y, sigma, pr, x_opt, g_opt, den)
    np.testing.assert_allclose(x_s, x_opt, rtol=0, atol=1e-10 * np.max(np.abs(x_opt)))


def test_direct_arrival_recovered():
    """Data made of D g_true alone: one g step recovers g_true exactly."""
    card = tiny_card(n_layers=2, nx=6, nz=5, n_scans=2, n_rx=3, n_samples=200)
    g_true = np.array([[0.7, -0.2, 1.3], [0.1, 0.0, -0.9]])
    y = operator.apply_direct(card, g_true)
    dbasis = operator.direct_basis(card)
    np.testing.assert_allclose(solver.direct_step(dbasis, y), g_true, rtol=1e-13, atol=1e-15)


def test_resume_equals_continuous_run():
    card, _, y, sigma = _problem(n_layers=3)
    pr = Prior()
    x20, g20, c20 = solver.sqs(card, y, sigma, pr, 20)
    x10, g10, c10 = solver.sqs(card, y, sigma, pr, 10)
    x2, g2, c2 = solver.sqs(card, y, sigma, pr, 10, x0=x10, g0=g10)
    np.testing.assert_allclose(x2, x20, rtol=0, atol=1e-13 * np.max(np.abs(x20)))
    np.testing.assert_allclose(c2, c20[10:], rtol=1e-13)


def test_sampled_curvature_and_first_step_equal_the_full_ones():
    """The voxel-sampled curvature and first iteration used at full size are
    the full-image ones restricted to the samples (on a small card, on two
    worker processes)."""
    from synth import tiny_card
    card = tiny_card(n_layers=3, nx=12, nz=10, n_scans=2, n_rx=3, n_samples=200)
    _, y, sigma = data.synthesize(card)
    y = y + operator.apply_direct(card, np.array([[0.5, -0.3, 0.8], [0.2, 0.9, -0.4]]))
    vox = np.array([0, 7, 33, 64, 119])
    dfull = solver.sqs_denominator(card, sigma).reshape(-1)
    dvox = solver.sqs_denominator_voxels(card, sigma, vox, workers=2)
    np.testing.assert_allclose(dvox, dfull[vox], rtol=1e-13)
    x1, g1, c = solver.sqs(card, y, sigma, card.prior, 1)
    xs, gs, c0 = solver.first_step_voxels(card, y, sigma, card.prior, vox, dvox, workers=2)
    np.testing.assert_allclose(xs, x1.reshape(-1)[vox], rtol=1e-12, atol=1e-15 * np.abs(x1).max())
    np.testing.assert_allclose(gs, g1, rtol=1e-12)
    assert c0 == pytest.approx(c[0], rel=1e-13)


def test_multicore_operator_equals_single_core():
    from synth import tiny_card, random_vector
    card = tiny_card(n_layers=3, nx=12, nz=10, n_scans=3, n_rx=3, n_samples=200)
    x = random_vector((card.grid.nz, card.grid.nx), seed=5)
    r = random_vector((3, 3, 200), seed=6)
    np.testing.assert_array_equal(operator.forward(card, x, workers=3), operator.forward(card, x))
    vox = np.arange(card.n_voxels)
    np.testing.assert_allclose(operator.adjoint_voxels(card, r, vox, workers=4),
                               operator.adjoint_voxels(card, r, vox), rtol=1e-13, atol=1e-15)
