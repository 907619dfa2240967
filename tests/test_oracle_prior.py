"""Pins of the oracle's QGGMRF prior (Eqs. (14)-(17)): closed values, symmetry,
convexity, the quadratic special case and derivatives by finite differences."""
import numpy as np
import pytest

from synth import tiny_card, random_vector
from synth.cards import Prior
from oracle import prior as qp


def _grid():
    return tiny_card(nx=7, nz=5).grid


def test_depth_modulation_end_values():
    """m_s = 1 at zero depth and m at the maximum depth (Eq. (17)); with a = 1
    it is linear in depth in between."""
    g = _grid()
    ms = qp.depth_modulation(g, 0.1, 1.0)
    depth = (np.arange(g.nz) + 0.5) * g.dz
    np.testing.assert_allclose(ms, 1.0 - 0.9 * depth / depth[-1], rtol=1e-15)
    assert abs(ms[-1] - 0.1) < 1e-15


def test_clique_count_and_weights():
    """8-neighbour pairs on an nz x nx grid: 4 nx nz - 3 (nx + nz) + 2, each once;
    an interior voxel's eight weights sum to one."""
    g = _grid()
    s, r, bw, sg = qp.cliques(g, Prior())
    nx, nz = g.nx, g.nz
    assert len(s) == 4 * nx * nz - 3 * (nx + nz) + 2
    pairs = {tuple(sorted(p)) for p in zip(s.tolist(), r.tolist())}
    assert len(pairs) == len(s)
    v = 2 * nx + 3
    tot = bw[s == v].sum() + bw[r == v].sum()
    assert abs(tot - 1.0) < 1e-15
    # sigma_g = sigma0 sqrt(m_s m_r) > 0
    assert np.all(sg > 0)


@pytest.mark.parametrize("p", [1.1, 1.5, 2.0])
def test_potential_even_zero_and_convex(p):
    pr = Prior(p=p)
    sg = 3.0
    d = np.linspace(-0.2, 0.2, 2001)
    rho = qp.rho(d, sg, pr)
    assert qp.rho(np.array(0.0), sg, pr) == 0.0
    np.testing.assert_array_equal(rho, qp.rho(-d, sg, pr))
    assert np.all(np.diff(rho, 2) >= -1e-18)


def test_quadratic_special_case():
    """p = q = 2: u^0 = 1, so rho = D^2 / (4 sg^2)."""
    pr = Prior(p=2.0, q=2.0)
    d = np.array([-1.0, -0.01, 0.0, 0.3, 2.0])
    np.testing.assert_allclose(qp.rho(d, 1.7, pr), d * d / (4 * 1.7 ** 2), rtol=1e-15)
    np.testing.assert_allclose(qp.half_curvature(d, 1.7, pr), 1.0 / (4 * 1.7 ** 2), rtol=1e-14)


def test_large_difference_limit():
    """For |D| >> T sg the ratio u^(q-p)/(1+u^(q-p)) tends to 1: rho -> |D|^p/(p sg^p)."""
    pr = Prior(p=1.1, T=0.01)
    sg = 1.0
    d = 1e6
    assert abs(qp.rho(np.array(d), sg, pr) / (d ** 1.1 / 1.1) - 1) < 1e-6


@pytest.mark.parametrize("p", [1.1, 1.6])
def test_derivatives_by_finite_differences(p):
    pr = Prior(p=p)
    sg = 2.5
    d = np.array([-0.3, -0.04, -0.002, 0.001, 0.02, 0.5])
    h = 1e-7
    num = (qp.rho(d + h, sg, pr) - qp.rho(d - h, sg, pr)) / (2 * h)
    np.testing.assert_allclose(qp.rho_prime(d, sg, pr), num, rtol=1e-6)
    np.testing.assert_allclose(qp.half_curvature(d, sg, pr), num / (2 * d), rtol=1e-6)
    # the limit at zero: 1 / (p sg^2 T^(2-p))
    lim = qp.half_curvature(np.array(0.0), sg, pr)
    assert abs(lim - 1.0 / (p * sg ** 2 * pr.T ** (2 - p))) < 1e-12 * lim


def test_gradient_by_finite_differences():
    g = _grid()
    pr = Prior()
    x = 0.05 * random_vector((g.nz, g.nx), seed=9)
    grad = qp.gradient(x, g, pr)
    h = 1e-7
    for v in (0, 9, 17, 34):
        e = np.zeros(g.nz * g.nx)
        e[v] = h
        e = e.reshape(x.shape)
        num = (qp.cost(x + e, g, pr) - qp.cost(x - e, g, pr)) / (2 * h)
        assert abs(grad.reshape(-1)[v] - num) <= 1e-6 * (abs(num) + 1e-3)


def test_surrogate_majorizes_and_touches():
    """The separable surrogate at x' equals the prior at x' and lies above it."""
    g = _grid()
    pr = Prior()
    xp = 0.05 * random_vector((g.nz, g.nx), seed=11)
    slope, curv = qp.surrogate(xp, g, pr)
    c0 = qp.cost(xp, g, pr)
    for seed in range(5):
        x = xp + 0.05 * random_vector((g.nz, g.nx), seed=20 + seed)
        d = x - xp
        q = c0 + np.sum(slope * d) + 0.5 * np.sum(curv * d * d)
        assert q >= qp.cost(x, g, pr) - 1e-12
