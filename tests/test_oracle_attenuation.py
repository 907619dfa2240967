"""Pins of the oracle's attenuated operator (Eqs. (3), (7), (9), (10), (13) with
alpha > 0): the quadrature of the attenuated response against a time-domain
convolution with the Lorentzian kernel that e^{-gamma |f|} transforms to, the
bin rule against each pair's exact gamma, and the binned operator against
single-voxel responses built from that convolution.  None of them reuses the
oracle's frequency-domain formula."""
import dataclasses

import numpy as np
import pytest

from synth import attenuated_card, card_c1, tiny_card, random_vector
from oracle import attenuation, geometry, operator, pulse


def _gauss_legendre(a, b, panels, nodes=20):
    x, w = np.polynomial.legendre.leggauss(nodes)
    e = np.linspace(a, b, panels + 1)
    h = 0.5 * np.diff(e)
    m = 0.5 * (e[1:] + e[:-1])
    return (m[:, None] + h[:, None] * x).reshape(-1), (h[:, None] * w).reshape(-1)


def lorentz_response(acq, gamma, t, panels=50):
    """h(gamma, t) as the time-domain convolution s * L_gamma with the
    Lorentzian L_gamma(t) = 2 gamma / (gamma^2 + 4 pi^2 t^2), the inverse
    transform of e^{-gamma |f|}.  Near the peak (|t'| < 10 gamma / (2 pi)) the
    substitution t' = gamma tan(phi) / (2 pi) turns the kernel into d(phi) / pi;
    beyond it t' = tau1 e^u grades the panels; past t_0 + 12 sigma_t the pulse
    vanishes.  Composite Gauss-Legendre throughout."""
    t = np.asarray(t, float)
    if gamma == 0.0:  # the kernel is a delta
        return pulse.pulse(t, acq)
    flat = t.reshape(-1)
    phi1 = np.arctan(10.0)
    phi, wp = _gauss_legendre(-phi1, phi1, panels)
    shift = gamma * np.tan(phi) / (2.0 * np.pi)
    out = np.array([np.sum(pulse.pulse(tt - shift, acq) * wp) for tt in flat]) / np.pi
    tau1 = 10.0 * gamma / (2.0 * np.pi)
    far = acq.t_win + 12.0 * acq.sigma_t
    if tau1 < far:
        u, wu = _gauss_legendre(0.0, np.log(far / tau1), panels)
        tau = tau1 * np.exp(u)
        k = 2.0 * gamma / (gamma ** 2 + 4.0 * np.pi ** 2 * tau ** 2) * tau * wu
        out += np.array([np.sum((pulse.pulse(tt - tau, acq) + pulse.pulse(tt + tau, acq)) * k) for tt in flat])
    return out.reshape(t.shape)


@pytest.mark.parametrize("mk", [card_c1, tiny_card])
def test_quadrature_at_zero_is_the_pulse(mk):
    """gamma = 0: h = F^-1{S} = s (Eq. (9))."""
    acq = mk().acq
    t = np.linspace(0.0, acq.t_win, 301)
    np.testing.assert_allclose(pulse.attenuated_response(0.0, t, acq), pulse.pulse(t, acq), rtol=0, atol=1e-13)


@pytest.mark.parametrize("mk,gammas", [(tiny_card, (1e-9, 1e-8, 1e-7, 5e-7)), (card_c1, (2e-7, 2e-6))])
def test_quadrature_matches_lorentzian_convolution(mk, gammas):
    acq = mk().acq
    t = np.linspace(0.02 * acq.t_win, 0.98 * acq.t_win, 41)
    for gm in gammas:
        h = pulse.attenuated_response(gm, t, acq)
        np.testing.assert_allclose(h, lorentz_response(acq, gm, t), rtol=0, atol=1e-12)
        # attenuation removes energy: the response shrinks
        assert np.max(np.abs(h)) < np.max(np.abs(pulse.pulse(t, acq)))


def test_bank_layout():
    card = attenuated_card()
    b = attenuation.bank(card)
    g = attenuation.n_bins(card)
    lh = pulse.window_samples(card.acq)
    assert b.shape == (g, card.acq.oversample * lh + 1) and g == 16
    np.testing.assert_array_equal(b[0], pulse.template(card.acq))
    assert np.all(b[:, 0] == 0.0) and np.all(b[:, -1] == 0.0)
    gm = attenuation.gammas(card)
    np.testing.assert_allclose(np.diff(gm), attenuation.step(card), rtol=1e-13)
    # a row at gamma_g is the Lorentzian-convolved pulse on the open window
    n = np.arange(5, b.shape[1] - 5, 37)
    t = n / (card.acq.oversample * card.acq.fs)
    np.testing.assert_allclose(b[7, n], lorentz_response(card.acq, gm[7], t), rtol=0, atol=1e-12)
    np.testing.assert_array_equal(attenuation.bank(card, absolute=True), np.abs(b))


def test_no_attenuation_is_one_template():
    card = tiny_card(n_layers=3)
    assert attenuation.n_bins(card) == 1
    np.testing.assert_array_equal(operator.default_bank(card)[0], pulse.template(card.acq))
    # attenuation below every voxel leaves one template too
    below = tiny_card(n_layers=3, nz=10, atten=(0.0, 0.0, 3e-5))
    assert attenuation.max_leg(below) == 0.0 and attenuation.n_bins(below) == 1


@pytest.mark.parametrize("g", [2, 5, 16, 64])
def test_bins_are_nearest(g):
    """Every (trace, voxel) lands in the bin nearest its exact gamma (the sum of
    its two legs as trace_geometry returns it): the same index as a brute-force
    search over all G template attenuations, |gamma - gamma_bin| <= dgamma / 2;
    2 Gamma_max bounds every gamma and is nearly reached."""
    card = attenuated_card(n_gamma=g)
    step = attenuation.step(card)
    grid_g = np.arange(g) * step
    top = 0.0
    for i in range(card.array.n_scans):
        for j in range(card.array.n_rx):
            _, _, gamma = geometry.trace_geometry(card, i, j)
            _, _, legs = geometry.trace_geometry(card, i, j, legs=True)
            b = attenuation.bins_of(legs, step, g)
            assert b.min() >= 0 and b.max() <= g - 1
            brute = np.argmin(np.abs(gamma[:, None] - grid_g[None, :]), axis=1)
            clear = attenuation.tie_distance(legs, step) > 1e-9
            assert np.array_equal(b[clear], brute[clear])
            assert np.all(np.abs(gamma - b * step) <= step * (0.5 + 1e-12))
            assert np.all(gamma <= (g - 1) * step * (1 + 1e-12))
            top = max(top, float(np.max(np.maximum(legs[0], legs[1]))))
    assert top == pytest.approx(attenuation.max_leg(card), rel=1e-12)


def test_near_ties_finds_planted_tie():
    """near_ties() names a pair whose gamma sits on a half-integer of bins: a
    card whose dgamma is chosen so (the two legs of one pair summed) that it
    does; none on the stock attenuated card."""
    card = attenuated_card(n_gamma=16)
    assert attenuation.near_ties(card) == []
    legs = (np.array([0.3, 0.25]), np.array([0.45, 0.1]))
    d = attenuation.tie_distance(legs, 0.5)  # gamma / dgamma = 1.5 and 0.7
    assert d[0] == pytest.approx(0.0, abs=1e-15) and d[1] == pytest.approx(0.2)
    assert list(attenuation.bins_of(legs, 0.5, 16)) == [2, 1]


def test_max_leg_is_largest_over_rows_and_offsets():
    """Gamma_max from the largest lateral distance equals a brute-force maximum
    over every row and every lateral distance on the half-voxel lattice."""
    card = attenuated_card()
    g = card.grid
    z = geometry.voxel_depths(g)
    X = np.arange(0, int(round(2 * attenuation.max_lateral(card) / g.dx)) + 1) * 0.5 * g.dx
    zz, xx = np.meshgrid(z, X, indexing="ij")
    _, _, att = geometry.leg(card.medium, zz, xx)
    assert attenuation.max_leg(card) == pytest.approx(float(att.max()), rel=1e-13)


def test_adjoint_identity_attenuated():
    card = attenuated_card()
    g, a = card.grid, card.array
    x = random_vector((g.nz, g.nx), seed=3)
    r = random_vector((a.n_scans, a.n_rx, card.acq.n_samples), seed=4)
    lhs = float(np.sum(operator.forward(card, x) * r))
    rhs = float(np.sum(x * operator.adjoint(card, r)))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(r)
    amat = operator.dense(card)
    np.testing.assert_allclose(amat @ x.reshape(-1), operator.forward(card, x).reshape(-1), rtol=0, atol=1e-12)


def _single_voxel_expected(card, v, i, j, gamma):
    """Trace (i, j) of A e_v built from the Lorentzian convolution at the given
    gamma: W h~(gamma, .) on the fine grid, interpolated linearly at the
    sample times (Eqs. (10), (13))."""
    acq = card.acq
    q, lh = acq.oversample, pulse.window_samples(acq)
    n = np.arange(q * lh + 1)
    b = lorentz_response(acq, gamma, n / (q * acq.fs))
    b[0] = b[-1] = 0.0
    delay, w, _ = geometry.trace_geometry(card, i, j, [v])
    m = np.arange(acq.n_samples)
    return w[0] * pulse.interp(b, (m - delay[0]) * q)


def test_single_voxel_uses_its_bin():
    """A e_v per trace is the voxel's weight times the template of its bin."""
    card = attenuated_card()
    step = attenuation.step(card)
    g = card.grid
    for v in (5, g.nx * 9 + 3, g.nx * g.nz - 2):
        x = np.zeros(g.nx * g.nz)
        x[v] = 1.0
        y = operator.forward(card, x.reshape(g.nz, g.nx))
        for i in range(card.array.n_scans):
            for j in range(card.array.n_rx):
                _, _, legs = geometry.trace_geometry(card, i, j, [v], legs=True)
                k = int(attenuation.bins_of(legs, step, 16)[0])
                np.testing.assert_allclose(y[i, j], _single_voxel_expected(card, v, i, j, k * step),
                                           rtol=0, atol=1e-10)


def test_binning_error_shrinks_with_more_bins():
    """Against each voxel's own gamma (the unbinned Eq. (13)) the binned
    operator's error falls as the bins get finer (about as 1 / G)."""
    g = attenuated_card().grid
    vox = [g.nx * 12 + 4, g.nx * 15 + 9]
    errs = []
    for n_gamma in (4, 16, 64):
        card = attenuated_card(n_gamma=n_gamma)
        e = 0.0
        for v in vox:
            x = np.zeros(g.nx * g.nz)
            x[v] = 1.0
            y = operator.forward(card, x.reshape(g.nz, g.nx), traces=[(0, 0), (1, 2)])
            for i, j in [(0, 0), (1, 2)]:
                _, _, gamma = geometry.trace_geometry(card, i, j, [v])
                e = max(e, float(np.max(np.abs(y[i, j] - _single_voxel_expected(card, v, i, j, gamma[0])))))
        errs.append(e)
    assert errs[0] > errs[1] > errs[2] > 0.0
    assert errs[2] < 0.25 * errs[0]


def test_bins_change_with_n_gamma_only_when_attenuating():
    plain = tiny_card(n_layers=3)
    card = dataclasses.replace(plain, acq=dataclasses.replace(plain.acq, n_gamma=4))
    assert attenuation.n_bins(card) == 1
    with pytest.raises(ValueError):
        attenuation.n_bins(attenuated_card(n_gamma=65))
