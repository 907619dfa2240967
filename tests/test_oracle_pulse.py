"""Pins of the oracle's pulse and template (Eqs. (8)-(10)): window support,
spectrum, interpolation exactness and the interpolation error bound.  None of
them re-evaluates the oracle's own pulse formula."""
import numpy as np
import pytest

from synth import card_c1, card_c2, tiny_card
from oracle import pulse


@pytest.mark.parametrize("mk", [card_c1, card_c2, tiny_card])
def test_window_is_open_interval(mk):
    """rect(t/t_0 - 1/2) is 1 only strictly inside (0, t_0): both ends are zero,
    and the template has Q L_h + 1 entries (Eq. (10))."""
    acq = mk().acq
    b = pulse.template(acq)
    lh = pulse.window_samples(acq)
    assert len(b) == acq.oversample * lh + 1
    assert b[0] == 0.0 and b[-1] == 0.0
    assert np.all(np.isfinite(b))
    # just outside the window the windowed response vanishes
    t = np.array([-1e-9, 0.0, acq.t_win, acq.t_win + 1e-9])
    assert np.all(pulse.windowed_response(t, acq) == 0.0)


def test_window_length_in_samples():
    assert pulse.window_samples(card_c1().acq) == 120
    assert pulse.window_samples(card_c2().acq) == 240


@pytest.mark.parametrize("mk", [card_c1, card_c2])
def test_spectrum_peaks_at_centre_frequency(mk):
    """An FFT of the tabulated pulse peaks at f_c (within one FFT bin), and its
    -6 dB band holds f_c; the FFT is independent of the pulse formula."""
    acq = mk().acq
    b = pulse.template(acq)
    fine_fs = acq.fs * acq.oversample
    n = 1 << 18
    spec = np.abs(np.fft.rfft(b, n))
    f = np.fft.rfftfreq(n, 1.0 / fine_fs)
    peak = f[np.argmax(spec)]
    assert abs(peak - acq.f_c) <= 2 * (f[1] - f[0]) + 0.02 * acq.f_c
    band = f[spec >= 0.5 * spec.max()]
    assert band.min() < acq.f_c < band.max()
    # a sigma_t = 1.25 us Gaussian envelope has a -6 dB band of 2*sqrt(2 ln 2)/(2 pi sigma_t)
    expect = 2 * np.sqrt(2 * np.log(2)) / (2 * np.pi * acq.sigma_t)
    assert abs((band.max() - band.min()) - expect) <= 0.05 * expect


def test_interpolation_exact_on_linear_data():
    """Linear interpolation reproduces any affine table exactly (brute check)."""
    b = np.linspace(-3.0, 5.0, 33)
    zf = np.array([0.25, 1.5, 7.75, 31.999, 16.0])
    val = pulse.interp(b, zf)
    np.testing.assert_allclose(val, -3.0 + 0.25 * zf, rtol=0, atol=1e-13)
    # zero at and beyond the ends
    assert np.all(pulse.interp(b, np.array([0.0, -1.0, 32.0, 40.0])) == 0.0)


@pytest.mark.parametrize("mk", [card_c1, card_c2])
def test_interpolation_error_within_bound(mk):
    """|I_b(z) - s(t)| <= h^2 max|s''| / 8 for linear interpolation with step h;
    |s''| <= (2 pi f_c)^2 (1 + small) for a wide-envelope sinusoid."""
    acq = mk().acq
    b = pulse.template(acq)
    lh = pulse.window_samples(acq)
    q = acq.oversample
    rng = np.random.default_rng(0)
    zf = rng.uniform(1.0, q * lh - 1.0, 5000)
    t = zf / (q * acq.fs)
    approx = pulse.interp(b, zf)
    # the analytic pulse written here from its definition (Gaussian-windowed sine)
    tc = acq.t_win / 2
    exact = np.sin(2 * np.pi * acq.f_c * (t - tc)) * np.exp(-(t - tc) ** 2 / (2 * acq.sigma_t ** 2))
    h = 1.0 / (q * acq.fs)
    w = 2 * np.pi * acq.f_c
    bound = h * h * (w + 1.0 / acq.sigma_t) ** 2 / 8
    assert np.max(np.abs(approx - exact)) <= bound
