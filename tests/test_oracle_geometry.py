"""Pins of the oracle's ray geometry (Sec. 2, Eqs. (4)-(6), (12)) against
closed forms, Fermat's principle and symmetry, none of which reuse its solver."""
import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

from synth import card_c1, tiny_card
from synth.cards import Medium, R_WATER_STEEL, R_STEEL_CEMENT, R_CEMENT_ROCK
from oracle import geometry

MM = 1e-3


def _medium(speeds, thick, dens=None):
    n = len(speeds)
    return Medium(speed=tuple(speeds), thickness=tuple(thick), atten=(0.0,) * n,
                  density=tuple(dens or (1000.0,) * n))


def test_single_layer_is_straight_ray():
    med = _medium([1480.0], [])
    z = np.array([0.25, 3.0, 17.5, 40.0]) * MM
    X = np.array([0.0, 5.0, 12.25, 90.0]) * MM
    T, th, _ = geometry.leg(med, z[:, None], X[None, :])
    R = np.hypot(z[:, None], X[None, :])
    # kappa is exact to an ulp or two; near grazing (X/z = 360 here) the
    # cosine 1 - kappa c loses digits, ~eps / (1 - kappa c) relative
    np.testing.assert_allclose(T, R / 1480.0, rtol=1e-10)
    steep = X[None, :] < 10 * z[:, None]
    np.testing.assert_allclose(T[steep], (R / 1480.0)[steep], rtol=1e-14)
    np.testing.assert_allclose(th, np.arctan2(X[None, :], z[:, None]), rtol=1e-12, atol=1e-15)


def test_equal_speeds_reduce_to_straight_ray():
    med = _medium([3000.0, 3000.0, 3000.0], [4 * MM, 7 * MM])
    z = np.array([2.0, 6.0, 20.0]) * MM
    X = np.array([1.0, 33.0]) * MM
    T, th, _ = geometry.leg(med, z[:, None], X[None, :])
    np.testing.assert_allclose(T, np.hypot(z[:, None], X[None, :]) / 3000.0, rtol=1e-13)
    # three equal angles sum to three times the straight-ray angle
    np.testing.assert_allclose(th[2], 3 * np.arctan2(X, z[2]), rtol=1e-12)


def _two_layer_quartic(c1, c2, h1, h2, X):
    """Travel time through two layers from the crossing point xi solving Snell's law.

    sin t1 / c1 = sin t2 / c2 with sin t1 = xi / r1, sin t2 = (X - xi) / r2 gives,
    after squaring, c2^2 xi^2 ((X-xi)^2 + h2^2) = c1^2 (X-xi)^2 (xi^2 + h1^2): a quartic.
    """
    a, b = c2 ** 2, c1 ** 2
    # expand a xi^2 ((X - xi)^2 + h2^2) - b (X - xi)^2 (xi^2 + h1^2)
    p_left = np.polymul([a, 0, 0], np.polyadd(np.polymul([1, -X], [1, -X]), [h2 ** 2]))
    p_right = np.polymul([b], np.polymul(np.polymul([1, -X], [1, -X]), [1, 0, h1 ** 2]))
    coeffs = np.polysub(p_left, p_right)
    best = None
    for root in np.roots(coeffs):
        if abs(root.imag) > 1e-9 * max(X, 1e-12):
            continue
        xi = root.real
        if xi < -1e-15 or xi > X + 1e-15:
            continue
        r1, r2 = np.hypot(xi, h1), np.hypot(X - xi, h2)
        # keep the root of the unsquared equation
        if abs(xi / (c1 * r1) - (X - xi) / (c2 * r2)) > 1e-9 / c1:
            continue
        T = r1 / c1 + r2 / c2
        best = T if best is None else min(best, T)
    return best


@pytest.mark.parametrize("c1,c2", [(1480.0, 5900.0), (5900.0, 3000.0), (3000.0, 1480.0)])
def test_two_layers_match_quartic(c1, c2):
    h1 = 10 * MM
    med = _medium([c1, c2], [h1])
    for depth in (13 * MM, 18 * MM, 40 * MM):
        for X in (0.7 * MM, 6 * MM, 25 * MM, 80 * MM):
            T, _, _ = geometry.leg(med, np.array(depth), np.array(X))
            Tq = _two_layer_quartic(c1, c2, h1, depth - h1, X)
            assert Tq is not None
            assert abs(float(T) - Tq) <= 1e-12 * Tq


def _fermat_time(med, depth, X):
    """Minimum over interface crossing points of sum_l sqrt(dxi_l^2 + eta_l^2) / c_l."""
    eta = geometry.path_thicknesses(med, np.array([depth]))[0]
    c = np.asarray(med.speed)
    used = eta > 0
    eta, c = eta[used], c[used]
    n = len(eta)

    def t_of(xi):
        pts = np.concatenate([[0.0], xi, [X]])
        return float(np.sum(np.hypot(np.diff(pts), eta) / c))

    if n == 1:
        return t_of(np.array([]))
    if n == 2:
        res = minimize_scalar(lambda u: t_of(np.array([u])), bounds=(0.0, X),
                              method="bounded", options={"xatol": 1e-16 * max(X, 1e-3)})
        return res.fun
    # dense grid then gradient polish of the convex objective
    best, arg = np.inf, None
    grid = np.linspace(0.0, X, 41)
    for u in grid:
        for w in grid:
            if w < u:
                continue
            xi = np.array([u, w] + [X] * (n - 3))[: n - 1]
            val = t_of(xi)
            if val < best:
                best, arg = val, xi
    res = minimize(t_of, arg, method="Nelder-Mead",
                   options={"xatol": 1e-15, "fatol": 1e-22, "maxiter": 40000, "maxfev": 80000})
    return min(res.fun, best)


@pytest.mark.parametrize("depth_mm,X_mm", [(12.0, 3.0), (15.5, 20.0), (22.0, 9.0), (30.0, 41.0), (19.0, 0.5)])
def test_three_layers_match_fermat_minimum(depth_mm, X_mm):
    card = card_c1()
    med = card.medium
    T, _, _ = geometry.leg(med, np.array(depth_mm * MM), np.array(X_mm * MM))
    Tf = _fermat_time(med, depth_mm * MM, X_mm * MM)
    # the Fermat time is a minimum, so it can only exceed the true one by the
    # optimiser's residual, which is quadratic in its position error
    assert Tf >= float(T) * (1 - 1e-13)
    assert Tf - float(T) <= 1e-12 * float(T)


def test_leg_symmetric_and_monotone():
    med = card_c1().medium
    z = np.linspace(0.25, 31.75, 64) * MM
    X = np.linspace(0.0, 60.0, 121) * MM
    T, th, _ = geometry.leg(med, z[:, None], X[None, :])
    Tm, thm, _ = geometry.leg(med, z[:, None], -X[None, :])
    np.testing.assert_array_equal(T, Tm)
    # within one layer the time grows with depth (vertical slowness > 0); just
    # below an interface into a faster layer it can drop, because the ray may
    # run along that layer (the Fermat minimum of a head-wave path)
    lay = geometry.voxel_layer(med, z)
    same = lay[1:] == lay[:-1]
    assert np.all(np.diff(T, axis=0)[same] > 0), "travel time grows with depth in a layer"
    assert np.all(np.diff(T, axis=1) > 0), "travel time grows with lateral offset"
    assert np.all(np.diff(th, axis=1) > 0)


def test_snell_invariant_along_leg():
    """sin(theta_l)/c_l is one constant on every crossed layer (Eq. (6)), checked
    by recovering each layer's angle from the path's own crossing offsets."""
    med = card_c1().medium
    depth, X = 25 * MM, 30 * MM
    eta = geometry.path_thicknesses(med, np.array([depth]))[0]
    kappa = geometry.solve_kappa(eta[None, :], np.asarray(med.speed), np.array([X]))[0]
    sines = kappa * np.asarray(med.speed)
    seg = eta * sines / np.sqrt(1 - sines ** 2)     # lateral run in each layer
    assert abs(seg.sum() - X) <= 1e-15 * X * 10
    ang = np.arctan2(seg, eta)
    np.testing.assert_allclose(np.sin(ang) / np.asarray(med.speed), kappa, rtol=1e-13)


def test_transmittance_equals_energy_balance():
    """Two-way transmission across an interface equals 1 - R^2 (R the pressure
    reflection coefficient): energy not reflected is transmitted."""
    card = tiny_card(n_layers=4)
    med = card.medium
    tops = geometry.layer_tops(med)
    depths = np.array([tops[1] - 1e-4, tops[1] + 1e-4, tops[2] + 1e-4, tops[3] + 1e-4])
    tau = geometry.transmittance(med, depths)
    expect = [1.0, 1 - R_WATER_STEEL ** 2, (1 - R_WATER_STEEL ** 2) * (1 - R_STEEL_CEMENT ** 2),
              (1 - R_WATER_STEEL ** 2) * (1 - R_STEEL_CEMENT ** 2) * (1 - R_CEMENT_ROCK ** 2)]
    # the card reflectivities are rounded to four digits
    np.testing.assert_allclose(tau, expect, rtol=2e-3)
    same = _medium([2000.0, 2000.0], [5 * MM])
    assert geometry.transmittance(same, np.array([9 * MM]))[0] == 1.0


def test_single_layer_apodization_closed_form():
    """With one layer the angle of a leg is atan(X / z), so Eq. (12) becomes
    (z / R_tx)^beta (z / R_rx)^beta."""
    card = tiny_card(n_layers=1, nx=9, nz=7, n_scans=2, n_rx=3, beta=5)
    for i in range(2):
        for j in range(3):
            d, w, _ = geometry.trace_geometry(card, i, j)
            z = np.repeat(geometry.voxel_depths(card.grid), card.grid.nx)
            xv = np.tile(geometry.voxel_laterals(card.grid), card.grid.nz)
            rt = np.hypot(z, xv - card.array.tx_x[i])
            rr = np.hypot(z, xv - geometry.receiver_x(card, i, j))
            np.testing.assert_allclose(w, (z / rt) ** 5 * (z / rr) ** 5, rtol=1e-12)
            # the tiny grid reaches X/z = 32, where kappa's last ulp costs ~1e-13
            np.testing.assert_allclose(d, card.acq.fs * (rt + rr) / card.medium.speed[0], rtol=1e-12)


def test_grazing_leg_beyond_critical_angle():
    """A leg to a far voxel below a fast layer still has a ray (kappa < 1/c_max),
    and its time matches the Fermat minimum."""
    med = card_c1().medium
    depth, X = 20 * MM, 150 * MM
    T, th, _ = geometry.leg(med, np.array(depth), np.array(X))
    assert np.isfinite(T)
    Tf = _fermat_time(med, depth, X)
    assert abs(Tf - float(T)) <= 1e-12 * float(T)


def test_time_drops_below_fast_interface_as_fermat_says():
    """0.25 mm into steel under 10 mm of water, 5 mm off axis: the ray that runs
    along the steel beats the straight water path, as a Fermat minimum must."""
    med = card_c1().medium
    t_above, _, _ = geometry.leg(med, np.array(9.75 * MM), np.array(5 * MM))
    t_below, _, _ = geometry.leg(med, np.array(10.25 * MM), np.array(5 * MM))
    assert float(t_below) < float(t_above)
    assert abs(_fermat_time(med, 10.25 * MM, 5 * MM) - float(t_below)) <= 1e-12 * float(t_below)
