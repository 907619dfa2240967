"""Pins of the oracle's operator A (Eqs. (11), (13)), its transpose and the
direct-arrival basis D (Eq. (1)): the adjoint identity between two separately
written sums, the dense matrix, linearity, single-voxel impulse responses
against the analytic pulse, and window support."""
import numpy as np
import pytest

from synth import card_c1, tiny_card, random_vector
from oracle import operator, geometry, pulse


def _inner(a, b):
    return float(np.sum(np.asarray(a) * np.asarray(b)))


@pytest.mark.parametrize("mk,kw", [(tiny_card, {}), (tiny_card, {"n_layers": 3}),
                                   (tiny_card, {"n_layers": 4, "beta": 3}), (card_c1, {})])
def test_adjoint_identity(mk, kw):
    """<A x, r> = <x, A^T r>: the forward scatters with bincount, the adjoint
    gathers window by window, so a slip in either breaks the identity."""
    card = mk(**kw)
    g = card.grid
    a = card.array
    x = random_vector((g.nz, g.nx), seed=1)
    r = random_vector((a.n_scans, a.n_rx, card.acq.n_samples), seed=2)
    lhs = _inner(operator.forward(card, x), r)
    rhs = _inner(x, operator.adjoint(card, r))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(r) * 1e-3)


def test_dense_matrix_matches_matrix_free():
    card = tiny_card(n_layers=3)
    amat = operator.dense(card)
    g = card.grid
    x = random_vector((g.nz, g.nx), seed=3)
    np.testing.assert_allclose(amat @ x.reshape(-1), operator.forward(card, x).reshape(-1),
                               rtol=0, atol=1e-12)
    r = random_vector(amat.shape[0], seed=4)
    np.testing.assert_allclose(amat.T @ r,
                               operator.adjoint(card, r.reshape(operator.forward(card, x).shape)).reshape(-1),
                               rtol=0, atol=1e-12)


def test_linearity():
    card = tiny_card(n_layers=2)
    g = card.grid
    x1 = random_vector((g.nz, g.nx), seed=5)
    x2 = random_vector((g.nz, g.nx), seed=6)
    lhs = operator.forward(card, 2.0 * x1 - 0.5 * x2)
    rhs = 2.0 * operator.forward(card, x1) - 0.5 * operator.forward(card, x2)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12)


def test_single_voxel_single_layer_impulse():
    """One layer, one voxel: trace (i, j) is W s(t - (R_tx + R_rx)/c) with W the
    straight-ray apodization, sampled; compared against the analytic pulse
    (written here from its definition) within the interpolation bound, and its
    envelope peaks near T + t_c."""
    card = tiny_card(n_layers=1, nx=8, nz=6, n_scans=1, n_rx=2, beta=2, n_samples=256)
    g, acq = card.grid, card.acq
    row, col = 4, 5
    x = np.zeros((g.nz, g.nx))
    x[row, col] = 1.0
    y = operator.forward(card, x)
    z = geometry.voxel_depths(g)[row]
    xv = geometry.voxel_laterals(g)[col]
    c = card.medium.speed[0]
    tc = acq.t_win / 2
    h = 1.0 / (acq.oversample * acq.fs)
    bound = h * h * (2 * np.pi * acq.f_c + 1 / acq.sigma_t) ** 2 / 8
    for j in range(2):
        xt = card.array.tx_x[0]
        xr = geometry.receiver_x(card, 0, j)
        rt, rr = np.hypot(z, xv - xt), np.hypot(z, xv - xr)
        T = (rt + rr) / c
        W = (z / rt) ** 2 * (z / rr) ** 2
        t = np.arange(acq.n_samples) / acq.fs - T
        u = t - tc
        s = np.sin(2 * np.pi * acq.f_c * u) * np.exp(-u * u / (2 * acq.sigma_t ** 2))
        s = np.where((t > 0) & (t < acq.t_win), s, 0.0)
        np.testing.assert_allclose(y[0, j], W * s, rtol=0, atol=W * bound)
        peak_t = np.argmax(np.abs(y[0, j])) / acq.fs
        assert abs(peak_t - (T + tc)) < 1.0 / acq.f_c


def test_window_support_per_voxel():
    """A voxel's echo occupies only samples m with 0 < m - fs T < L_h."""
    card = card_c1()
    g, acq = card.grid, card.acq
    lh = pulse.window_samples(acq)
    for v in (0, 777, 2080, 4095):
        x = np.zeros(g.nz * g.nx)
        x[v] = 1.0
        y = operator.forward(card, x.reshape(g.nz, g.nx))
        for j in range(card.array.n_rx):
            d, _, _ = geometry.trace_geometry(card, 0, j, [v])
            m = np.nonzero(y[0, j])[0]
            if len(m):
                assert m.min() > d[0] and m.max() < d[0] + lh


def test_abs_operator_dominates():
    """|A| (built from |W| and |b|) bounds A entrywise, so |A|^T |A| 1 >= diag(A^T A)."""
    card = tiny_card(n_layers=3)
    amat = operator.dense(card)
    babs = operator.abs_template(card.acq)
    g = card.grid
    ones = np.ones((g.nz, g.nx))
    col = operator.forward(card, ones, b=babs, weight_abs=True)
    den = operator.adjoint(card, col, b=babs, weight_abs=True).reshape(-1)
    diag = np.sum(amat ** 2, axis=0)
    assert np.all(den >= diag * (1 - 1e-12))
    # and row sums of |A| equal the |A| forward of ones
    np.testing.assert_allclose(np.abs(amat).sum(axis=1), col.reshape(-1), rtol=1e-12, atol=1e-15)


def test_direct_basis_is_delayed_template():
    """Column (i, j) of D is the template starting at |x_rx - x_tx| / c_1."""
    card = tiny_card(n_layers=2, n_scans=2, n_rx=3, n_samples=256)
    acq = card.acq
    d = operator.direct_basis(card)
    for i in range(2):
        for j in range(3):
            dist = abs(card.array.rx_offset[j])
            t0 = dist / card.medium.speed[0]
            t = np.arange(acq.n_samples) / acq.fs - t0
            nz = np.nonzero(d[i, j])[0]
            assert np.all((t[nz] > 0) & (t[nz] < acq.t_win))
    g = np.arange(6, dtype=float).reshape(2, 3)
    np.testing.assert_array_equal(operator.apply_direct(card, g), d * g[:, :, None])
