"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.  Tolerance for float32 results: relative L2 <= 1e-5
(element by element on the sizes the oracle runs in seconds; on sampled
outputs at the full plain-FP32 workload)."""
import numpy as np
import pytest

from synth import card_c1, card_c2, tiny_card, random_vector, phantom
from synth.cards import Prior
from oracle import geometry as og, operator as oo, pulse as op, solver as osv, data as odata

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
umbir = pytest.importorskip("paper_2202_09703_amd.umbir")

TOL = 1e-5


def direct_arrival_bar(y_with, y_without):
    """Image bar on data with injected direct arrivals.  The FP32 residual
    e = y - A x - D g rounds every sample at about u |y|, so its rounding error
    grows with the size of the data it is formed from, while the part the image
    is fitted to (y without the direct arrivals) does not.  Without direct
    arrivals the surrogate iteration holds the image within 1e-6 of the oracle
    (measured 1e-7 to 3e-7); injected arrivals scale that rounding by
    rho = ||y_with|| / ||y_without||, so the bar is max(1e-5, 1e-6 rho)."""
    rho = float(np.linalg.norm(y_with) / np.linalg.norm(y_without))
    return max(TOL, 1e-6 * rho)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def t32(a, dev):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)


TINY = [dict(n_layers=1), dict(n_layers=2), dict(n_layers=3, beta=3), dict(n_layers=4),
        dict(n_layers=3, nx=17, nz=13, n_scans=3, n_rx=4, n_samples=300, oversample=16),
        dict(n_layers=2, nx=1, nz=1, n_scans=1, n_rx=1),
        dict(n_layers=3, oversample=1, beta=0),
        dict(n_layers=3, n_samples=40),  # record shorter than many echoes: truncation
        # matrix-core convolution and correlation: ragged record and trace count, short window
        dict(n_layers=3, nx=17, nz=13, n_scans=3, n_rx=4, n_samples=300, oversample=32),
        dict(n_layers=2, nx=9, nz=11, n_scans=2, n_rx=5, n_samples=130, oversample=64)]


def _cards():
    return [("tiny%d" % k, tiny_card(**kw)) for k, kw in enumerate(TINY)] + [("c1", card_c1())]


@pytest.mark.parametrize("name,card", _cards())
def test_leg_table(dev, name, card):
    geom = umbir.build_geometry(card)
    dl = geom.table(umbir.TABLE_DELAY).astype(np.float64) / 2.0 ** 32
    ap = geom.table(umbir.TABLE_APOD).astype(np.float64)
    depth = og.voxel_depths(card.grid)[:, None]
    X = np.arange(geom.n_off)[None, :] * card.grid.dx / 2
    T, th, _ = og.leg(card.medium, depth + 0 * X, X + 0 * depth)
    err = np.max(np.abs(dl - card.acq.fs * T))
    print(f"{name}: max leg delay error {err:.2e} samples")
    assert err < 1e-6
    np.testing.assert_allclose(ap, np.cos(th) ** card.array.beta, rtol=1e-6, atol=1e-7)
    tau = geom.table(umbir.TABLE_TAU)
    np.testing.assert_allclose(tau, og.transmittance(card.medium, og.voxel_depths(card.grid)), rtol=1e-6)


@pytest.mark.parametrize("name,card", _cards())
def test_bank_and_direct_basis(dev, name, card):
    geom = umbir.build_geometry(card)
    bank = geom.table(umbir.TABLE_BANK).astype(np.float64)
    assert bank.shape[0] == 1
    bank = bank[0]
    ref = op.template(card.acq)
    np.testing.assert_allclose(bank[:len(ref)], ref, rtol=0, atol=1e-7)
    assert np.all(bank[len(ref):] == 0)
    d = geom.table(umbir.TABLE_DBASIS)
    np.testing.assert_allclose(d, oo.direct_basis(card), rtol=0, atol=3e-7)


@pytest.mark.parametrize("name,card", _cards())
def test_forward_parity(dev, name, card):
    geom = umbir.build_geometry(card)
    g = card.grid
    for x in (phantom(card) if card.phantom.n_reflectors <= g.nx * g.nz // 8 else None,
              random_vector((g.nz, g.nx), seed=11)):
        if x is None:
            continue
        y = umbir.forward(geom, t32(x, dev)).cpu().numpy()
        ref = oo.forward(card, x)
        e = rel(y, ref)
        print(f"{name}: forward rel L2 {e:.2e}")
        assert e <= TOL
    # accumulate mode adds to what is there
    x = random_vector((g.nz, g.nx), seed=12)
    y0 = t32(random_vector(geom.trace_shape, seed=13), dev)
    y1 = umbir.forward(geom, t32(x, dev), y0.clone(), accumulate=True).cpu().numpy()
    assert rel(y1, y0.cpu().numpy() + oo.forward(card, x)) <= TOL


@pytest.mark.parametrize("name,card", _cards())
def test_adjoint_parity_and_identity(dev, name, card):
    geom = umbir.build_geometry(card)
    g = card.grid
    r = random_vector(geom.trace_shape, seed=21)
    xa = umbir.adjoint(geom, t32(r, dev)).cpu().numpy()
    ref = oo.adjoint(card, r)
    e = rel(xa, ref)
    print(f"{name}: adjoint rel L2 {e:.2e}")
    assert e <= TOL
    # the GPU pair is an exact transpose up to float rounding
    x = random_vector((g.nz, g.nx), seed=22)
    ax = umbir.forward(geom, t32(x, dev)).cpu().numpy().astype(np.float64)
    lhs, rhs = float(np.sum(ax * r)), float(np.sum(x * xa))
    scale = np.linalg.norm(ax) * np.linalg.norm(r)
    assert abs(lhs - rhs) <= TOL * scale


@pytest.mark.parametrize("name,card", [_cards()[3], ("c2", card_c2())])
def test_operators_are_deterministic(dev, name, card):
    """Both sweeps are bitwise reproducible: the adjoint sums in a fixed order
    and the forward's splat accumulates in fixed point."""
    geom = umbir.build_geometry(card)
    g = card.grid
    r = t32(random_vector(geom.trace_shape, seed=31), dev)
    assert torch.equal(umbir.adjoint(geom, r), umbir.adjoint(geom, r))
    x = t32(random_vector((g.nz, g.nx), seed=32), dev)
    assert torch.equal(umbir.forward(geom, x), umbir.forward(geom, x))


def test_forward_scale_extremes(dev):
    """The fixed-point splat scales by the largest |x|: tiny and huge images
    give the same relative accuracy."""
    card = tiny_card(n_layers=3)
    geom = umbir.build_geometry(card)
    g = card.grid
    x = random_vector((g.nz, g.nx), seed=33)
    ref = oo.forward(card, x)
    for scale in (1e-30, 1e-6, 1e6, 1e30):
        y = umbir.forward(geom, t32(x * scale, dev)).cpu().numpy().astype(np.float64) / scale
        assert rel(y, ref) <= TOL
    z = umbir.forward(geom, torch.zeros((g.nz, g.nx), dtype=torch.float32, device=dev))
    assert torch.count_nonzero(z) == 0


@pytest.mark.parametrize("name,card", _cards()[:3] + _cards()[-1:])
def test_direct_parity(dev, name, card):
    geom = umbir.build_geometry(card)
    gvals = random_vector(geom.trace_shape[:2], seed=41)
    y = umbir.direct(geom, t32(gvals, dev)).cpu().numpy()
    assert rel(y, oo.apply_direct(card, gvals)) <= TOL


@pytest.mark.parametrize("name,card", [_cards()[2], _cards()[-1]])
def test_sqs_denominator_parity(dev, name, card):
    geom = umbir.build_geometry(card)
    sigma = 0.01
    d = umbir.sqs_denominator(geom, sigma).cpu().numpy()
    e = rel(d, osv.sqs_denominator(card, sigma))
    print(f"{name}: sqs denominator rel L2 {e:.2e}")
    assert e <= TOL


def _recon_case():
    card = card_c1()
    x_true, y, sigma = odata.synthesize(card)
    return card, y, sigma


def test_reconstruct_parity_c1(dev):
    """20 iterations on the 64x64 workload: per-iteration cost and final image
    against the oracle's surrogate iteration."""
    card, y, sigma = _recon_case()
    geom = umbir.build_geometry(card)
    pr = card.prior
    n = card.n_iter
    x, g, cost = umbir.reconstruct(geom, pr, sigma, t32(y, dev), n)
    cost = cost.cpu().numpy()
    xo, go, co, its = osv.sqs(card, y, sigma, pr, n, history=True)
    ce = np.max(np.abs(cost - co) / np.abs(co))
    xe = rel(x.cpu().numpy(), xo)
    ge = rel(g.cpu().numpy(), go) if np.linalg.norm(go) > 0 else float(np.max(np.abs(g.cpu().numpy())))
    print(f"c1 recon: max cost rel err {ce:.2e}, x rel L2 {xe:.2e}, g err {ge:.2e}")
    assert ce <= 1e-6
    assert xe <= 1e-5
    # monotone within float32 rounding
    assert np.all(np.diff(cost) <= 1e-6 * np.abs(cost[:-1]))
    # one iteration, element by element
    x1, g1, _ = umbir.reconstruct(geom, pr, sigma, t32(y, dev), 1)
    assert rel(x1.cpu().numpy(), its[0][0]) <= TOL


def test_reconstruct_resume(dev):
    card, y, sigma = _recon_case()
    geom = umbir.build_geometry(card)
    yt = t32(y, dev)
    x20, g20, c20 = umbir.reconstruct(geom, card.prior, sigma, yt, 20)
    x10, g10, c10 = umbir.reconstruct(geom, card.prior, sigma, yt, 10)
    x2, g2, c2 = umbir.reconstruct(geom, card.prior, sigma, yt, 10, x=x10, g=g10)
    # the iteration keeps no state beyond (x, g) and every sweep is deterministic
    assert torch.equal(x2, x20) and torch.equal(g2, g20)
    assert torch.equal(c2, c20[10:])


def test_reconstruct_with_direct_arrivals(dev):
    """Data with injected direct arrivals: g is estimated and matches the oracle."""
    card = tiny_card(n_layers=3, nx=12, nz=10, n_scans=2, n_rx=3, n_samples=200)
    x_true, y, sigma = odata.synthesize(card)
    g_true = np.array([[0.5, -0.3, 0.8], [0.2, 0.9, -0.4]])
    y = y + oo.apply_direct(card, g_true)
    geom = umbir.build_geometry(card)
    x, g, cost = umbir.reconstruct(geom, card.prior, sigma, t32(y, dev), 8)
    xo, go, co = osv.sqs(card, y, sigma, card.prior, 8)
    bar = direct_arrival_bar(y, y - oo.apply_direct(card, g_true))
    xe = rel(x.cpu().numpy(), xo)
    print(f"recon with direct arrivals: x rel L2 {xe:.2e} (bar {bar:.2e})")
    assert rel(g.cpu().numpy(), go) <= 1e-5
    assert xe <= bar
    assert np.max(np.abs(cost.cpu().numpy() - co) / co) <= 1e-6


# ---- full-size plain FP32 workload (256x256, 32 x 16 traces, 2048 samples): sampled outputs


@pytest.fixture(scope="module")
def c2geom(dev):
    card = card_c2()
    return card, umbir.build_geometry(card)


def test_c2_forward_sampled(dev, c2geom):
    card, geom = c2geom
    x = phantom(card)
    y = umbir.forward(geom, t32(x, dev)).cpu().numpy()
    rng = np.random.default_rng(5)
    traces = [(int(rng.integers(card.array.n_scans)), int(rng.integers(card.array.n_rx))) for _ in range(3)]
    ref = oo.forward(card, x, traces=traces)
    for i, j in traces:
        e = rel(y[i, j], ref[i, j])
        print(f"c2 forward trace ({i},{j}) rel L2 {e:.2e}")
        assert e <= TOL


def test_c2_adjoint_sampled(dev, c2geom):
    card, geom = c2geom
    r = random_vector(geom.trace_shape, seed=51)
    xa = umbir.adjoint(geom, t32(r, dev)).cpu().numpy().reshape(-1)
    vox = np.random.default_rng(6).choice(card.n_voxels, 24, replace=False)
    ref = oo.adjoint_voxels(card, r, vox)
    e = rel(xa[vox], ref)
    print(f"c2 adjoint sampled rel L2 {e:.2e}")
    assert e <= TOL
    # property at full size: adjoint identity against the GPU forward
    x = random_vector((card.grid.nz, card.grid.nx), seed=52)
    ax = umbir.forward(geom, t32(x, dev)).cpu().numpy().astype(np.float64)
    lhs, rhs = float(np.sum(ax * r)), float(np.sum(x.reshape(-1) * xa))
    assert abs(lhs - rhs) <= TOL * np.linalg.norm(ax) * np.linalg.norm(r)


def test_c2_products_forms_at_fp32_level(dev, c2geom):
    """The matrix-core sweeps' two forms of an FP32 product (FP32 products;
    three bf16 pieces per factor, six piece products) both stay within FP32
    rounding of the FP64 oracle at full size: sampled traces and voxels to
    2e-6 relative (about 34 unit roundoffs; either form measures 3e-7 to 7e-7
    on these random inputs)."""
    card, geom = c2geom
    x = random_vector((card.grid.nz, card.grid.nx), seed=53)
    r = random_vector(geom.trace_shape, seed=54)
    traces = [(3, 7), (27, 12)]
    vox = np.random.default_rng(8).choice(card.n_voxels, 24, replace=False)
    fref, aref = oo.forward(card, x, traces=traces), oo.adjoint_voxels(card, r, vox)
    t0 = geom.tuning()
    try:
        for prod in (1, 2):
            geom.set_tuning(products=prod)
            y = umbir.forward(geom, t32(x, dev)).cpu().numpy()
            xa = umbir.adjoint(geom, t32(r, dev)).cpu().numpy().reshape(-1)
            fe = max(rel(y[i, j], fref[i, j]) for i, j in traces)
            ae = rel(xa[vox], aref)
            print(f"c2 products {prod}: forward {fe:.2e}, adjoint {ae:.2e}")
            assert fe <= 2e-6 and ae <= 2e-6
    finally:
        geom.set_tuning(products=t0["products"])


def test_c2_leg_table(dev, c2geom):
    card, geom = c2geom
    dl = geom.table(umbir.TABLE_DELAY).astype(np.float64) / 2.0 ** 32
    rows = np.arange(0, card.grid.nz, 7)
    depth = og.voxel_depths(card.grid)[rows][:, None]
    X = np.arange(geom.n_off)[None, :] * card.grid.dx / 2
    T, _, _ = og.leg(card.medium, depth + 0 * X, X + 0 * depth)
    err = np.max(np.abs(dl[rows] - card.acq.fs * T))
    print(f"c2 max leg delay error {err:.2e} samples")
    assert err < 1e-6


# ---- resident solver sessions (captured iteration graphs)


def test_solver_session_matches_reconstruct(dev):
    """A session stepped in chunks, with eager reads and synchronisations between
    the graph replays, holds bitwise the result of the one-shot reconstruction
    after every chunk."""
    card, y, sigma = _recon_case()
    geom = umbir.build_geometry(card)
    yt = t32(y, dev)
    sess = umbir.Solver(geom, card.prior, sigma, yt, max_iter=20)
    done = 0
    for chunk in (1, 4, 5, 10):
        sess.step(chunk)
        done += chunk
        xs, gs, cs = sess.read()
        torch.cuda.synchronize()
        xr, gr, cr = umbir.reconstruct(geom, card.prior, sigma, yt, done)
        torch.cuda.synchronize()
        assert torch.equal(xs, xr) and torch.equal(gs, gr), f"after {done} iterations"
        assert torch.equal(cs, cr)
    assert sess.iterations == 20
    with pytest.raises(umbir.UmbirError):
        sess.step(1)  # past max_iter
    sess.free()


def test_solver_session_warm_start_and_direct(dev):
    card = tiny_card(n_layers=3, nx=12, nz=10, n_scans=2, n_rx=3, n_samples=200)
    x_true, y, sigma = odata.synthesize(card)
    y = y + oo.apply_direct(card, np.array([[0.5, -0.3, 0.8], [0.2, 0.9, -0.4]]))
    geom = umbir.build_geometry(card)
    yt = t32(y, dev)
    x4, g4, _ = umbir.reconstruct(geom, card.prior, sigma, yt, 4)
    sess = umbir.Solver(geom, card.prior, sigma, yt, max_iter=4, x0=x4.clone(), g0=g4.clone())
    sess.step(4)
    xs, gs, cs = sess.read()
    x8, g8, c8 = umbir.reconstruct(geom, card.prior, sigma, yt, 8)
    assert torch.equal(xs, x8) and torch.equal(gs, g8)
    assert torch.equal(cs, c8[4:])
    xo, go, co = osv.sqs(card, y, sigma, card.prior, 8)
    g_true = np.array([[0.5, -0.3, 0.8], [0.2, 0.9, -0.4]])
    assert rel(xs.cpu().numpy(), xo) <= direct_arrival_bar(y, y - oo.apply_direct(card, g_true))


# ---- full-size 512x512 four-layer workload (2048 traces, 4096 samples): sampled outputs


@pytest.fixture(scope="module")
def c3geom(dev):
    from synth import card_c3
    card = card_c3()
    return card, umbir.build_geometry(card)


def test_c3_forward_and_adjoint_sampled(dev, c3geom):
    card, geom = c3geom
    x = phantom(card)
    y = umbir.forward(geom, t32(x, dev)).cpu().numpy()
    traces = [(5, 3), (40, 30)]
    ref = oo.forward(card, x, traces=traces)
    for i, j in traces:
        e = rel(y[i, j], ref[i, j])
        print(f"c3 forward trace ({i},{j}) rel L2 {e:.2e}")
        assert e <= TOL
    r = random_vector(geom.trace_shape, seed=61)
    xa = umbir.adjoint(geom, t32(r, dev)).cpu().numpy().reshape(-1)
    vox = np.random.default_rng(7).choice(card.n_voxels, 6, replace=False)
    refa = oo.adjoint_voxels(card, r, vox)
    e = rel(xa[vox], refa)
    print(f"c3 adjoint sampled rel L2 {e:.2e}")
    assert e <= TOL
    xr = random_vector((card.grid.nz, card.grid.nx), seed=62)
    ax = umbir.forward(geom, t32(xr, dev)).cpu().numpy().astype(np.float64)
    lhs, rhs = float(np.sum(ax * r)), float(np.sum(xr.reshape(-1) * xa))
    assert abs(lhs - rhs) <= TOL * np.linalg.norm(ax) * np.linalg.norm(r)


def test_c3_full_size_solver(dev, c3geom):
    card, geom = c3geom
    _full_size_solver_case(dev, card, geom, "c3", 8, 81)


# ---- full-size solver parity: curvature, one whole iteration, a whole scan
# position of the forward and a large voxel sample of the adjoint, against the
# oracle on all host cores (and, for the curvature, which needs Abar 1 over
# every voxel of every trace, against oracle values stored by
# tests/golden/make_full_size_samples.py)


def _golden(key):
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "full_size_samples.json")
    doc = json.load(open(path))
    if key not in doc:
        pytest.skip(f"no stored oracle samples for {key}")
    return np.array(doc[key]["voxels"], np.int64), np.array(doc[key]["abs_normal"])


def _full_size_solver_case(dev, card, geom, key, n_traces, seed):
    """d at the stored voxel samples; one reconstruct iteration from x = 0 on
    seeded data with injected direct arrivals (x^1 at the samples, g^1 in
    full, cost C(0, 0)); the forward of the given traces; the adjoint at the
    samples (all on every host core)."""
    vox, dstore = _golden(key)
    sigma = 0.05
    d = umbir.sqs_denominator(geom, sigma).cpu().numpy().reshape(-1)
    de = rel(d[vox], dstore / sigma ** 2)
    print(f"{key}: curvature at {len(vox)} voxels rel L2 {de:.2e}")
    assert de <= TOL
    a = card.array
    g_true = np.linspace(-0.4, 0.6, card.n_traces).reshape(a.n_scans, a.n_rx)
    y = 0.3 * random_vector(geom.trace_shape, seed=seed) + oo.apply_direct(card, g_true)
    x1, g1, c1 = umbir.reconstruct(geom, card.prior, sigma, t32(y, dev), 1)
    xo, go, co = osv.first_step_voxels(card, y, sigma, card.prior, vox, dstore / sigma ** 2, workers=None)
    xe = rel(x1.cpu().numpy().reshape(-1)[vox], xo)
    ge = rel(g1.cpu().numpy(), go)
    ce = abs(float(c1.cpu().numpy()[0]) - co) / co
    print(f"{key}: one iteration x^1 at {len(vox)} voxels {xe:.2e}, g^1 {ge:.2e}, cost[0] {ce:.2e}")
    assert xe <= TOL and ge <= TOL and ce <= 1e-6
    # the forward over whole receivers' traces of one scan position
    x = phantom(card)
    yf = umbir.forward(geom, t32(x, dev)).cpu().numpy()
    i = a.n_scans // 3
    traces = [(i, j) for j in range(min(n_traces, a.n_rx))]
    ref = oo.forward(card, x, traces=traces, workers=None)
    fe = rel(yf[i, :len(traces)], ref[i, :len(traces)])
    print(f"{key}: forward over scan position {i}, {len(traces)} traces, rel L2 {fe:.2e}")
    assert fe <= TOL
    # the adjoint at the voxel samples
    r = random_vector(geom.trace_shape, seed=seed + 1)
    xa = umbir.adjoint(geom, t32(r, dev)).cpu().numpy().reshape(-1)
    ae = rel(xa[vox], oo.adjoint_voxels(card, r, vox, workers=None))
    print(f"{key}: adjoint at {len(vox)} voxels rel L2 {ae:.2e}")
    assert ae <= TOL


def test_c2_full_size_solver(dev, c2geom):
    card, geom = c2geom
    _full_size_solver_case(dev, card, geom, "c2", 16, 71)


# ---- the direct (unfactored) form of the operator (umbir_tuning.operator_form = 2)


DIRECT = [("tiny3", tiny_card(n_layers=3, beta=3)),
          ("tiny4-ragged", tiny_card(n_layers=4, nx=17, nz=13, n_scans=3, n_rx=4, n_samples=300, oversample=16)),
          ("tiny-narrow", tiny_card(n_layers=3, nx=40, nz=30, n_scans=2, n_rx=3, n_samples=200, oversample=32)),
          ("tiny-short", tiny_card(n_layers=3, n_samples=40)),
          ("c1", card_c1())]


@pytest.mark.parametrize("name,card", DIRECT)
def test_direct_form_parity(dev, name, card):
    """A, A^T and the curvature in the direct form against the oracle; the
    forward stays bitwise reproducible (fixed-point sample sums)."""
    geom = umbir.build_geometry(card)
    geom.set_tuning(operator_form=2)
    assert geom.tuning()["operator_form"] == 2
    g = card.grid
    x = random_vector((g.nz, g.nx), seed=91)
    xt = t32(x, dev)
    y = umbir.forward(geom, xt)
    fe = rel(y.cpu().numpy(), oo.forward(card, x))
    r = random_vector(geom.trace_shape, seed=92)
    xa = umbir.adjoint(geom, t32(r, dev)).cpu().numpy()
    ae = rel(xa, oo.adjoint(card, r))
    d = umbir.sqs_denominator(geom, 0.01).cpu().numpy()
    de = rel(d, osv.sqs_denominator(card, 0.01))
    print(f"{name} direct form: forward {fe:.2e}, adjoint {ae:.2e}, curvature {de:.2e}")
    assert fe <= TOL and ae <= TOL and de <= TOL
    assert torch.equal(umbir.forward(geom, xt), y)
    y0 = t32(random_vector(geom.trace_shape, seed=93), dev)
    y1 = umbir.forward(geom, xt, y0.clone(), accumulate=True).cpu().numpy()
    assert rel(y1, y0.cpu().numpy() + oo.forward(card, x)) <= TOL


def test_direct_form_reconstruct_c1(dev):
    card, y, sigma = _recon_case()
    geom = umbir.build_geometry(card)
    geom.set_tuning(operator_form=2)
    x, g, cost = umbir.reconstruct(geom, card.prior, sigma, t32(y, dev), card.n_iter)
    xo, go, co = osv.sqs(card, y, sigma, card.prior, card.n_iter)
    xe = rel(x.cpu().numpy(), xo)
    ce = float(np.max(np.abs(cost.cpu().numpy() - co) / np.abs(co)))
    print(f"c1 direct-form reconstruction: x {xe:.2e}, cost {ce:.2e}")
    assert xe <= TOL and ce <= 1e-6


def test_direct_form_rejections(dev):
    import dataclasses
    geom = umbir.build_geometry(card_c2())  # 8 M + 4 (Q L_h + 2) = 16 KiB + 30 KiB fits
    geom.set_tuning(operator_form=2)
    long_rec = dataclasses.replace(card_c1(), acq=dataclasses.replace(card_c1().acq, n_samples=8192))
    g2 = umbir.build_geometry(long_rec)  # 64 KiB of samples alone
    with pytest.raises(umbir.UmbirError) as err:
        g2.set_tuning(operator_form=2)
    assert err.value.status == umbir.ENOTSUP
    with pytest.raises(umbir.UmbirError) as err:
        geom.set_tuning(operator_form=3)
    assert err.value.status == umbir.EINVAL
