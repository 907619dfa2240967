"""Reduced-precision storage (FP16 / BF16 traces, fine grid and taps, FP32
accumulation) against the FP64 oracle on the same seeded inputs.

Error model.  With unit roundoff u of the storage format (2^-11 for FP16,
2^-8 for BF16) a forward result carries three independent roundings: the fine
grid bin, the template tap and the stored output, each of relative size <= u
and of RMS size about u/sqrt(3), so the relative L2 error is about u; the bound
is 4u.
The adjoint takes its input already rounded to the format (one rounding of r),
rounds the correlated fine grid once more and accumulates in FP32: bound 4u.
A reconstruction on rounded data amplifies the data error by the conditioning
of the surrogate iteration; over the c1 workload's 20 iterations the bound is
32u on the image and 8u on the cost history."""
import dataclasses

import numpy as np
import pytest

from synth import card_c1, tiny_card, random_vector, phantom
from oracle import operator as oo, solver as osv, data as odata

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
umbir = pytest.importorskip("paper_2202_09703_amd.umbir")

MODES = [("f16", umbir.STORAGE_F16, 2.0 ** -11), ("bf16", umbir.STORAGE_BF16, 2.0 ** -8)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def with_storage(card, st):
    return dataclasses.replace(card, acq=dataclasses.replace(card.acq, storage=st))


def traces(a, geom, dev):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device=dev).to(geom.trace_dtype)


def f32(a, dev):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)


def host(t):
    return t.float().cpu().numpy()


# 16-bit storage takes oversampling factors 32 and 64 (the matrix-core tiles)
CARDS = [("tiny-1layer", tiny_card(n_layers=1, oversample=32)),
         ("tiny-3layer", tiny_card(n_layers=3, beta=3, oversample=32)),
         ("tiny-ragged", tiny_card(n_layers=3, nx=17, nz=13, n_scans=3, n_rx=4, n_samples=300, oversample=32)),
         ("tiny-short", tiny_card(n_layers=3, n_samples=40, oversample=32)),
         ("c1", card_c1())]


@pytest.mark.parametrize("mode,st,u", MODES)
@pytest.mark.parametrize("name,card", CARDS)
def test_forward_and_adjoint_error(dev, mode, st, u, name, card):
    card = with_storage(card, st)
    geom = umbir.build_geometry(card)
    assert geom.storage == st and geom.trace_dtype != torch.float32
    g = card.grid
    x = random_vector((g.nz, g.nx), seed=11)
    y = umbir.forward(geom, f32(x, dev))
    assert y.dtype == geom.trace_dtype
    ef = rel(host(y), oo.forward(card, x))
    r = random_vector(geom.trace_shape, seed=21)
    xa = host(umbir.adjoint(geom, traces(r, geom, dev)))
    ea = rel(xa, oo.adjoint(card, r))
    print(f"{name} {mode}: forward rel L2 {ef:.2e}, adjoint rel L2 {ea:.2e} (u = {u:.1e})")
    assert ef <= 4 * u and ea <= 4 * u
    # accumulate mode
    y0 = traces(random_vector(geom.trace_shape, seed=13), geom, dev)
    y1 = host(umbir.forward(geom, f32(x, dev), y0.clone(), accumulate=True))
    assert rel(y1, host(y0) + oo.forward(card, x)) <= 4 * u


@pytest.mark.parametrize("mode,st,u", MODES)
def test_phantom_forward_and_determinism(dev, mode, st, u):
    card = with_storage(card_c1(), st)
    geom = umbir.build_geometry(card)
    x = f32(phantom(card), dev)
    y = umbir.forward(geom, x)
    assert torch.equal(y, umbir.forward(geom, x))
    r = traces(random_vector(geom.trace_shape, seed=31), geom, dev)
    assert torch.equal(umbir.adjoint(geom, r), umbir.adjoint(geom, r))
    e = rel(host(y), oo.forward(card, phantom(card)))
    print(f"c1 {mode}: phantom forward rel L2 {e:.2e}")
    assert e <= 4 * u


@pytest.mark.parametrize("mode,st,u", MODES)
def test_direct_and_denominator(dev, mode, st, u):
    card = with_storage(tiny_card(n_layers=3, nx=12, nz=10, n_scans=2, n_rx=3, n_samples=200,
                                  oversample=32), st)
    geom = umbir.build_geometry(card)
    gdir = np.array([[0.5, -0.3, 0.8], [0.2, 0.9, -0.4]])
    yd = host(umbir.direct(geom, f32(gdir, dev)))
    e = rel(yd, oo.apply_direct(card, gdir))
    d = umbir.sqs_denominator(geom, 0.01).cpu().numpy()
    ed = rel(d, osv.sqs_denominator(card, 0.01))
    print(f"{mode}: direct rel L2 {e:.2e}, sqs denominator rel L2 {ed:.2e}")
    assert e <= 2 * u and ed <= 4 * u


@pytest.mark.parametrize("mode,st,u", MODES)
def test_reconstruct_error_c1(dev, mode, st, u):
    """20 iterations on 16-bit data against the oracle's FP64 iteration on the
    unrounded data: the whole error the storage format costs."""
    base = card_c1()
    x_true, y, sigma = odata.synthesize(base)
    card = with_storage(base, st)
    geom = umbir.build_geometry(card)
    n = base.n_iter
    x, g, cost = umbir.reconstruct(geom, base.prior, sigma, traces(y, geom, dev), n)
    xo, go, co = osv.sqs(base, y, sigma, base.prior, n)
    xe = rel(x.cpu().numpy(), xo)
    ce = float(np.max(np.abs(cost.cpu().numpy() - co) / np.abs(co)))
    te = rel(x.cpu().numpy(), x_true)
    to = rel(xo, x_true)
    print(f"c1 recon {mode}: x rel L2 vs oracle {xe:.2e}, max cost rel err {ce:.2e}; "
          f"distance to truth {te:.4f} (oracle {to:.4f})")
    assert xe <= 32 * u and ce <= 8 * u
    # a resident session on 16-bit data reproduces the one-shot result bitwise
    sess = umbir.Solver(geom, base.prior, sigma, traces(y, geom, dev), max_iter=n)
    sess.step(n)
    xs, gs, cs = sess.read()
    assert torch.equal(xs, x) and torch.equal(cs, cost)
    sess.free()


@pytest.mark.parametrize("mode,st,u", MODES)
def test_c3_sampled(dev, mode, st, u):
    from synth import card_c3
    card = with_storage(card_c3(), st)
    geom = umbir.build_geometry(card)
    x = phantom(card)
    y = host(umbir.forward(geom, f32(x, dev)))
    tr = [(5, 3), (40, 30)]
    ref = oo.forward(card, x, traces=tr)
    for i, j in tr:
        e = rel(y[i, j], ref[i, j])
        print(f"c3 {mode} forward trace ({i},{j}) rel L2 {e:.2e}")
        assert e <= 4 * u
    r = random_vector(geom.trace_shape, seed=61)
    xa = host(umbir.adjoint(geom, traces(r, geom, dev))).reshape(-1)
    vox = np.random.default_rng(7).choice(card.n_voxels, 6, replace=False)
    e = rel(xa[vox], oo.adjoint_voxels(card, r, vox))
    print(f"c3 {mode} adjoint sampled rel L2 {e:.2e}")
    assert e <= 4 * u

