"""Launch-shape tuning and batched sessions (many problems advanced by one
graph launch per iteration) through the C ABI."""
import dataclasses

import numpy as np
import pytest

from synth import card_c1, tiny_card, random_vector
from oracle import data as odata, solver as osv

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
umbir = pytest.importorskip("paper_2202_09703_amd.umbir")
batch = pytest.importorskip("paper_2202_09703_amd.batch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def f32(a, dev):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)


@pytest.mark.parametrize("name,card", [("tiny", tiny_card(n_layers=3, nx=17, nz=13, n_scans=3, n_rx=4)),
                                       ("tiny-q32", tiny_card(n_layers=3, nx=17, nz=13, n_scans=3, n_rx=13,
                                                              n_samples=700, oversample=32)),
                                       ("c1", card_c1())])
def test_tuning_changes_no_result(dev, name, card):
    """Any splat split, convolution tile order, correlation tile shape and
    workgroup count gives bitwise the same forward and adjoint; gather
    batches, the convolution's output tiles per workgroup and the form of the
    matrix-core products change only the order of sums."""
    geom = umbir.build_geometry(card)
    g = card.grid
    x = f32(random_vector((g.nz, g.nx), seed=3), dev)
    r = f32(random_vector(geom.trace_shape, seed=4), dev)
    y0, a0 = umbir.forward(geom, x), umbir.adjoint(geom, r)
    t0 = geom.tuning()
    assert t0["splat_blocks"] > 0 and t0["gather_batch_kb"] > 0
    assert t0["conv_grid"] == 1 and t0["corr_tile_rows"] == 128 and t0["corr_blocks"] == 512
    # bf16-piece products by default: 128-sample tiles when at least 256
    # workgroups remain, else 64 likewise, else 64 when 512 remain, else 32
    assert t0["products"] == 2
    tt, m = (geom.n_scans * geom.n_rx + 31) // 32, card.acq.n_samples
    rows = (128 if tt * ((m + 127) // 128) >= 256 else 64 if tt * ((m + 63) // 64) >= 256
            else 64 if tt * ((m + 63) // 64) >= 512 else 32)
    assert t0["conv_tile_rows"] == rows
    # FP32 products: the same operator to rounding
    geom.set_tuning(products=1)
    assert geom.tuning()["products"] == 1
    y1, a1 = umbir.forward(geom, x), umbir.adjoint(geom, r)
    for u, v in ((y1, y0), (a1, a0)):
        assert float(torch.linalg.norm((u - v).double()) / torch.linalg.norm(v.double())) <= 1e-6
    geom.set_tuning(products=2)
    assert torch.equal(umbir.forward(geom, x), y0)
    for cg, rows, nb in [(2, 32, 1), (1, 64, 100000), (2, 128, 7)]:
        geom.set_tuning(conv_grid=cg, corr_tile_rows=rows, corr_blocks=nb)
        assert torch.equal(umbir.forward(geom, x), y0)
        assert torch.equal(umbir.adjoint(geom, r), a0)
    for ct in (64, 128, t0["conv_tile_rows"]):
        geom.set_tuning(conv_tile_rows=ct)
        assert geom.tuning()["conv_tile_rows"] == ct
        y = umbir.forward(geom, x)
        assert torch.allclose(y, y0, rtol=1e-6, atol=1e-6 * float(y0.abs().max()))
        for cg in (1, 2):  # the tile order changes nothing for a given tile count
            geom.set_tuning(conv_grid=cg)
            assert torch.equal(umbir.forward(geom, x), y)
    for blocks, kb in [(1, 1), (geom.n_scans * geom.n_rx * 4, 64), (100000, 1 << 20)]:
        geom.set_tuning(splat_blocks=blocks, gather_batch_kb=kb)
        assert torch.equal(umbir.forward(geom, x), y0)
        a = umbir.adjoint(geom, r)
        assert torch.allclose(a, a0, rtol=1e-6, atol=1e-6 * float(a0.abs().max()))
    with pytest.raises(umbir.UmbirError) as err:
        geom.set_tuning(conv_grid=3)
    assert err.value.status == umbir.EINVAL
    with pytest.raises(umbir.UmbirError):
        geom.set_tuning(corr_tile_rows=48)
    with pytest.raises(umbir.UmbirError):
        geom.set_tuning(conv_tile_rows=96)
    with pytest.raises(umbir.UmbirError):
        geom.set_tuning(products=3)
    chosen = geom.autotune()
    assert chosen == geom.tuning() and chosen["splat_blocks"] > 0 and chosen["gather_batch_kb"] > 0
    if (chosen["operator_form"] == 1 and chosen["conv_tile_rows"] == t0["conv_tile_rows"]
            and chosen["products"] == t0["products"]):
        assert torch.equal(umbir.forward(geom, x), y0)
    else:  # the direct form, or other convolution tiles, sum in another order
        yd = umbir.forward(geom, x)
        assert float(torch.linalg.norm((yd - y0).double()) / torch.linalg.norm(y0.double())) <= 1e-5
    # zeros keep the current values; a cache reuses the choice for the same shape
    geom.set_tuning(0, 0)
    assert geom.tuning() == chosen
    cache = {}
    assert geom.autotune(cache=cache) == geom.autotune(cache=cache)
    assert len(cache) == 1


def _problems(dev):
    cards = [dataclasses.replace(tiny_card(n_layers=3, nx=12, nz=10, n_scans=2, n_rx=3, n_samples=200), n_iter=7),
             dataclasses.replace(tiny_card(n_layers=2, nx=17, nz=13, n_scans=3, n_rx=4, n_samples=300), n_iter=4),
             dataclasses.replace(card_c1(), n_iter=10)]
    return batch.prepare(umbir, cards, device=dev, log=lambda *a, **k: None)


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_equals_one_at_a_time(dev, mode):
    probs = _problems(dev)
    _, plain = batch.run_plain(umbir, probs)
    _, batched, rebuilds = batch.run_batched(umbir, probs, mode)
    assert rebuilds == 3  # the problems leave the batch at 4, 7 and 10 iterations
    for p, a, b in zip(probs, plain, batched):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), p["card"].name
        assert torch.equal(a[2], b[2]) and a[2].numel() == p["n_iter"] + 1
    # and the one-at-a-time session equals the one-shot reconstruction
    p = probs[2]
    x, g, cost = umbir.reconstruct(p["geom"], p["card"].prior, p["sigma"], p["y"], p["n_iter"])
    assert torch.equal(x, plain[2][0]) and torch.equal(cost, plain[2][2])


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_members_match_oracle(dev, mode):
    """Every member of a batch of uneven problems (data synthesised by the
    oracle) against the oracle's surrogate iteration for its own iteration
    count: image within 1e-5 relative L2, cost history within 1e-6."""
    cards = [dataclasses.replace(tiny_card(n_layers=3, nx=12, nz=10, n_scans=2, n_rx=3, n_samples=200), n_iter=7),
             dataclasses.replace(tiny_card(n_layers=2, nx=17, nz=13, n_scans=3, n_rx=4, n_samples=300), n_iter=4),
             dataclasses.replace(card_c1(), n_iter=10),
             dataclasses.replace(tiny_card(n_layers=4, nx=20, nz=14, n_scans=3, n_rx=2, n_samples=256,
                                           oversample=32), n_iter=6)]
    data = [odata.synthesize(c)[1:] for c in cards]
    probs = batch.prepare(umbir, cards, device=dev, log=lambda *a, **k: None, data=data)
    _, batched, _ = batch.run_batched(umbir, probs, mode)
    for c, (y, sigma), (x, g, cost) in zip(cards, data, batched):
        xo, go, co = osv.sqs(c, y, sigma, c.prior, c.n_iter)
        xe = rel(x.cpu().numpy(), xo)
        ce = float(np.max(np.abs(cost.cpu().numpy() - co) / np.abs(co)))
        print(f"{c.name} ({c.n_iter} iterations) in the batch: x {xe:.2e}, cost {ce:.2e}")
        assert xe <= 1e-5 and ce <= 1e-6
    for p in probs:
        p["geom"].free()


def _q_cards(q):
    """Uneven problems of one oversampling factor (work-list batches need one):
    up to and beyond 1024 voxels (both fixed-point conversions of the splat)."""
    return [dataclasses.replace(tiny_card(n_layers=3, nx=12, nz=10, n_scans=2, n_rx=3, n_samples=200,
                                          oversample=q), n_iter=7),
            dataclasses.replace(tiny_card(n_layers=2, nx=40, nz=30, n_scans=3, n_rx=4, n_samples=300,
                                          oversample=q), n_iter=4),
            dataclasses.replace(tiny_card(n_layers=4, nx=20, nz=14, n_scans=3, n_rx=2, n_samples=256,
                                          oversample=q), n_iter=6)]


@pytest.mark.parametrize("q", [32, 64])
def test_worklist_batch(dev, q):
    """The work-list batch (per lane one launch per stage over its problems'
    work items, problems leaving as they reach their count) holds bitwise each
    problem's one-at-a-time result, and that matches the oracle.  One problem
    runs with small splat chunks and one-trace gather batches, so its items
    cover several chunks and its gather items several batches; the problems
    take 32-, 64- and 128-sample convolution tiles, so the work list runs each
    with its own; two run the windowed gather (its own work-list stage) and
    the others the row-wise one."""
    cards = _q_cards(q) + ([dataclasses.replace(card_c1(), n_iter=5)] if q == 64 else [])
    data = [odata.synthesize(c)[1:] for c in cards]
    probs = batch.prepare(umbir, cards, device=dev, log=lambda *a, **k: None, data=data)
    probs[2]["geom"].set_tuning(splat_blocks=probs[2]["geom"].n_scans * probs[2]["geom"].n_rx * 4, gather_batch_kb=1)
    probs[0]["geom"].set_tuning(conv_tile_rows=64)
    probs[1]["geom"].set_tuning(conv_tile_rows=128, conv_grid=2)
    for i in (1, 2):
        probs[i]["geom"].set_tuning(gather_form=2)
    probs[0]["geom"].set_tuning(gather_form=1)
    _, plain = batch.run_plain(umbir, probs)
    _, wl, n_batches = batch.run_batched(umbir, probs, umbir.BATCH_WORKLIST)
    assert n_batches == 1
    for c, (y, sigma), a, b in zip(cards, data, plain, wl):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2]), c.name
        assert b[2].numel() == c.n_iter + 1
        xo, go, co = osv.sqs(c, y, sigma, c.prior, c.n_iter)
        xe = rel(b[0].cpu().numpy(), xo)
        ce = float(np.max(np.abs(b[2].cpu().numpy() - co) / np.abs(co)))
        print(f"{c.name} ({c.n_iter} iterations) in the work-list batch: x {xe:.2e}, cost {ce:.2e}")
        assert xe <= 1e-5 and ce <= 1e-6
    for p in probs:
        p["geom"].free()


def test_worklist_batch_rejections(dev):
    cards = [tiny_card(n_layers=3, oversample=32), tiny_card(n_layers=3, oversample=64)]
    probs = batch.prepare(umbir, cards, device=dev, log=lambda *a, **k: None)
    ss = batch.sessions(umbir, probs)
    with pytest.raises(umbir.UmbirError) as err:  # two oversampling factors
        umbir.Batch(ss, umbir.BATCH_WORKLIST)
    assert err.value.status == umbir.ENOTSUP
    for s in ss:
        s.free()
    probs8 = batch.prepare(umbir, [tiny_card(n_layers=3)], device=dev, log=lambda *a, **k: None)  # Q = 8
    ss = batch.sessions(umbir, probs8)
    with pytest.raises(umbir.UmbirError) as err:
        umbir.Batch(ss, umbir.BATCH_WORKLIST)
    assert err.value.status == umbir.ENOTSUP
    for s in ss:
        s.free()


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_guards(dev, mode):
    probs = _problems(dev)[:2]
    ss = batch.sessions(umbir, probs)
    b = umbir.Batch(ss, mode)
    b.step(2)
    torch.cuda.synchronize()
    assert [s.iterations for s in ss] == [2, 2]
    with pytest.raises(umbir.UmbirError):
        b.step(3)  # the second problem allows 4 iterations
    ss[0].step(1)  # stepped alone: the batch no longer matches it
    with pytest.raises(umbir.UmbirError):
        b.step(1)
    b.free()
    with pytest.raises(umbir.UmbirError):
        umbir.Batch([ss[0], ss[0]], mode)
    for s in ss:
        s.free()


def test_free_right_after_step_waits_for_the_launches(dev):
    """umbir_batch_free and umbir_solver_free wait for the graph launches they
    queued: a batch freed at once after a long step leaves its sessions' work
    intact, and equal to stepping them one at a time."""
    cards = [dataclasses.replace(card_c1(), n_iter=30), dataclasses.replace(card_c1(), n_iter=30)]
    probs = batch.prepare(umbir, cards, device=dev, log=lambda *a, **k: None)
    _, plain = batch.run_plain(umbir, probs)
    ss = batch.sessions(umbir, probs)
    b = umbir.Batch(ss, umbir.BATCH_GRAPH)
    b.step(30)
    b.free()
    out = [s.read() for s in ss]
    torch.cuda.synchronize()
    for a, o in zip(plain, out):
        assert torch.equal(a[0], o[0]) and torch.equal(a[2], o[2])
    for s in ss:
        s.free()
