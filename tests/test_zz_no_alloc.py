"""umbir_reconstruct_noalloc (the reconstruction with the library's static
device scratch as workspace) through the C ABI, against umbir_reconstruct with
its own workspace: bitwise the same image, direct-arrival weights and cost
history, on two calls in a row (the second on a smaller problem, so the
scratch holds the first call's data when it starts), plus the size limit."""
import numpy as np
import pytest

from synth import card_c1, card_c2, tiny_card
from oracle import data as odata, operator as oo

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
umbir = pytest.importorskip("paper_2202_09703_amd.umbir")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _case(card, dev, direct=False):
    _, y, sigma = odata.synthesize(card)
    if direct:
        a = card.array
        y = y + oo.apply_direct(card, np.linspace(-0.5, 0.7, card.n_traces).reshape(a.n_scans, a.n_rx))
    geom = umbir.build_geometry(card)
    return geom, torch.tensor(y, dtype=torch.float32, device=dev), sigma


def _both(geom, card, sigma, yt, n, dev):
    ref = umbir.reconstruct(geom, card.prior, sigma, yt, n)
    x = torch.zeros(geom.image_shape, dtype=torch.float32, device=dev)
    g = torch.zeros(geom.trace_shape[:2], dtype=torch.float32, device=dev)
    cost = torch.empty(n + 1, dtype=torch.float64, device=dev)
    got = umbir.reconstruct_noalloc(geom, card.prior, sigma, yt, n, x, g, cost)
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_equals_reconstruct_twice(dev):
    big = card_c1()
    small = tiny_card(n_layers=3, nx=12, nz=10, n_scans=2, n_rx=3, n_samples=200)
    for card, n, direct in ((big, 12, False), (small, 7, True)):
        geom, yt, sigma = _case(card, dev, direct)
        assert geom.workspace_bytes(umbir.WORK_RECONSTRUCT) <= umbir.NOALLOC_SCRATCH_BYTES
        (xr, gr, cr), (x, g, c) = _both(geom, card, sigma, yt, n, dev)
        print(f"{card.name}: {n} iterations, noalloc vs reconstruct max |dx| "
              f"{float((x - xr).abs().max()):.3e}")
        assert torch.equal(x, xr) and torch.equal(g, gr) and torch.equal(c, cr)
        geom.free()


def test_noalloc_rejects_a_problem_beyond_the_scratch(dev):
    # 512 traces x 2048 samples x Q = 32 of fine grid fits; double the record does not
    import dataclasses
    card = card_c2()
    card = dataclasses.replace(card, acq=dataclasses.replace(card.acq, n_samples=4096))
    geom = umbir.build_geometry(card)
    assert geom.workspace_bytes(umbir.WORK_RECONSTRUCT) > umbir.NOALLOC_SCRATCH_BYTES
    y = torch.zeros(geom.trace_shape, dtype=torch.float32, device=dev)
    x = torch.zeros(geom.image_shape, dtype=torch.float32, device=dev)
    g = torch.zeros(geom.trace_shape[:2], dtype=torch.float32, device=dev)
    cost = torch.empty(2, dtype=torch.float64, device=dev)
    with pytest.raises(umbir.UmbirError) as err:
        umbir.reconstruct_noalloc(geom, card.prior, 0.1, y, 1, x, g, cost)
    assert err.value.status == umbir.ENOTSUP
    assert "static scratch" in str(err.value)
    geom.free()


def test_noalloc_on_the_plain_256x256_workload(dev):
    """The benchmark problem fits the scratch: 3 iterations equal
    umbir_reconstruct's bitwise (data: seeded noise)."""
    from synth import noise
    card = card_c2()
    geom = umbir.build_geometry(card)
    need = geom.workspace_bytes(umbir.WORK_RECONSTRUCT)
    print(f"256x256 workload: {need / 2**20:.1f} MiB of scratch")
    assert need <= umbir.NOALLOC_SCRATCH_BYTES
    yt = torch.tensor(noise(card), dtype=torch.float32, device=dev)
    (xr, gr, cr), (x, g, c) = _both(geom, card, 0.05, yt, 3, dev)
    assert torch.equal(x, xr) and torch.equal(g, gr) and torch.equal(c, cr)
    geom.free()
