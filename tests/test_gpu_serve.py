"""The continuous-batching server on the GPU: every request completes, its
result is bitwise the one-request-at-a-time result (alone vs in the mix), and
the admitted set respects the HBM budget."""
import numpy as np
import pytest

from synth import card_c1, tiny_card

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
umbir = pytest.importorskip("paper_2202_09703_amd.umbir")
from paper_2202_09703_amd import serve  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_served_equals_alone(dev):
    cards = {"c1": card_c1(), "t3": tiny_card(n_layers=3, nx=16, nz=12, n_scans=2, n_rx=3, n_samples=192),
             "t4": tiny_card(n_layers=4, nx=20, nz=14, n_scans=3, n_rx=2, n_samples=256)}
    specs = [{"rid": i, "arrival": 0.002 * i, "kind": k, "n_iter": n}
             for i, (k, n) in enumerate([("c1", 12), ("t3", 7), ("t4", 9), ("t3", 3), ("c1", 5),
                                         ("t4", 11), ("t3", 8), ("c1", 6)])]
    reqs = serve.synthesize(umbir, cards, specs)
    ex = serve.GpuExecutor(umbir)
    budget = max(ex.bytes_needed(r) for r in reqs) * 2
    srv = serve.Server(ex, hbm_budget=budget, max_slots=4, chunk=3)
    served = srv.run(reqs)
    plain = serve.plain_run(umbir, reqs)
    assert [r.rid for r in served] == list(range(len(specs)))
    assert srv.peak_bytes <= budget and not srv.rejected
    for a, b in zip(served, plain):
        assert torch.equal(a.x, b.x), f"request {a.rid}"
        assert torch.equal(a.cost, b.cost)
    s = serve.summarize(served)
    assert s["requests"] == len(specs) and np.isfinite(s["p99_ms"])
