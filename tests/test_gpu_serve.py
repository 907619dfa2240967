"""The continuous-batching server on the GPU: every request completes, its
result is bitwise the one-request-at-a-time result (alone vs in the mix) and
matches the FP64 oracle's surrogate iteration (image 1e-5 relative L2, cost
history 1e-6), and the admitted set respects the HBM budget."""
import numpy as np
import pytest

from synth import card_c1, tiny_card
from oracle import data as odata, solver as osv

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
    host = {k: odata.synthesize(c)[1:] for k, c in cards.items()}
    reqs = serve.synthesize(umbir, cards, specs, host_data=host)
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
    # the oracle: one run per kind to its longest request, with every iterate
    ref = {}
    for k, c in cards.items():
        n = max(sp["n_iter"] for sp in specs if sp["kind"] == k)
        y, sigma = host[k]
        _, _, co, its = osv.sqs(c, y, sigma, c.prior, n, history=True)
        ref[k] = (co, its)
    for r, sp in zip(served, specs):
        co, its = ref[sp["kind"]]
        n = sp["n_iter"]
        xo = its[n - 1][0]
        x = r.x.cpu().numpy().astype(np.float64)
        xe = float(np.linalg.norm(x - xo) / np.linalg.norm(xo))
        ce = float(np.max(np.abs(r.cost.cpu().numpy() - co[:n + 1]) / np.abs(co[:n + 1])))
        print(f"request {r.rid} ({sp['kind']}, {n} iterations): x {xe:.2e}, cost {ce:.2e}")
        assert xe <= 1e-5 and ce <= 1e-6
