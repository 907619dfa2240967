"""Scheduler logic of the continuous-batching server, on the CPU with a
simulated executor: admission by HBM budget and slots in arrival order,
rejection of requests that can never fit, chunked interleaving, and
completion of every request exactly once."""
import pytest

from paper_2202_09703_amd.serve import Server, Request, make_requests, summarize


class FakeExecutor:
    """One simulated device executing queued chunks in submission order.
    Per-iteration time and bytes depend on the request kind."""

    T_ITER = {"small": 0.001, "big": 0.02}
    BYTES = {"small": 100, "big": 900}

    def __init__(self):
        self.t = 0.0
        self.device_free = 0.0
        self.done_at = {}
        self.log = []
        self.live_bytes = 0
        self.max_live = 0

    def now(self):
        return self.t

    def wait(self, dt):
        self.t += dt if dt > 0 else 1e-4

    def bytes_needed(self, req):
        return self.BYTES[req.kind]

    def start(self, req):
        self.live_bytes += self.BYTES[req.kind]
        self.max_live = max(self.max_live, self.live_bytes)
        h = {"req": req, "iters": 0}
        self.done_at[id(h)] = self.t
        return h

    def advance(self, h, n):
        begin = max(self.t, self.device_free)
        self.device_free = begin + n * self.T_ITER[h["req"].kind]
        self.done_at[id(h)] = self.device_free
        h["iters"] += n
        self.log.append((h["req"].rid, n))

    def idle(self, h):
        return self.t >= self.done_at[id(h)]

    def finish(self, h):
        return ("x", h["req"].rid, h["iters"]), None

    def release(self, h):
        self.live_bytes -= self.BYTES[h["req"].kind]


def _reqs(specs):
    return [Request(rid=i, arrival=a, n_iter=n, card=None, prior=None, sigma=1.0, kind=k)
            for i, (a, k, n) in enumerate(specs)]


def test_all_complete_once_within_budget():
    specs = [(0.001 * i, "big" if i % 5 == 0 else "small", 20 + i % 7) for i in range(40)]
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=1200, max_slots=4, chunk=5)
    res = srv.run(_reqs(specs))
    assert sorted(r.rid for r in res) == list(range(40))
    assert all(r.x[2] == specs[r.rid][2] for r in res)  # exactly n_iter iterations each
    assert srv.peak_bytes <= 1200 and ex.max_live <= 1200
    assert srv.peak_slots <= 4
    assert all(r.finished >= r.admitted >= r.arrival for r in res)


def test_admission_in_arrival_order():
    specs = [(0.0, "big", 30), (0.0001, "big", 30), (0.0002, "small", 10), (0.0003, "small", 10)]
    srv = Server(FakeExecutor(), hbm_budget=1000, max_slots=8, chunk=5)
    res = srv.run(_reqs(specs))
    adm = [r.admitted for r in sorted(res, key=lambda r: r.rid)]
    # the second big request must wait for the first; the small ones may not overtake it
    assert adm == sorted(adm)
    assert adm[1] > adm[0] and adm[2] >= adm[1]


def test_oversized_request_rejected():
    specs = [(0.0, "big", 10), (0.0, "small", 10)]
    srv = Server(FakeExecutor(), hbm_budget=500, max_slots=2, chunk=5)
    res = srv.run(_reqs(specs))
    assert srv.rejected == [0]
    assert [r.rid for r in res] == [1]


def test_small_requests_overtake_a_long_one_in_time():
    """Continuous batching: small requests arriving while a long one runs are
    admitted at once and finish long before it (chunks interleave)."""
    specs = [(0.0, "big", 50)] + [(0.01 + 0.001 * i, "small", 20) for i in range(5)]
    res = Server(FakeExecutor(), hbm_budget=2000, max_slots=8, chunk=5).run(_reqs(specs))
    big = res[0]
    assert all(r.finished < big.finished for r in res[1:])
    # one at a time (a single slot), each small request would wait for the big one
    res1 = Server(FakeExecutor(), hbm_budget=2000, max_slots=1, chunk=5).run(_reqs(specs))
    assert all(r.finished > res1[0].finished for r in res1[1:])
    assert summarize(res)["p50_ms"] < summarize(res1)["p50_ms"]


def test_chunking_respects_iteration_counts():
    ex = FakeExecutor()
    Server(ex, hbm_budget=2000, max_slots=2, chunk=7).run(_reqs([(0.0, "small", 23), (0.0, "small", 5)]))
    per = {}
    for rid, n in ex.log:
        per.setdefault(rid, []).append(n)
    assert per[0] == [7, 7, 7, 2] and per[1] == [5]


def test_chunk_per_kind():
    """A mapping gives each kind its own chunk; kinds not listed take 5."""
    ex = FakeExecutor()
    Server(ex, hbm_budget=2000, max_slots=3, chunk={"small": 11}).run(
        _reqs([(0.0, "small", 23), (0.0, "big", 12)]))
    per = {}
    for rid, n in ex.log:
        per.setdefault(rid, []).append(n)
    assert per[0] == [11, 11, 1] and per[1] == [5, 5, 2]
    with pytest.raises(ValueError):
        Server(FakeExecutor(), hbm_budget=10, chunk={"small": 0})


def test_summary_per_kind():
    res = Server(FakeExecutor(), hbm_budget=2000, max_slots=8, chunk=5).run(
        _reqs([(0.0, "big", 40), (0.001, "small", 5), (0.002, "small", 5)]))
    s = summarize(res)
    assert set(s["per_kind"]) == {"big", "small"} and s["per_kind"]["small"]["requests"] == 2
    assert s["per_kind"]["small"]["p99_ms"] <= s["per_kind"]["big"]["p99_ms"]


def test_arrivals_are_seeded_poisson():
    a = make_requests(500, rate_hz=100.0, seed=5)
    b = make_requests(500, rate_hz=100.0, seed=5)
    assert a == b
    gaps = [y["arrival"] - x["arrival"] for x, y in zip(a, a[1:])]
    mean = sum(gaps) / len(gaps)
    assert abs(mean - 0.01) < 0.0015
    kinds = [s["kind"] for s in a]
    assert abs(kinds.count("c1") / 500 - 0.5) < 0.07
    assert all(20 <= s["n_iter"] <= 50 for s in a)


def test_bad_configuration():
    with pytest.raises(ValueError):
        Server(FakeExecutor(), hbm_budget=10, chunk=0)
