"""Continuous-batching reconstruction server over resident solver sessions.

Requests (a problem, its data and an iteration count) arrive over time.  The
scheduler admits them in arrival order as soon as a slot is free and their
device bytes (geometry + solver session, from the library's own estimates)
fit the HBM budget; every admitted request gets its own HIP stream, and the
scheduler advances each one by a chunk of iterations whenever its previous
chunk has finished, so the work of all admitted requests overlaps on the
device and a new arrival starts at the next iteration boundary instead of
waiting for whole reconstructions ahead of it.  A request that could never
fit the budget alone is rejected.

The scheduling logic is independent of the device: `Server` drives an
executor with the small interface of `GpuExecutor`; tests drive it with a
simulated executor on the CPU.  `plain_run` is the one-request-at-a-time
reference path (one `reconstruct` call per request, in arrival order).

    python -m paper_2202_09703_amd.serve --requests 200   # the serving workload
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    n_iter: int
    card: Any                 # problem description (see umbir.Problem)
    prior: Any
    sigma: float
    y: Any = None             # device tensor [P][K][M]
    kind: str = ""


@dataclass
class Result:
    rid: int
    kind: str
    arrival: float
    admitted: float
    finished: float
    x: Any = None
    cost: Any = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class _Slot:
    req: Request
    handle: Any
    bytes: int
    admitted: float
    queued: int = 0           # iterations queued so far


class Server:
    """Continuous-batching scheduler.

    executor methods:  bytes_needed(req) -> int;  start(req) -> handle;
    advance(handle, n);  idle(handle) -> bool (queued work finished);
    finish(handle) -> (x, cost);  release(handle);  now() -> seconds;
    wait(dt) (sleep or advance a simulated clock)."""

    def __init__(self, executor, hbm_budget: int, max_slots: int = 8, chunk=5):
        """chunk: iterations queued per step of a request, one number or a
        mapping from request kind to number (kinds not listed take 5)."""
        chunks = chunk.values() if isinstance(chunk, dict) else [chunk]
        if any(int(c) < 1 for c in chunks) or max_slots < 1:
            raise ValueError("chunk and max_slots must be >= 1")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.chunk = dict(chunk) if isinstance(chunk, dict) else int(chunk)
        self.rejected: List[int] = []
        self.peak_bytes = 0
        self.peak_slots = 0

    def chunk_of(self, req: Request) -> int:
        if isinstance(self.chunk, dict):
            return int(self.chunk.get(req.kind, 5))
        return self.chunk

    def run(self, requests: List[Request]) -> List[Result]:
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        active: List[_Slot] = []
        results: List[Result] = []
        used = 0
        t0 = self.ex.now()
        while pending or active:
            now = self.ex.now() - t0
            # admit in arrival order (no overtaking: the head blocks later arrivals)
            while pending and pending[0].arrival <= now and len(active) < self.max_slots:
                req = pending[0]
                need = self.ex.bytes_needed(req)
                if need > self.budget:
                    self.rejected.append(req.rid)
                    pending.pop(0)
                    continue
                if used + need > self.budget:
                    break
                pending.pop(0)
                handle = self.ex.start(req)
                active.append(_Slot(req, handle, need, admitted=self.ex.now() - t0))
                used += need
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_slots = max(self.peak_slots, len(active))
            progressed = False
            for slot in list(active):
                if not self.ex.idle(slot.handle):
                    continue
                if slot.queued < slot.req.n_iter:
                    n = min(self.chunk_of(slot.req), slot.req.n_iter - slot.queued)
                    self.ex.advance(slot.handle, n)
                    slot.queued += n
                    progressed = True
                else:
                    x, cost = self.ex.finish(slot.handle)
                    done = self.ex.now() - t0
                    results.append(Result(slot.req.rid, slot.req.kind, slot.req.arrival, slot.admitted, done, x, cost))
                    self.ex.release(slot.handle)
                    used -= slot.bytes
                    active.remove(slot)
                    progressed = True
            if not progressed:
                nxt = pending[0].arrival - now if pending and not active else 0.0
                self.ex.wait(max(nxt, 0.0))
        return sorted(results, key=lambda r: r.rid)


class GpuExecutor:
    """Runs requests as resident solver sessions, one HIP stream each.  Geometries
    are cached per problem (they are immutable and shareable)."""

    def __init__(self, umbir, device: str = "cuda:0", poll: float = 20e-6):
        import torch
        self.torch = torch
        self.u = umbir
        self.device = torch.device(device)
        self.poll = poll
        self._geoms: Dict[str, Any] = {}

    def now(self) -> float:
        return time.perf_counter()

    def wait(self, dt: float):
        time.sleep(min(max(dt, 0.0), 1e-3) if dt > 0 else self.poll)

    def geometry(self, req: Request):
        key = req.kind or repr(req.card)
        g = self._geoms.get(key)
        if g is None:
            g = self.u.build_geometry(req.card)
            self._geoms[key] = g
        return g

    def bytes_needed(self, req: Request) -> int:
        g = self.geometry(req)
        return g.bytes + self.u.solver_bytes(g, req.n_iter)

    def start(self, req: Request):
        torch = self.torch
        g = self.geometry(req)
        stream = torch.cuda.Stream(device=self.device)
        ev = torch.cuda.Event()
        with torch.cuda.stream(stream):
            # the data were produced on the default stream
            stream.wait_stream(torch.cuda.default_stream(self.device))
            sess = self.u.Solver(g, req.prior, req.sigma, req.y, max_iter=req.n_iter, stream=stream)
            ev.record(stream)
        return {"sess": sess, "stream": stream, "event": ev}

    def advance(self, h, n: int):
        with self.torch.cuda.stream(h["stream"]):
            h["sess"].step(n, stream=h["stream"])
            h["event"].record(h["stream"])

    def idle(self, h) -> bool:
        return h["event"].query()

    def finish(self, h):
        with self.torch.cuda.stream(h["stream"]):
            x, g, cost = h["sess"].read(stream=h["stream"])
        h["stream"].synchronize()
        return x, cost

    def release(self, h):
        h["sess"].free()


def plain_run(umbir, requests: List[Request], now: Callable[[], float] = time.perf_counter,
              sleep: Callable[[float], None] = time.sleep) -> List[Result]:
    """One request at a time in arrival order: build the geometry, one
    reconstruct call, synchronise.  Latency includes the wait behind earlier requests."""
    import torch
    geoms: Dict[str, Any] = {}
    out = []
    t0 = now()
    for req in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        while now() - t0 < req.arrival:
            sleep(min(1e-3, req.arrival - (now() - t0)))
        start = now() - t0
        key = req.kind or repr(req.card)
        if key not in geoms:
            geoms[key] = umbir.build_geometry(req.card)
        x, g, cost = umbir.reconstruct(geoms[key], req.prior, req.sigma, req.y, req.n_iter)
        torch.cuda.synchronize()
        out.append(Result(req.rid, req.kind, req.arrival, start, now() - t0, x, cost))
    return out


def summarize(results: List[Result]) -> Dict[str, float]:
    lat = np.array([r.latency for r in results]) * 1e3
    span = max(r.finished for r in results) - min(r.arrival for r in results)
    out = {"requests": len(results), "p50_ms": float(np.percentile(lat, 50)),
           "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
           "recon_per_s": len(results) / span, "span_s": span}
    kinds = sorted({r.kind for r in results})
    if len(kinds) > 1:
        out["per_kind"] = {k: {"requests": int(sum(r.kind == k for r in results)),
                               "p50_ms": float(np.percentile([r.latency * 1e3 for r in results if r.kind == k], 50)),
                               "p99_ms": float(np.percentile([r.latency * 1e3 for r in results if r.kind == k], 99))}
                           for k in kinds}
    return out


# ---------------------------------------------------------------- workload

def make_requests(n: int, rate_hz: float, seed: int, mix=(("c1", 0.5), ("c2", 0.35), ("c3", 0.15)),
                  iters=(20, 50)) -> List[Dict[str, Any]]:
    """Seeded Poisson arrivals with a size mix and uniform iteration counts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = [k for k, _ in mix]
    probs = np.array([p for _, p in mix], float)
    probs /= probs.sum()
    t = 0.0
    out = []
    for rid in range(n):
        t += rng.exponential(1.0 / rate_hz)
        out.append({"rid": rid, "arrival": t, "kind": kinds[int(rng.choice(len(kinds), p=probs))],
                    "n_iter": int(rng.integers(iters[0], iters[1] + 1))})
    return out


def synthesize(umbir, cards: Dict[str, Any], specs, device="cuda:0", host_data=None) -> List[Request]:
    """Requests with data y = A x_true + sigma * noise made on the device (one
    geometry per kind); sigma from the card's SNR.  With `host_data`
    ({kind: (y [P][K][M], sigma)}) those data are copied to the device instead."""
    import torch
    from synth import phantom, noise
    data = {}
    for kind, card in cards.items():
        if host_data is not None:
            y, sigma = host_data[kind]
            data[kind] = (torch.tensor(y, dtype=torch.float32, device=device), float(sigma))
            continue
        g = umbir.build_geometry(card)
        xt = torch.tensor(phantom(card), dtype=torch.float32, device=device)
        clean = umbir.forward(g, xt)
        sigma = float(torch.sqrt(torch.mean(clean.double() ** 2) / 10.0 ** (card.snr_db / 10.0)))
        y = clean + sigma * torch.tensor(noise(card), dtype=torch.float32, device=device)
        data[kind] = (y, sigma)
        g.free()
    torch.cuda.synchronize()
    return [Request(s["rid"], s["arrival"], s["n_iter"], cards[s["kind"]], cards[s["kind"]].prior,
                    data[s["kind"]][1], data[s["kind"]][0], s["kind"]) for s in specs]


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--load", type=float, default=0.8, help="arrival rate as a fraction of plain-path capacity")
    ap.add_argument("--budget-gb", type=float, default=2.0)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--chunk", type=int, default=5, help="iterations per scheduling step (c2 and c3 requests)")
    ap.add_argument("--chunk-small", type=int, default=50,
                    help="iterations per scheduling step of the small (64 x 64) requests")
    ap.add_argument("--seed", type=int, default=5)
    args = ap.parse_args()
    import torch
    from paper_2202_09703_amd import umbir
    from synth import card_c1, card_c2, card_c3
    cards = {"c1": card_c1(), "c2": card_c2(), "c3": card_c3()}
    # plain-path capacity from one timed reconstruction per kind, weighted by the mix and
    # the mean iteration count
    mix = {"c1": 0.5, "c2": 0.35, "c3": 0.15}
    probe = synthesize(umbir, cards, [{"rid": i, "arrival": 0.0, "kind": k, "n_iter": 35}
                                      for i, k in enumerate(cards)])
    warm = plain_run(umbir, probe)
    timed = plain_run(umbir, probe)
    mean_service = sum(mix[r.kind] * (r.finished - r.admitted) for r in timed)
    capacity = 1.0 / mean_service
    rate = args.load * capacity
    print(f"plain service per kind (ms): " + ", ".join(f"{r.kind} {1e3 * (r.finished - r.admitted):.1f}"
                                                       for r in timed), file=sys.stderr, flush=True)
    specs = make_requests(args.requests, rate, args.seed)
    reqs = synthesize(umbir, cards, specs)
    print(f"{len(reqs)} requests at {rate:.2f}/s; plain path ...", file=sys.stderr, flush=True)
    plain = plain_run(umbir, reqs)
    print(f"plain done: {summarize(plain)}; served path ...", file=sys.stderr, flush=True)
    chunk = {"c1": args.chunk_small, "c2": args.chunk, "c3": args.chunk}
    srv = Server(GpuExecutor(umbir), hbm_budget=int(args.budget_gb * (1 << 30)), max_slots=args.slots,
                 chunk=chunk)
    served = srv.run(reqs)
    print(f"served done: {summarize(served)}", file=sys.stderr, flush=True)
    # each result equals its plain (one-at-a-time) result
    worst = 0.0
    by_id = {r.rid: r for r in plain}
    for r in served:
        a, b = r.x.double(), by_id[r.rid].x.double()
        worst = max(worst, float(torch.linalg.norm(a - b) / max(float(torch.linalg.norm(b)), 1e-300)))
    out = {"workload": f"{args.requests} requests, Poisson arrivals at {rate:.2f}/s "
                       f"({args.load:.0%} of plain capacity {capacity:.2f}/s), mix c1/c2/c3 = 0.5/0.35/0.15, "
                       f"20-50 iterations, HBM budget {args.budget_gb} GB",
           "plain": summarize(plain), "served": summarize(served),
           "served_rejected": len(srv.rejected), "peak_slots": srv.peak_slots,
           "peak_bytes": srv.peak_bytes, "chunk": chunk,
           "max_rel_diff_served_vs_plain": worst,
           "per_kind_p50_ms": {k: {"plain": float(np.percentile([r.latency * 1e3 for r in plain if r.kind == k], 50)),
                                   "served": float(np.percentile([r.latency * 1e3 for r in served if r.kind == k], 50))}
                               for k in cards if any(r.kind == k for r in plain)}}
    del warm
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
