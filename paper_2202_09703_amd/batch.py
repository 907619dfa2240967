"""Batched reconstructions of many uneven problems.

Every problem keeps a resident solver session (geometry tables, data, iterate
and one captured graph per iteration).  The batched path advances all
unfinished sessions together: one graph launch per iteration runs every
session's captured iteration side by side on the device (umbir_batch_*).
Problems with fewer iterations leave the batch when they reach their count,
and the batch graph is rebuilt for the rest.  Launch shapes per problem shape
come from the library's autotuner (umbir_autotune), cached by shape, and are
set before the sessions capture their graphs.

The plain path steps the same kind of sessions one problem at a time on one
stream; the comparison therefore isolates batching.  Each batched result is
checked bitwise against its plain result.

    python -m paper_2202_09703_amd.batch --problems 48
"""
from __future__ import annotations

import argparse
import json
import time
from typing import Any, Dict, List


def prepare(umbir, cards, device="cuda:0", log=print, data=None):
    """Geometry and data per card: y = A x_true + sigma * noise made on the
    device, sigma from the card's SNR; or, with `data`, the given host data
    (a list of (y [P][K][M], sigma) per card) copied to the device."""
    import torch
    from synth import phantom, noise
    probs = []
    for i, card in enumerate(cards):
        g = umbir.build_geometry(card)
        if data is not None:
            y = torch.tensor(data[i][0], dtype=torch.float32, device=device)
            sigma = float(data[i][1])
            probs.append({"card": card, "geom": g, "y": y, "sigma": sigma, "n_iter": card.n_iter})
            continue
        xt = torch.tensor(phantom(card), dtype=torch.float32, device=device)
        clean = umbir.forward(g, xt)
        sigma = float(torch.sqrt(torch.mean(clean.double() ** 2) / 10.0 ** (card.snr_db / 10.0)))
        y = clean + sigma * torch.tensor(noise(card), dtype=torch.float32, device=device)
        probs.append({"card": card, "geom": g, "y": y, "sigma": sigma, "n_iter": card.n_iter})
        if (i + 1) % 8 == 0:
            log(f"prepared {i + 1}/{len(cards)} problems", flush=True)
    torch.cuda.synchronize()
    return probs


def tune(umbir, probs, cache: Dict[Any, Any], log=print):
    """Autotune every geometry; shapes seen before reuse the cached choice."""
    import torch
    t0 = time.perf_counter()
    chosen = [p["geom"].autotune(cache=cache) for p in probs]
    torch.cuda.synchronize()
    log(f"autotuned {len(cache)} shapes for {len(probs)} problems in {time.perf_counter() - t0:.2f} s", flush=True)
    return chosen


def sessions(umbir, probs):
    return [umbir.Solver(p["geom"], p["card"].prior, p["sigma"], p["y"], max_iter=p["n_iter"]) for p in probs]


def run_plain(umbir, probs):
    """One problem at a time: each session stepped to its count in turn."""
    import torch
    ss = sessions(umbir, probs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, p in zip(ss, probs):
        s.step(p["n_iter"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = [s.read() for s in ss]
    torch.cuda.synchronize()
    for s in ss:
        s.free()
    return dt, out


def run_batched(umbir, probs, mode: int = 0):
    """All unfinished sessions advanced together by umbir_batch_step (mode
    BATCH_STREAMS: each session's graphs on four streams; BATCH_GRAPH: one
    graph per iteration captured across them; BATCH_WORKLIST: per lane of
    problems one launch per stage of the iteration over all its problems'
    work items, one batch stepped to the largest iteration count, problems
    leaving as they reach theirs)."""
    import torch
    ss = sessions(umbir, probs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    live = list(range(len(ss)))
    batches = []  # kept until the device is done with them
    if mode == umbir.BATCH_WORKLIST:
        b = umbir.Batch(ss, mode)
        b.step(max(p["n_iter"] for p in probs))
        batches.append(b)
        live = []
    while live:
        k = min(probs[i]["n_iter"] - ss[i].iterations for i in live)
        b = umbir.Batch([ss[i] for i in live], mode)
        b.step(k)
        batches.append(b)
        live = [i for i in live if ss[i].iterations < probs[i]["n_iter"]]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rebuilds = len(batches)
    for b in batches:
        b.free()
    out = [s.read() for s in ss]
    torch.cuda.synchronize()
    for s in ss:
        s.free()
    return dt, out, rebuilds


def run_streams(umbir, probs, n_streams: int = 4):
    """Each session stepped to its count on one of n_streams streams (default
    priority), so independent problems may overlap on the device."""
    import torch
    ss = sessions(umbir, probs)
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (s, p) in enumerate(zip(ss, probs)):
        with torch.cuda.stream(streams[i % n_streams]):
            s.step(p["n_iter"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = [s.read() for s in ss]
    torch.cuda.synchronize()
    for s in ss:
        s.free()
    return dt, out


def evals(probs) -> int:
    """A + A^T voxel-trace pairs of the whole job (iterations x traces x voxels)."""
    return sum(p["n_iter"] * p["card"].n_traces * p["card"].n_voxels for p in probs)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--problems", type=int, default=48)
    ap.add_argument("--seed", type=int, default=11)
    args = ap.parse_args()
    import torch
    from paper_2202_09703_amd import umbir
    from synth import batch_cards
    cards = batch_cards(args.problems, args.seed)
    probs = prepare(umbir, cards)
    work = evals(probs)
    t_default, _ = run_plain(umbir, probs)
    print(f"plain, default launch shapes: {t_default:.3f} s", flush=True)
    cache: Dict[Any, Any] = {}
    chosen = tune(umbir, probs, cache)
    t_plain, plain = run_plain(umbir, probs)
    print(f"plain, tuned: {t_plain:.3f} s", flush=True)
    t_batch, batched, rebuilds = run_batched(umbir, probs, umbir.BATCH_STREAMS)
    print(f"batched (streams), tuned: {t_batch:.3f} s ({rebuilds} batches)", flush=True)
    t_graph, graphed, _ = run_batched(umbir, probs, umbir.BATCH_GRAPH)
    print(f"batched (one graph per iteration), tuned: {t_graph:.3f} s", flush=True)
    t_wl, wl, _ = run_batched(umbir, probs, umbir.BATCH_WORKLIST)
    print(f"batched (work lists), tuned: {t_wl:.3f} s", flush=True)
    same = all(torch.equal(a[0], b[0]) and torch.equal(a[2], b[2]) and torch.equal(a[0], c[0])
               and torch.equal(a[2], c[2]) and torch.equal(a[0], d[0]) and torch.equal(a[2], d[2])
               for a, b, c, d in zip(plain, batched, graphed, wl))
    res = {"problems": len(probs), "iterations": sum(p["n_iter"] for p in probs),
           "evals": work, "plain_default_s": t_default, "plain_tuned_s": t_plain, "batched_s": t_batch,
           "evals_per_s_plain": work / t_plain, "evals_per_s_batched": work / t_batch,
           "recon_per_s_plain": len(probs) / t_plain, "recon_per_s_batched": len(probs) / t_batch,
           "speedup": t_plain / t_batch, "batches": rebuilds, "batched_graph_s": t_graph,
           "speedup_graph": t_plain / t_graph, "batched_worklist_s": t_wl,
           "speedup_worklist": t_plain / t_wl, "recon_per_s_worklist": len(probs) / t_wl,
           "bitwise_equal": bool(same),
           "shapes_tuned": len(cache),
           "tuning": {c.name: t for c, t in zip(cards, chosen)}}
    print(json.dumps(res), flush=True)
    for p in probs:
        p["geom"].free()


if __name__ == "__main__":
    main()
