"""Benchmark of the MAP reconstruction hot path on one MI355X.

One step = one whole reconstruction of the plain FP32 workload (256 x 256
grid, 0.5 mm voxels, water/steel/cement, 32 scan positions x 16 receivers,
2048 samples at 20 MHz, 50 surrogate iterations): build the geometry (leg
table, template, direct-arrival columns), the data-term curvature (one |A|
and one |A|^T), then per iteration one A x with the residual and g step, one
A^T e, the prior-weighted image update and the cost.

value = A+A^T voxel-receiver evals per second of whole-job time:
P K N (n_iter + 1) / (seconds per step); the +1 is the curvature pass.
Inputs are resident in HBM before the timed region; the data are synthetic
(seeded phantom, A x_true plus seeded Gaussian noise at 15 dB).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12   # MI355X published fp32 FLOP/s (vector and dense matrix)
PEAK_HBM = 8.0e12      # MI355X published HBM3E bytes/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_plain_256x256.json")
LAUNCH_SAMPLE = 10     # the timed steps bracket every 10th launch of the dominant kernel with events


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--quick", action="store_true", help="skip parity sampling and the CPU baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale HBM counters)")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write the per-kernel HBM traffic file from four rocprofv3 --pmc counter CSVs")
    return ap.parse_args()


def source_digest():
    """SHA-256 over the HIP sources: traffic counters are valid for this exact source only."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2202_09703_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def traffic_from(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv):
    """Average FETCH_SIZE / WRITE_SIZE (KiB per dispatch) per kernel, scaled so a
    plain 1 GiB copy reads and writes 1 GiB, written to TRAFFIC_FILE."""
    import csv
    import re

    def per_kernel(path):
        acc = {}
        for row in csv.DictReader(open(path)):
            m = re.search(r"k_([a-z_0-9]+)", row["Kernel_Name"])
            if not m:
                continue
            # the library's launch names: k_conv_mfma / k_conv_mfma16 launch
            # as "conv", k_corr_mfma / k_corr_x3 as "corr", k_gather_lds as
            # "gather"
            name = re.sub(r"_(mfma(16)?|x3|lds)$", "", m.group(1))
            n, v = acc.setdefault(name, [0, 0.0]), float(row["Counter_Value"])
            n[0] += 1
            n[1] += v
        return {k: v[1] / v[0] for k, v in acc.items()}

    def copy_kib(path):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path)) if "copyBuffer" in r["Kernel_Name"]]
        return sum(vals) / len(vals)

    gib_kib = float(1 << 20)
    kf, kw = gib_kib / copy_kib(copy_fetch_csv), gib_kib / copy_kib(copy_write_csv)
    fetch, write = per_kernel(fetch_csv), per_kernel(write_csv)
    doc = {"source_sha256": source_digest(),
           "calibration": {"fetch_scale": kf, "write_scale": kw,
                           "note": "a 1 GiB device copy defines the scale of each counter"},
           "kernels": {k: {"fetch_bytes": fetch[k] * kf * 1024, "write_bytes": write.get(k, 0.0) * kw * 1024}
                       for k in sorted(fetch)}}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    print(json.dumps(doc["kernels"], indent=1))


def copy_calibration():
    """A plain device copy of known size: 1 GiB read + 1 GiB written per launch."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": 4 * n, "copy_bytes_written_per_launch": 4 * n,
                      "launches": 3}), flush=True)


def gather_launches(card, trace_groups, gather_batch_kb, elem=4):
    """Launches of the gather per adjoint: each covers a batch of every trace
    group's traces, gather_batch_kb KiB of fine grid per group (at least one
    trace)."""
    acq = card.acq
    PK = card.array.n_scans * card.array.n_rx
    tpg = -(-PK // trace_groups)
    batch = max(1, min(tpg, (gather_batch_kb << 10) // (acq.n_samples * acq.oversample * elem)))
    return -(-tpg // batch)


def kernel_work(name, card, n_off, trace_groups, gather_batch_kb=4096, elem=4):
    """Algorithmic work of one launch and its bound.

    conv / corr: the polyphase convolution and correlation, 2 M Q L_h flop per
    trace (on the matrix cores when Q is 32 or 64).  splat / gather: compulsory
    HBM bytes.  The splat reads the leg table, the image and the row
    transmittances and writes the fine-grid signal (M Q elements per trace)
    once.  The adjoint's fine grid is read once over its gather launches, each
    of which also reads the leg table and the transmittances and writes the
    trace groups' partial images (the first launch writes them, later ones
    read and write them): the per-launch figure is that total over the
    launches."""
    acq = card.acq
    P, K, M, Q = card.array.n_scans, card.array.n_rx, acq.n_samples, acq.oversample
    lh = int(round(acq.t_win * acq.fs))
    N, nz = card.n_voxels, card.grid.nz
    legs = nz * n_off * 16
    fine = P * K * M * Q * elem
    if name in ("conv", "corr"):
        return 2.0 * P * K * M * Q * lh, ("mfma" if Q in (32, 64) else "alu")
    if name == "splat":
        return float(legs + 4 * N + 4 * nz + fine), "hbm"
    if name == "gather":
        n = gather_launches(card, trace_groups, gather_batch_kb, elem)
        partial = 4 * N * trace_groups * (2 * n - 1)
        return float(fine + n * (legs + 4 * nz) + partial) / n, "hbm"
    if name == "gstep":  # residual and g step: read e and the direct-arrival columns, write e
        return float(12 * P * K * M), "hbm"
    if name == "prior":  # image update: read x, A^T e and the curvature, write x
        return float(16 * N), "hbm"
    return None, None


def copy_rate():
    """Bytes per second of a plain 1 GiB device copy (read + write), the
    practical HBM ceiling the small update kernels are measured against."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    rate = 5 * 8.0 * n / (e0.elapsed_time(e1) / 1e3)
    del a, b
    return rate


PEAK_MFMA = {4: 157.3e12, 2: 2.5e15}  # dense matrix peak by element bytes: FP32, FP16/BF16
PIECE_PRODUCTS = 6  # bf16 piece products per FP32 product (umbir_tuning.products = 2)


def roofline(name, prof, steps, card, n_off, trace_groups, gather_batch_kb=4096, elem=4, products=1):
    """One kernel's achieved rate against its bound.  With products = 2 the
    FP32 convolution and correlation run on the bf16 matrix cores, six piece
    products per FP32 product: the record then counts those bf16 flops
    against the bf16 peak, and gives the FP32 figures beside them."""
    if name not in prof:
        return None
    launches, ms = prof[name]
    avg_s = ms / launches / 1e3
    amount, bound = kernel_work(name, card, n_off, trace_groups, gather_batch_kb, elem)
    if bound is None:
        return None
    pieces = bound == "mfma" and elem == 4 and products == 2
    executed = amount * PIECE_PRODUCTS if pieces else amount
    achieved = executed / avg_s
    peak = PEAK_HBM if bound == "hbm" else (PEAK_MFMA[2 if pieces else elem] if bound == "mfma" else PEAK_FP32)
    unit, div = ("GB/s", 1e9) if bound == "hbm" else ("TFLOP/s", 1e12)
    rec = {"bound": bound, "achieved": achieved / div, "peak": peak / div, "unit": unit,
           "frac": achieved / peak, "kernel": name, "avg_launch_us": avg_s * 1e6,
           "launches_per_step": launches / steps, "work_per_launch": executed,
           "work_unit": "byte" if bound == "hbm" else "flop"}
    if pieces:
        rec["work_unit"] = "bf16 flop (%d piece products per FP32 product)" % PIECE_PRODUCTS
        rec["fp32_flop_per_launch"] = amount
        rec["fp32_equivalent_TFLOPs"] = amount / avg_s / 1e12
        rec["fp32_equivalent_frac_of_fp32_peak"] = amount / avg_s / PEAK_MFMA[4]
    return rec


def host_cpu():
    """The host's core count and CPU model (for the CPU baseline record)."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def operator_roofline(card, t_pair, triples, n_off, elem=4):
    """One A + A^T pair against the two ceilings of the operator's own
    definition (Eq. (13)): 2 L_h flop per (trace, voxel) per operator on the
    FP32 units, and the operator's algorithmic HBM bytes (image, traces, leg
    table and template read or written once per operator)."""
    acq, a, g = card.acq, card.array, card.grid
    lh = int(round(acq.t_win * acq.fs))
    flop = 2.0 * 2 * lh * triples
    per_op = (4.0 * g.nx * g.nz + elem * a.n_scans * a.n_rx * acq.n_samples + 16.0 * g.nz * n_off
              + 4.0 * (acq.oversample * lh + 2))
    return {"pair_ms": t_pair * 1e3, "flop_per_pair": flop, "achieved_TFLOPs": flop / t_pair / 1e12,
            "frac_of_fp32": flop / t_pair / PEAK_FP32,
            "algorithmic_bytes_per_pair": 2 * per_op,
            "hbm_frac_at_algorithmic_bytes": 2 * per_op / t_pair / PEAK_HBM,
            "note": "operator work as Eq. (13) defines it (2 L_h flop per triple per operator), "
                    "whichever way the kernels factor it; at its algorithmic bytes (image, traces, leg table, "
                    "template once per operator) HBM is not what bounds a matrix-free sweep"}


def time_pair(umbir, torch, gm, x, y, xo, work, reps=10):
    """Seconds per A and per A^T (plain calls, events on the current stream)."""
    for _ in range(2):
        umbir.forward(gm, x, y, work=work)
        umbir.adjoint(gm, y, xo, work=work)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(reps):
        umbir.forward(gm, x, y, work=work)
    ev[1].record()
    for _ in range(reps):
        umbir.adjoint(gm, y, xo, work=work)
    ev[2].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) / reps / 1e3, ev[1].elapsed_time(ev[2]) / reps / 1e3


def precision_section(umbir, torch, dev, with_parity):
    """The 512 x 512 four-layer workload (64 x 32 traces, 4096 samples) per
    storage type: A and A^T rates, every sweep kernel's roofline from one
    profiled pair, the dominant one named, and (with_parity) sampled traces and
    voxels against the FP64 oracle on unrounded inputs."""
    import dataclasses
    from synth import card_c3, phantom, random_vector
    base = card_c3()
    P, K, M, N = base.array.n_scans, base.array.n_rx, base.acq.n_samples, base.n_voxels
    triples = P * K * N
    x_np = phantom(base)
    r_np = random_vector((P, K, M), seed=61)
    traces = [(5, 3), (40, 30)]
    vox = np.random.default_rng(7).choice(N, 16, replace=False)
    ref = None
    if with_parity:
        from oracle import operator as oo
        ref = (oo.forward(base, x_np, traces=traces, workers=None), oo.adjoint_voxels(base, r_np, vox, workers=None))
    out = {"workload": "512x512, 4 layers (water/steel/cement/rock), 64 scans x 32 rx, 4096 samples @ 20 MHz",
           "triples_per_sweep": triples}
    for name, st in (("f32", umbir.STORAGE_F32), ("f16", umbir.STORAGE_F16), ("bf16", umbir.STORAGE_BF16)):
        card = dataclasses.replace(base, acq=dataclasses.replace(base.acq, storage=st))
        gm = umbir.build_geometry(card)
        work = gm.workspace(umbir.WORK_ADJOINT)
        x = torch.tensor(x_np, dtype=torch.float32, device=dev)
        y = torch.empty(gm.trace_shape, dtype=gm.trace_dtype, device=dev)
        xo = torch.empty(gm.image_shape, dtype=torch.float32, device=dev)
        t_a, t_at = time_pair(umbir, torch, gm, x, y, xo, work)
        umbir.profile_select(None)
        umbir.profile_enable(True)
        umbir.profile_collect()
        for _ in range(3):
            umbir.forward(gm, x, y, work=work)
            umbir.adjoint(gm, y, xo, work=work)
        torch.cuda.synchronize()
        umbir.profile_enable(False)
        prof = umbir.profile_collect()
        elem = 4 if st == umbir.STORAGE_F32 else 2
        tn = gm.tuning()
        kb = tn["gather_batch_kb"]
        kern = {k: roofline(k, prof, 3, card, gm.n_off, gm.trace_groups, kb, elem, tn["products"])
                for k in ("splat", "conv", "corr", "gather")}
        dom = max(kern, key=lambda k: kern[k]["avg_launch_us"] * kern[k]["launches_per_step"] if kern[k] else -1)
        res = {"A_evals_per_s": triples / t_a, "AT_evals_per_s": triples / t_at,
               "A_plus_AT_evals_per_s": triples / (t_a + t_at), "A_ms": t_a * 1e3, "AT_ms": t_at * 1e3,
               "dominant_kernel": dom, "roofline": kern[dom], "sweep_kernels": kern,
               "operator_roofline": operator_roofline(card, t_a + t_at, triples, gm.n_off, elem)}
        if ref is not None:
            yf = umbir.forward(gm, x).float().cpu().numpy()
            rt = torch.tensor(r_np, dtype=torch.float32, device=dev).to(gm.trace_dtype)
            xa = umbir.adjoint(gm, rt).cpu().numpy().reshape(-1)
            fe = max(float(np.linalg.norm(yf[i, j] - ref[0][i, j]) / np.linalg.norm(ref[0][i, j])) for i, j in traces)
            ae = float(np.linalg.norm(xa[vox] - ref[1]) / np.linalg.norm(ref[1]))
            res["parity_vs_oracle"] = {"forward_rel_l2_max_of_2_traces": fe, "adjoint_rel_l2_16_voxels": ae,
                                       "unit_roundoff": {"f32": 2.0 ** -24, "f16": 2.0 ** -11,
                                                         "bf16": 2.0 ** -8}[name]}
        out[name] = res
        gm.free()
        del work
    return out


def batch_section(umbir, torch, dev):
    """48 seeded uneven problems (128^2 to 384^2, 3-4 layers, 8-32 receivers,
    1024-4096 samples, 20-50 iterations): one at a time against the batched
    paths (sessions' graphs on four streams; work-list launches per stage over
    four lanes of problems), all autotuned; results bitwise equal."""
    from paper_2202_09703_amd import batch
    from synth import batch_cards
    cards = batch_cards(48, 11)
    quiet = lambda *a, **k: None  # noqa: E731
    probs = batch.prepare(umbir, cards, device=dev, log=quiet)
    cache = {}
    batch.tune(umbir, probs, cache, log=quiet)
    batch.run_plain(umbir, probs)  # warm
    t_plain, plain = batch.run_plain(umbir, probs)
    t_batch, batched, rebuilds = batch.run_batched(umbir, probs, umbir.BATCH_STREAMS)
    t_wl, wl, _ = batch.run_batched(umbir, probs, umbir.BATCH_WORKLIST)
    same = all(torch.equal(a[0], b[0]) and torch.equal(a[2], b[2]) and torch.equal(a[0], c[0])
               and torch.equal(a[2], c[2]) for a, b, c in zip(plain, batched, wl))
    work = batch.evals(probs)
    for p in probs:
        p["geom"].free()
    return {"problems": len(cards), "iterations": sum(c.n_iter for c in cards),
            "plain_s": t_plain, "batched_s": t_batch, "recon_per_s_plain": len(cards) / t_plain,
            "recon_per_s_batched": len(cards) / t_batch, "speedup": t_plain / t_batch,
            "evals_per_s_plain": work / t_plain, "evals_per_s_batched": work / t_batch,
            "batches": rebuilds, "worklist_s": t_wl, "recon_per_s_worklist": len(cards) / t_wl,
            "speedup_worklist": t_plain / t_wl, "bitwise_equal_to_plain": bool(same)}


def cpu_baseline_section(card):
    """The oracle (FP64 numpy) on bounded samples of the same workload, one A
    and one A^T over all voxels: 6 traces on one core, and one whole scan
    position (16 traces) on all host cores (at most 16 processes)."""
    import dataclasses
    from oracle import operator as oo
    from synth import phantom
    P, N = card.array.n_scans, card.n_voxels
    xs = phantom(card).astype(np.float64)
    nproc, model = host_cpu()
    res = []
    for ks, workers in ((6, 1), (card.array.n_rx, None)):
        sub = dataclasses.replace(card, array=dataclasses.replace(
            card.array, tx_x=(card.array.tx_x[P // 2],), rx_offset=card.array.rx_offset[:ks]))
        used = min(oo.host_workers(workers), ks)
        t0 = time.perf_counter()
        ys = oo.forward(sub, xs, workers=workers)
        oo.adjoint_voxels(sub, ys, np.arange(N), workers=workers)
        tc = time.perf_counter() - t0
        res.append({"value": ks * N / tc, "unit": "evals/s", "cores": used, "kind": "oracle",
                    "sample": f"{ks} traces (one scan position) of the same workload: one A and one A^T over all "
                              f"{N} voxels in FP64 numpy on {used} process(es), {tc:.1f} s",
                    "host_cores": nproc, "host_cpu": model})
    return res


def main():
    args = parse()
    if args.traffic_from:
        traffic_from(*args.traffic_from)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): sharding over several "
              "GPUs is designed (scan positions per GPU, one all-reduce of the adjoint image per "
              "iteration) but not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2202_09703_amd import umbir
    from synth import card_c2, phantom, noise

    def say(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    card = card_c2()
    P, K, M = card.array.n_scans, card.array.n_rx, card.acq.n_samples
    N = card.n_voxels
    n_iter = card.n_iter
    triples = P * K * N

    # ---- synthetic inputs, resident in HBM before timing
    geom = umbir.build_geometry(card)
    x_true = torch.tensor(phantom(card), dtype=torch.float32, device=dev)
    clean = umbir.forward(geom, x_true)
    sigma = float(torch.sqrt(torch.mean(clean.double() ** 2) / 10.0 ** (card.snr_db / 10.0)))
    y = clean + sigma * torch.tensor(noise(card), dtype=torch.float32, device=dev)
    work = geom.workspace(umbir.WORK_RECONSTRUCT)
    x = torch.zeros(geom.image_shape, dtype=torch.float32, device=dev)
    g = torch.zeros(geom.trace_shape[:2], dtype=torch.float32, device=dev)
    cost = torch.empty(n_iter + 1, dtype=torch.float64, device=dev)
    tuning = geom.tuning()  # the library's default launch shapes
    geom.free()
    torch.cuda.synchronize()

    def step():
        gm = umbir.build_geometry(card)
        x.zero_()
        g.zero_()
        umbir.reconstruct(gm, card.prior, sigma, y, n_iter, x=x, g=g, cost=cost, work=work)
        return gm

    for _ in range(args.warmup):
        step().free()
    torch.cuda.synchronize()

    # one untimed step with every kernel bracketed by events: the per-kernel
    # breakdown, and which kernel dominates
    umbir.profile_select(None)
    umbir.profile_enable(True)
    umbir.profile_collect()
    step().free()
    torch.cuda.synchronize()
    umbir.profile_enable(False)
    prof_all = umbir.profile_collect()
    dname = max(prof_all.items(), key=lambda kv: kv[1][1])[0]

    # the timed steps bracket only the dominant kernel, and only a sample of
    # its launches (every LAUNCH_SAMPLE-th): its duration measured live, with
    # few event records in the work timed
    umbir.profile_select([dname])
    umbir.profile_stride(LAUNCH_SAMPLE)
    umbir.profile_enable(True)
    umbir.profile_collect()
    # no synchronisation between steps: the host part of the next problem's
    # geometry build runs while the GPU still runs the previous reconstruction
    # (build_geometry then waits for the stream before it returns); per-step
    # latency is the GPU time between stream events at the step boundaries
    keep = []
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    marks[0].record()
    for k in range(args.steps):
        keep.append(step())
        marks[k + 1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    lat = [marks[k].elapsed_time(marks[k + 1]) / 1e3 for k in range(args.steps)]
    umbir.profile_enable(False)
    prof = umbir.profile_collect()
    umbir.profile_stride(1)
    umbir.profile_select(None)
    for gm in keep:
        gm.free()
    say(f"timed {args.steps} reconstructions: {elapsed / args.steps * 1e3:.2f} ms each")

    sec_per_step = elapsed / args.steps
    evals_per_step = triples * (n_iter + 1)
    value = evals_per_step / sec_per_step
    costs = cost.cpu().numpy()

    # ---- per-operator rates (plain calls, HIP events on the current stream)
    gm = umbir.build_geometry(card)
    wf = gm.workspace(umbir.WORK_ADJOINT)
    xr = torch.randn(gm.image_shape, generator=torch.Generator().manual_seed(3)).to(dev)
    yr = torch.empty(gm.trace_shape, dtype=torch.float32, device=dev)
    xo = torch.empty(gm.image_shape, dtype=torch.float32, device=dev)
    t_fwd, t_adj = time_pair(umbir, torch, gm, xr, yr, xo, wf)

    # ---- rooflines: the dominant kernel from the timed steps; every sweep
    # kernel from the profiled untimed step
    tg, kb = gm.trace_groups, tuning["gather_batch_kb"]
    pr = tuning["products"]
    kernels = {k: roofline(k, prof_all, 1, card, gm.n_off, tg, kb, products=pr) for k in ("splat", "conv", "corr", "gather")}
    roof = roofline(dname, prof, args.steps, card, gm.n_off, tg, kb, products=pr)
    if roof is not None:  # launches per step from the fully profiled step; the timed ones are a sample
        roof["launches_per_step"] = prof_all[dname][0]
        roof["timed_launches"] = prof[dname][0]
        roof["timed_every"] = LAUNCH_SAMPLE
    # measured HBM bytes per launch, valid only for the exact sources they were taken on
    measured = {}
    try:
        tf = json.load(open(TRAFFIC_FILE))
        if tf.get("source_sha256") == source_digest():
            measured = {k: t["fetch_bytes"] + t["write_bytes"] for k, t in tf["kernels"].items()}
    except (OSError, ValueError, KeyError):
        measured = {}
    for k, r in kernels.items():
        if r is not None:
            r["traffic"] = measured.get(k)
    if roof is not None:
        roof["traffic"] = measured.get(dname)

    out = {
        "metric": "A+Aᵀ voxel-receiver evals/sec",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_note": ("FP32 data and accumulation; the convolution and correlation form each FP32 product "
                       "from three bf16 pieces per factor on the bf16 matrix cores (six piece products, "
                       "error below 2^-23 of the product)" if tuning.get("products") == 2 else
                       "FP32 data, products and accumulation"),
        "data": "synthetic",
        "config": {"workload": "plain FP32 MBIR 256x256, 3 layers, 32 scans x 16 rx, 2048 samples "
                               "@ 20 MHz, 50 iterations", "grid": [256, 256], "scans": P, "receivers": K,
                   "samples": M, "iterations": n_iter, "triples_per_sweep": triples},
        "recon_per_s": 1.0 / sec_per_step,
        "latency_ms_p50": float(np.percentile(np.array(lat) * 1e3, 50)),
        "latency_ms_p99": float(np.percentile(np.array(lat) * 1e3, 99)),
        "latency_note": "GPU time per reconstruction between stream events at the step boundaries "
                        "(steps are not synchronised with the host)",
        "A_evals_per_s": triples / t_fwd,
        "AT_evals_per_s": triples / t_adj,
        "A_ms": t_fwd * 1e3,
        "AT_ms": t_adj * 1e3,
        "cost_first_last": [float(costs[0]), float(costs[-1])],
        "kernels_ms_per_step": {k: v[1] for k, v in sorted(prof_all.items())},
        "kernels_ms_note": "one untimed step with every launch bracketed by events; the timed steps "
                           "bracket only the dominant kernel",
        "tuning": tuning,
        "roofline": roof,
        "sweep_kernels": kernels,
        "operator_roofline": operator_roofline(card, t_fwd + t_adj, triples, gm.n_off),
    }
    # the HBM-bound update kernels against the published peak and a measured copy
    crate = copy_rate()
    small = {}
    for k in ("gstep", "prior"):
        r = roofline(k, prof_all, 1, card, gm.n_off, tg)
        if r is not None:
            r["copy_GBps"] = crate / 1e9
            r["frac_of_copy"] = r["achieved"] * 1e9 / crate
            small[k] = r
    out["update_kernels"] = small

    if not args.quick:
        from oracle import operator as oo
        xs = x_true.cpu().numpy().astype(np.float64)
        yf = umbir.forward(gm, x_true).cpu().numpy()
        i, j = 13, 5
        ref = oo.forward(card, xs, traces=[(i, j)])[i, j]
        fe = float(np.linalg.norm(yf[i, j] - ref) / np.linalg.norm(ref))
        rr = np.asarray(noise(card), np.float64)
        xa = umbir.adjoint(gm, torch.tensor(rr, dtype=torch.float32, device=dev)).cpu().numpy().reshape(-1)
        vox = np.random.default_rng(9).choice(N, 64, replace=False)
        refa = oo.adjoint_voxels(card, rr, vox, workers=None)
        ae = float(np.linalg.norm(xa[vox] - refa) / np.linalg.norm(refa))
        out["parity_vs_oracle"] = {"forward_rel_l2_trace": fe, "adjoint_rel_l2_64_voxels": ae,
                                   "tolerance": 1e-5}
        say("parity sampled")
    gm.free()
    del wf, work

    if not args.quick:
        out["precision_512x512"] = precision_section(umbir, torch, dev, with_parity=True)
        say("512x512 storage types done")
        out["batch_48"] = batch_section(umbir, torch, dev)
        say("48-problem batch done")

    if not args.quick and not args.no_cpu:
        base = cpu_baseline_section(card)
        out["cpu_baseline"] = base[0]
        out["cpu_baseline_all_cores"] = base[1]
        say("CPU baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
