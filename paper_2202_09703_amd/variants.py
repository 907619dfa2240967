"""Timing of the method variants on the plain 256 x 256 workload.

  attenuation  the forward and adjoint with water and concrete lossy (the
               paper's figures per MHz), for 1, 4 and 16 templates, against
               the lossless operator
  icd          grouped ICD sweeps (umbir_reconstruct_icd) against the
               surrogate iteration of umbir_reconstruct, with the cost reached
  forms        the factored and the direct form of the operator (A + A^T
               pair and a whole reconstruction) on the 64 x 64, 256 x 256
               and 512 x 512 workloads
  sweeps       --reps A + A^T pairs of the plain operator on a dense random
               image (the program a profiler wraps to count the sweep
               kernels); --workload c2 (256 x 256) or c3 (512 x 512, with
               --storage f32, f16 or bf16)

Data are synthesised on the device (A x_true + seeded noise at the card's
SNR).  Each line of output is one JSON record.

    python -m paper_2202_09703_amd.variants attenuation
    python -m paper_2202_09703_amd.variants icd
    python -m paper_2202_09703_amd.variants forms
    python -m paper_2202_09703_amd.variants sweeps --reps 5 --workload c2
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import time


def _setup(umbir, card, dev):
    import torch
    from synth import phantom, noise
    geom = umbir.build_geometry(card)
    xt = torch.tensor(phantom(card), dtype=torch.float32, device=dev)
    clean = umbir.forward(geom, xt)
    sigma = float(torch.sqrt(torch.mean(clean.double() ** 2) / 10.0 ** (card.snr_db / 10.0)))
    y = clean + sigma * torch.tensor(noise(card), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    return geom, xt, y, sigma


def attenuation(umbir, dev, reps: int):
    import torch
    from synth import card_c2
    from synth.cards import ALPHA_WATER, ALPHA_CEMENT
    base = card_c2()
    for g in (1, 4, 16):
        card = base
        if g > 1:
            alpha = [0.0] * base.medium.n_layers
            alpha[0], alpha[2] = ALPHA_WATER, ALPHA_CEMENT  # water, cement
            card = dataclasses.replace(base, medium=dataclasses.replace(base.medium, atten=tuple(alpha)),
                                       acq=dataclasses.replace(base.acq, n_gamma=g))
        geom, x, _, _ = _setup(umbir, card, dev)
        work = geom.workspace(umbir.WORK_ADJOINT)
        y = umbir.forward(geom, x, work=work)
        for _ in range(2):
            umbir.forward(geom, x, y, work=work)
            umbir.adjoint(geom, y, work=work)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            umbir.forward(geom, x, y, work=work)
            umbir.adjoint(geom, y, work=work)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        print(json.dumps({"variant": "attenuation", "templates": geom.n_gamma, "gamma_step_s": geom.gamma_step,
                          "a_plus_at_ms": dt * 1e3, "evals_per_s": card.n_traces * card.n_voxels / dt,
                          "workspace_MB": geom.workspace_bytes(umbir.WORK_ADJOINT) / 1e6}), flush=True)
        geom.free()


def icd(umbir, dev, reps: int):
    import torch
    from synth import card_c2
    card = card_c2()
    geom, _, y, sigma = _setup(umbir, card, dev)
    work = geom.workspace(umbir.WORK_RECONSTRUCT)
    umbir.reconstruct(geom, card.prior, sigma, y, 2, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, _, cost = umbir.reconstruct(geom, card.prior, sigma, y, card.n_iter, work=work)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / reps
    print(json.dumps({"variant": "surrogate", "iterations": card.n_iter, "ms": ts * 1e3,
                      "cost_first_last": [float(cost[0]), float(cost[-1])]}), flush=True)
    for group in ((8, 8), (16, 16)):
        umbir.reconstruct_icd(geom, card.prior, sigma, y, 1, group=group)
        torch.cuda.synchronize()
        for sweeps in (1, 3):
            t0 = time.perf_counter()
            for _ in range(reps):
                _, _, cost = umbir.reconstruct_icd(geom, card.prior, sigma, y, sweeps, group=group)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            print(json.dumps({"variant": "icd", "group": list(group), "sweeps": sweeps, "ms": dt * 1e3,
                              "cost": [float(c) for c in cost.cpu()]}), flush=True)
    geom.free()


def forms(umbir, dev, reps: int):
    import torch
    from synth import card_c1, card_c2, card_c3
    for card in (card_c1(), card_c2(), card_c3()):
        geom, x, y, sigma = _setup(umbir, card, dev)
        work = geom.workspace(umbir.WORK_RECONSTRUCT)
        yo = torch.empty_like(y)
        xo = torch.empty(geom.image_shape, dtype=torch.float32, device=dev)
        out = {"variant": "forms", "workload": card.name, "triples": card.n_traces * card.n_voxels}
        for form in (1, 2):
            geom.set_tuning(operator_form=form)
            for _ in range(2):
                umbir.forward(geom, x, yo, work=work)
                umbir.adjoint(geom, yo, xo, work=work)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                umbir.forward(geom, x, yo, work=work)
                umbir.adjoint(geom, yo, xo, work=work)
            torch.cuda.synchronize()
            pair = (time.perf_counter() - t0) / reps
            n = min(card.n_iter, 20)
            umbir.reconstruct(geom, card.prior, sigma, y, 1, work=work)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            umbir.reconstruct(geom, card.prior, sigma, y, n, work=work)
            torch.cuda.synchronize()
            rec = time.perf_counter() - t0
            name = "factored" if form == 1 else "direct"
            out[name] = {"pair_ms": pair * 1e3, "evals_per_s": out["triples"] / pair,
                         f"reconstruct_{n}_iterations_ms": rec * 1e3}
        geom.set_tuning(operator_form=1)
        chosen = geom.autotune()
        out["autotune_chose"] = "factored" if chosen["operator_form"] == 1 else "direct"
        print(json.dumps(out), flush=True)
        geom.free()


def sweeps(umbir, dev, reps: int, workload: str = "c2", storage: str = "f32"):
    import torch
    from synth import card_c2, card_c3
    card = card_c2() if workload == "c2" else card_c3()
    st = {"f32": umbir.STORAGE_F32, "f16": umbir.STORAGE_F16, "bf16": umbir.STORAGE_BF16}[storage]
    card = dataclasses.replace(card, acq=dataclasses.replace(card.acq, storage=st))
    geom = umbir.build_geometry(card)
    work = geom.workspace(umbir.WORK_ADJOINT)
    x = torch.randn(geom.image_shape, generator=torch.Generator().manual_seed(3)).to(dev)
    y = torch.empty(geom.trace_shape, dtype=geom.trace_dtype, device=dev)
    xo = torch.empty(geom.image_shape, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        umbir.forward(geom, x, y, work=work)
        umbir.adjoint(geom, y, xo, work=work)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"variant": "sweeps", "workload": card.name, "storage": storage, "pairs": reps,
                      "a_plus_at_ms": dt * 1e3}), flush=True)
    geom.free()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("which", choices=("attenuation", "icd", "forms", "sweeps"))
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--workload", choices=("c2", "c3"), default="c2")
    ap.add_argument("--storage", choices=("f32", "f16", "bf16"), default="f32")
    args = ap.parse_args()
    import torch
    from paper_2202_09703_amd import umbir
    dev = torch.device("cuda:0")
    if args.which == "sweeps":
        sweeps(umbir, dev, args.reps, args.workload, args.storage)
    else:
        {"attenuation": attenuation, "icd": icd, "forms": forms}[args.which](umbir, dev, args.reps)


if __name__ == "__main__":
    main()
