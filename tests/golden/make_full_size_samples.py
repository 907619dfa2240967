"""Writes full_size_samples.json: the separable-surrogate curvature
d = Abar^T Abar 1 (sigma = 1) of the oracle at seeded voxel samples of the
256 x 256 plain workload and the 512 x 512 four-layer workload.

Abar 1 needs every voxel of every trace, so at these sizes the oracle takes
minutes (256 x 256) to about an hour (512 x 512) on all host cores; the GPU
tests compare against the stored values.  Calls only the oracle.

    python tests/golden/make_full_size_samples.py [--only c2|c3] [--workers N]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import operator, solver  # noqa: E402
from synth import card_c2, card_c3  # noqa: E402

OUT = os.path.join(HERE, "full_size_samples.json")
# workload -> (card, number of sampled voxels, seed of the sample)
CASES = {"c2": (card_c2, 256, 2202), "c3": (card_c3, 64, 9703)}


def sample_voxels(card, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(card.n_voxels, n, replace=False))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=sorted(CASES))
    ap.add_argument("--workers", type=int, default=None)
    args = ap.parse_args()
    doc = json.load(open(OUT)) if os.path.exists(OUT) else {}
    doc["note"] = ("oracle (FP64) curvature d = Abar^T Abar 1 at sigma = 1 (Abar: the operator of |W| and the "
                   "absolute template), at seeded voxel samples; written by make_full_size_samples.py")
    for key, (mk, n, seed) in CASES.items():
        if args.only and key != args.only:
            continue
        card = mk()
        vox = sample_voxels(card, n, seed)
        t0 = time.perf_counter()
        d = solver.sqs_denominator_voxels(card, 1.0, vox, workers=args.workers)
        dt = time.perf_counter() - t0
        doc[key] = {"card": card.name, "voxels": [int(v) for v in vox], "seed": seed,
                    "abs_normal": [float(v) for v in d], "seconds": round(dt, 1),
                    "workers": operator.host_workers(args.workers)}
        print(f"{key}: {n} voxels in {dt:.0f} s", flush=True)
        with open(OUT, "w") as f:
            json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
