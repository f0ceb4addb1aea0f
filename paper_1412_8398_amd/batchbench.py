"""Batched solves of the training-data distribution on one GPU.

    python -m paper_1412_8398_amd.batchbench --n 512 --out batch.json

Samples: sphere-Boolean cells with grid edges drawn from {32, 48, 64, 96},
volume fraction U[0.05, 0.4], log10 contrast U[-2, 3] (matrix E = 1), one
Poisson ratio U[0.2, 0.4] for both phases, sphere radius U[3, 8] voxels, one
unit macroscopic strain among the six (microstructure.batch_samples).  The
accelerated scheme with the rotated operator, float32 fields, tolerance 1e-6.

Runs of fe_solve_batched over the whole batch, each float32 launch (one per
pass; one cooperative persistent launch) with refine off (the float32
iteration alone) and on (then float64 iterations for the samples whose
float32 strain does not verify to the tolerance).  Reports device seconds,
voxel-iterations per second, the status counts and the float64-verified eta
of the returned strains.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--seed", type=int, default=4512)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=1500)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    import torch

    import paper_1412_8398_amd as fe
    from microstructure import batch_samples

    t0 = time.time()
    samples = batch_samples(args.n, args.seed)
    print(json.dumps({"msg": "samples", "n": args.n, "seconds": round(time.time() - t0, 1),
                      "voxels": int(sum(s.L ** 3 for s in samples))}), flush=True)
    phases = [torch.from_numpy(s.phase).cuda() for s in samples]
    outs = [torch.empty((6, s.L, s.L, s.L), dtype=torch.float32, device="cuda") for s in samples]
    specs = [fe.BatchSampleSpec(p, [1.0, s.contrast], [s.nu, s.nu], s.macro_strain, e)
             for p, s, e in zip(phases, samples, outs)]
    rep = {"n": args.n, "seed": args.seed, "tol": args.tol, "max_iter": args.max_iter,
           "sizes": {str(L): sum(1 for s in samples if s.L == L) for L in (32, 48, 64, 96)}}
    for launch, refine in (("per_pass", False), ("persistent", False), ("per_pass", True), ("persistent", True)):
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        res, status, sec = fe.solve_batched(specs, args.tol, green="R", scheme="AS", precision="fp32",
                                            max_iter=args.max_iter, refine=refine, raise_on_error=False,
                                            launch=launch)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        its = np.array([r.iterations for r in res])
        st = np.array([r.status for r in res])
        ev = np.array([r.eta_verify_fp64 for r in res])
        vox_it = float(sum(s.L ** 3 * r.iterations for s, r in zip(samples, res)))
        row = {"launch": launch, "refine": refine, "device_seconds": round(sec, 4), "wall_seconds": round(wall, 3),
               "voxel_iterations": vox_it, "gvoxel_iter_per_s": round(vox_it / sec / 1e9, 2),
               "status_counts": {fe.status_string(int(k)): int(np.sum(st == k)) for k in np.unique(st)},
               "iterations_mean": float(its.mean()), "iterations_max": int(its.max()),
               "eta_verify_fp64_max": float(ev.max()), "eta_verify_fp64_median": float(np.median(ev)),
               "verified_to_tol": int(np.sum(ev <= args.tol))}
        rep[f"{launch}_{'refine' if refine else 'float32'}"] = row
        print(json.dumps(row), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(rep, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
