"""Effective stiffness of a seeded three-phase Voronoi cell on one GPU.

    python -m paper_1412_8398_amd.stiffness --size 1024 --seeds 4096 --out c.json

Each Voronoi cell draws one of three isotropic phases, (E, nu) in
{(1, 0.2), (5, 0.3), (50, 0.35)}; the six unit macroscopic strains are solved
with the accelerated scheme and the rotated operator (float32 fields, float64
reductions and re-anchoring) to eta <= tol, and <sigma> gives the 6x6
effective stiffness (eq. (5)).  Reports timings, iteration counts and the
checks that hold for any size: symmetry, positive definiteness, Voigt and
Reuss bounds.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

E3, NU3 = (1.0, 5.0, 50.0), (0.2, 0.3, 0.35)


def iso_mandel(E, nu):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    M = np.zeros((6, 6))
    M[:3, :3] = lam
    M[np.arange(6), np.arange(6)] += 2 * mu
    return M


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--seeds", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=4096)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    import torch

    import paper_1412_8398_amd as fe
    from microstructure import voronoi_cells_torch

    L = args.size
    t0 = time.time()
    def progress(z):
        if z % 64 == 63:
            print(json.dumps({"msg": "labelling", "planes": z + 1, "of": L, "seconds": round(time.time() - t0, 1)}),
                  flush=True)

    phase, _, _ = voronoi_cells_torch((L, L, L), args.seeds, 3, args.seed, progress=progress)
    torch.cuda.synchronize()
    t_gen = time.time() - t0
    print(json.dumps({"msg": "microstructure", "seconds": round(t_gen, 1)}), flush=True)
    frac = (torch.bincount(phase.view(-1), minlength=3).double() / phase.numel()).cpu().numpy()
    with fe.Plan(L, green="R", scheme="AS", precision="fp32", max_iter=3000) as plan:
        torch.cuda.synchronize()
        t0 = time.time()
        Cv, its, st = plan.effective_stiffness(phase, list(E3), list(NU3), args.tol)
        torch.cuda.synchronize()
        t_solve = time.time() - t0
        ws = plan.workspace_bytes
    w = np.array([1, 1, 1, math.sqrt(2), math.sqrt(2), math.sqrt(2)])
    M = Cv * w[:, None] * w[None, :]
    Ms = 0.5 * (M + M.T)
    Cs = [iso_mandel(E, n) for E, n in zip(E3, NU3)]
    voigt = sum(frac[i] * Cs[i] for i in range(3))
    reuss = np.linalg.inv(sum(frac[i] * np.linalg.inv(Cs[i]) for i in range(3)))
    rep = {
        "size": L, "cells": args.seeds, "seed": args.seed, "tol": args.tol, "status": int(st),
        "phase_fractions": frac.tolist(), "iterations": list(its),
        "generation_seconds": round(t_gen, 2), "solve_seconds": round(t_solve, 2),
        "voxel_iterations_per_second": float(L ** 3 * sum(its) / t_solve),
        "workspace_gib": round(ws / 2 ** 30, 1),
        "C_voigt_tensor_shear": Cv.tolist(),
        "asymmetry": float(np.abs(M - M.T).max() / np.abs(M).max()),
        "min_eig": float(np.linalg.eigvalsh(Ms).min()),
        "voigt_minus_C_min_eig": float(np.linalg.eigvalsh(voigt - Ms).min()),
        "C_minus_reuss_min_eig": float(np.linalg.eigvalsh(Ms - reuss).min()),
    }
    print(json.dumps(rep), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(rep, fh, indent=1)
    return 0 if st == fe.FE_OK else 1


if __name__ == "__main__":
    sys.exit(main())
