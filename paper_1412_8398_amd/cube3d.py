"""The 3D cubic-inclusion study of §5.2 on the GPU: sigma_12 for one
quasi-rigid cube (one of the eight cubes of the periodic cell, volume fraction
12.5%) centred in the cell, for the four Green operators.

Cell: voxel i along each axis covers [i/L - 1/2, (i+1)/L - 1/2); the
inclusion is [-1/4, 1/4)^3, voxels L/4 <= i < 3L/4 on every axis; contrast
chi = 1e3; the paper's 3D matrix moduli kappa = 1, mu = 0.6, lambda = 0.6
(E = 1.5, nu = 0.25, the same in the inclusion); macroscopic strain
eps_12 = 1/2 (the loading of the 2D study).  Accelerated scheme, float64,
eta <= tol (the paper iterates to round-off).

Reported per operator and resolution: the largest sigma_12 and the share of
voxels above 8.5 (the paper's colour threshold, under 0.04% of its voxels);
the departure from the symmetries of the exact solution, which is even in
sigma_12 under each of the three mirrors through the cell centre
(i -> L - 1 - i); and on the paper's section x_3 = -0.2461 (voxel plane
i_3 = round(0.2539 L), inside the inclusion next to its face) the grid-scale
roughness of sigma_12 over the inclusion's part of the section (RMS of the
5-point Laplacian) and, between successive resolutions, the relative L2
distance of the section to the 2 x 2 block average of the finer one.

    python -m paper_1412_8398_amd.cube3d --sizes 256 512 --out c.json
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

CHI = 1e3
E1, NU = 1.5, 0.25  # kappa = 1, mu = 0.6, lambda = 0.6
MU1 = E1 / (2 * (1 + NU))
MACRO = (0.0, 0.0, 0.0, 0.0, 0.0, 0.5)
SECTION_X3 = -0.2461
THRESHOLD = 8.5


def cube_inclusion(L):
    """(L, L, L) labels [z][y][x]: 1 on the centred cube L/4 <= i < 3L/4."""
    if L % 4:
        raise ValueError("L must be a multiple of 4")
    ph = np.zeros((L, L, L), dtype=np.uint8)
    a, b = L // 4, 3 * L // 4
    ph[a:b, a:b, a:b] = 1
    return ph


def section_index(L):
    """Voxel plane whose lower face is nearest to x_3 = -0.2461."""
    return int(round((SECTION_X3 + 0.5) * L))


def coarsen2(s):
    """2 x 2 block average of a square section."""
    n = s.shape[0] // 2
    return s.reshape(n, 2, n, 2).mean(axis=(1, 3))


def study(L, op, tol=1e-11, max_iter=50000):
    """Solve the L^3 cell with operator ``op``; returns (row, section of
    sigma_12 at the paper's plane as a float64 array)."""
    import torch

    import paper_1412_8398_amd as fe

    phase = torch.from_numpy(cube_inclusion(L)).cuda()
    eps = torch.empty((6, L, L, L), dtype=torch.float64, device="cuda")
    with fe.Plan(L, green=op, scheme="AS", precision="fp64", max_iter=max_iter) as plan:
        torch.cuda.synchronize()
        t0 = time.time()
        r = plan.solve(phase, [E1, CHI * E1], [NU, NU], MACRO, tol, strain=eps, raise_on_error=False)
        torch.cuda.synchronize()
        sec = time.time() - t0
    # sigma_12 = 2 mu eps_12 (tensor component), mu per phase
    mu = torch.tensor([MU1, CHI * MU1], dtype=torch.float64, device="cuda")
    s12 = 2.0 * mu[phase.long()] * eps[5]
    del eps
    peak = float(s12.abs().max())
    asym = max(float((s12 - torch.flip(s12, dims=(a,))).abs().max()) for a in (0, 1, 2)) / peak
    k = section_index(L)
    sec_np = s12[k].cpu().numpy()
    row = {"L": L, "op": op, "iterations": int(r.iterations), "eta": float(r.eta), "status": int(r.status),
           "seconds": round(sec, 2), "max_s12": float(s12.max()), "min_s12": float(s12.min()),
           "share_above_8_5": float((s12 > THRESHOLD).double().mean()), "mean_s12": float(s12.mean()),
           "mirror_asymmetry": asym, "section_plane": k}
    del s12, phase
    torch.cuda.empty_cache()
    a, b = L // 4, 3 * L // 4
    lap = (np.roll(sec_np, 1, 0) + np.roll(sec_np, -1, 0) + np.roll(sec_np, 1, 1) + np.roll(sec_np, -1, 1)
           - 4 * sec_np)
    inner = lap[a:b, a:b]
    row["section_inclusion_roughness"] = float(np.sqrt(np.mean(inner * inner)))
    row["section_max"] = float(sec_np.max())
    row["section_min"] = float(sec_np.min())
    return row, sec_np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=[256, 512])
    ap.add_argument("--ops", nargs="+", default=["MS", "C", "W", "R"])
    ap.add_argument("--tol", type=float, default=1e-11)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    rows, sections = [], {}
    for L in sorted(args.sizes):
        for op in args.ops:
            row, sec = study(L, op, args.tol)
            prev = sections.get((L // 2, op))
            if prev is not None:
                row["section_distance_to_half_resolution"] = float(
                    np.linalg.norm(coarsen2(sec) - prev) / np.linalg.norm(prev))
            sections[(L, op)] = sec
            rows.append(row)
            print(json.dumps(row), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump({"chi": CHI, "E": E1, "nu": NU, "macro": list(MACRO), "tol": args.tol,
                       "section_x3": SECTION_X3, "rows": rows}, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
