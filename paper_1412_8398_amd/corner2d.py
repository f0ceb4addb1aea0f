"""The 2D square-inclusion study of §5.1 on the GPU: local stress sigma_12 near
the corner of a quasi-rigid square inclusion for the four Green operators.

Cell: the periodic square [-1/2, 1/2]^2 with one square inclusion of a quarter
of its area, [-1/2, 0) x [0, 1/2) (the simplified four-cell microstructure),
contrast chi = 1e3; matrix with the paper's 2D moduli kappa = 1, mu = 0.6,
lambda = 0.4 (a one-plane cell in plane strain has the in-plane response of
lambda and mu: E = 1.44, nu = 0.2 here); macroscopic strain eps_12 = 1/2.
Accelerated scheme, float64, eta <= tol (the paper iterates to round-off).

Reported per operator and resolution: the largest sigma_12, the share of
pixels above 3.5, the range of sigma_12 in the window [-0.04, 0.04]^2 around
the corner at (0, 0), and the departure from the symmetry of the exact
solution under the point reflection through the inclusion's centre
(sigma_12 is even under it): zero for the centered operators, not for WP.

    python -m paper_1412_8398_amd.corner2d --sizes 512 1024 --out c.json
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
E1, NU = 1.44, 0.2  # lambda = 0.4, mu = 0.6
MACRO = (0.0, 0.0, 0.0, 0.0, 0.0, 0.5)


def square_inclusion(L):
    """(1, L, L) labels: 1 on x in [-1/2, 0), y in [0, 1/2) (pixel centres)."""
    ph = np.zeros((1, L, L), dtype=np.uint8)
    ph[0, L // 2:, : L // 2] = 1  # [z][y][x]: y index >= L/2, x index < L/2
    return ph


def point_reflect(f, L):
    """f[y, x] -> f at the point reflection through the inclusion's centre
    (-1/4, 1/4): pixel x index i -> L/2 - 1 - i, y index j -> 3L/2 - 1 - j (mod L)."""
    i = (L // 2 - 1 - np.arange(L)) % L
    j = (3 * L // 2 - 1 - np.arange(L)) % L
    return f[np.ix_(j, i)]


def study(L, op, tol=1e-11, max_iter=50000):
    import torch

    import paper_1412_8398_amd as fe

    phase = torch.from_numpy(square_inclusion(L)).cuda()
    sig = torch.empty((6, 1, L, L), dtype=torch.float64, device="cuda")
    with fe.Plan((L, L, 1), green=op, scheme="AS", precision="fp64", max_iter=max_iter) as plan:
        torch.cuda.synchronize()
        t0 = time.time()
        r = plan.solve(phase, [E1, CHI * E1], [NU, NU], MACRO, tol, stress=sig, raise_on_error=False)
        torch.cuda.synchronize()
        sec = time.time() - t0
    s12 = sig[5, 0].cpu().numpy()
    x = (np.arange(L) + 0.5) / L - 0.5
    win = np.abs(x) <= 0.04
    w = s12[np.ix_(win, win)]
    asym = float(np.abs(s12 - point_reflect(s12, L)).max() / np.abs(s12).max())
    # oscillation in the window: RMS of the 5-point discrete Laplacian (grid-scale
    # roughness) and the checkerboard component |<sigma_12 (-1)^(i+j)>|
    lap = (np.roll(s12, 1, 0) + np.roll(s12, -1, 0) + np.roll(s12, 1, 1) + np.roll(s12, -1, 1) - 4 * s12)
    lw = lap[np.ix_(win, win)]
    ii, jj = np.meshgrid(np.arange(L)[win], np.arange(L)[win], indexing="ij")
    cb = float(abs(np.mean(w * (-1.0) ** (ii + jj))))
    return {"L": L, "op": op, "iterations": int(r.iterations), "eta": float(r.eta), "status": int(r.status),
            "seconds": round(sec, 2), "max_s12": float(s12.max()), "share_above_3_5": float((s12 > 3.5).mean()),
            "window_min": float(w.min()), "window_max": float(w.max()), "reflection_asymmetry": asym,
            "window_roughness": float(np.sqrt(np.mean(lw * lw))), "window_checkerboard": cb,
            "share_above_1_75": float((s12 > 1.75).mean()), "mean_s12": float(s12.mean())}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=[512, 1024])
    ap.add_argument("--ops", nargs="+", default=["MS", "C", "W", "R"])
    ap.add_argument("--tol", type=float, default=1e-11)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    rows = []
    for L in args.sizes:
        for op in args.ops:
            row = study(L, op, args.tol)
            rows.append(row)
            print(json.dumps(row), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump({"chi": CHI, "E": E1, "nu": NU, "macro": list(MACRO), "tol": args.tol, "rows": rows}, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
