"""Convergence of the effective modulus with the iterations (§6.2) on the GPU.

C_11,11 is estimated at every iteration of the accelerated schemes (AS with
the continuous, centered, WP and rotated operators) as <sigma_11> under the
applied strain eps_bar = e1 (x) e1, on the Boolean medium of §6.1 (L = 64,
radius 2.5, fraction 0.17, seed 1412) carried to a finer grid: the same
sphere centres and radius scaled by L / 64.  Quasi-porous spheres
(chi = 1e-4) at L = 512 and quasi-rigid spheres (chi = 1e4) at L = 256, as in
the paper; float64.

Reference media: §6.2 uses those the §6.1 descent finds on the coarse grid;
here the descent of ``refscan.descend`` at the same contrast on the L = 64
medium, per operator (tol 1e-8).

Per operator: C_11,11 at every iteration (its own limit is the value at the
end of the run, eta <= tol, 1e-7 by default), the first iteration from which the relative
error to that limit stays below 1e-2, and the largest relative error after
iteration 10 (the oscillation the paper describes).

    python -m paper_1412_8398_amd.moduli_rate --out m.json
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

E1, NU = 1.5, 0.25
MACRO = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)
OPS = ("MS", "C", "W", "R")
CASES = (("porous", 1e-4, 512), ("rigid", 1e4, 256))


def medium(L, seed=1412):
    from microstructure import boolean_spheres

    return boolean_spheres((L, L, L), 2.5 * L / 64.0, 0.17, seed)


def settle(c, rel=1e-2):
    """First index from which |c_k / c_end - 1| stays below ``rel``."""
    err = np.abs(c / c[-1] - 1.0)
    bad = np.nonzero(err >= rel)[0]
    return int(bad[-1] + 1) if len(bad) else 0


def optimal_E0(chi, op, cap):
    """The §6.1 descent on the L = 64 medium (AS, tol 1e-8)."""
    import torch

    from paper_1412_8398_amd import refscan

    ph, _ = medium(64)
    cnt = refscan.Counter(torch.from_numpy(ph).cuda(), chi, op, "AS", 1e-8, cap)
    cnt.E = [E1, chi * E1]
    cnt.nu = [NU, NU]
    E0, n, _ = refscan.descend(cnt, math.sqrt(E1 * chi * E1), max_steps=20)
    return E0, n


def run(L, chi, op, E0, tol, cap, scheme="AS"):
    import torch

    import paper_1412_8398_amd as fe

    ph, info = medium(L)
    phase = torch.from_numpy(ph).cuda()
    with fe.Plan(L, green=op, scheme=scheme, precision="fp64", max_iter=cap, ref_rule="explicit", E0=E0,
                 nu0=NU) as plan:
        torch.cuda.synchronize()
        t0 = time.time()
        r = plan.solve(phase, [E1, chi * E1], [NU, NU], MACRO, tol, history=cap + 1, mean_history=True,
                       raise_on_error=False)
        torch.cuda.synchronize()
        sec = time.time() - t0
    del phase
    torch.cuda.empty_cache()
    c = np.asarray(r.mean_stress_history[:, 0])
    return c, r, sec, info


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--cases", nargs="+", default=["porous", "rigid"])
    ap.add_argument("--ops", nargs="+", default=list(OPS))
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--cap", type=int, default=3000)
    ap.add_argument("--scheme", choices=("AS", "CG"), default="AS",
                    help="CG: conjugate gradients (W, R), whose iterates do not depend on E0 (taken as E1)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    rows = []
    for name, chi, L in CASES:
        if name not in args.cases:
            continue
        for op in args.ops:
            if args.scheme == "CG":
                E0, n64 = E1, None
            else:
                E0, n64 = optimal_E0(chi, op, 3000 if chi < 1 else 12000)
            print(json.dumps({"msg": "E0", "case": name, "op": op, "E0": E0, "N64": n64}), flush=True)
            c, r, sec, info = run(L, chi, op, E0, args.tol, args.cap, args.scheme)
            after = np.abs(c[10:] / c[-1] - 1.0) if len(c) > 10 else np.array([0.0])
            row = {"case": name, "scheme": args.scheme, "chi": chi, "L": L, "op": op, "E0": E0,
                   "fraction": info.volume_fraction,
                   "iterations": int(r.iterations), "status": int(r.status), "eta": float(r.eta),
                   "seconds": round(sec, 2), "C1111_limit": float(c[-1]), "settle_1e-2": settle(c),
                   "max_rel_error_after_10": float(after.max()),
                   "C1111_first": [float(v) for v in c[:101]]}
            rows.append(row)
            print(json.dumps({k: v for k, v in row.items() if k != "C1111_first"}), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump({"E1": E1, "nu": NU, "macro": list(MACRO), "tol": args.tol, "rows": rows}, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
