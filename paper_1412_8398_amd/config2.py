"""The scheme x operator x precision matrix on the 256^3 Boolean medium of
the convergence study (§6.1), at contrast 100 and near-porous (1e-6).

    python -m paper_1412_8398_amd.config2 --out c2.json

Medium: Boolean model of Poisson spheres of radius 8 voxels, target volume
fraction 0.3 (seed 2790), matrix E = 1.5 (the paper's units), inclusions
E = chi 1.5, nu = 0.25 in both phases, macroscopic shear eps_12 = 1.
Runs: {direct, accelerated} x {MS, WP, rotated} x {float64, float32} per
contrast, plus conjugate gradients (WP, rotated) in both precisions.
Tolerance 1e-6 on eta (eq. (43)); float32 runs re-anchor in float64 when
their own arithmetic stalls.  Reference media: eqs. (17)/(18) at contrast
100; near-porous, the section's optimised media: direct beta = 0.509, AS
with E0 = 0.01 (MS), 0.7 + sqrt(chi) (WP), 0.12 + sqrt(chi) (rotated), in
units of the matrix modulus, nu0 = 0.25 (conjugate gradients: eq. (17);
their iterates do not depend on the scale of C0).  Iteration cap 5000.

Per run: status, iterations, seconds, eta and its float64 verification,
the effective shear modulus C_12,12 = <sigma_12>/2, and for float32 runs
the relative L2 distance of the strain field to the float64 run of the
same scheme and operator.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

L = 256
RADIUS, FRACTION, SEED = 8.0, 0.3, 2790
E1, NU = 1.5, 0.25
SHEAR = (0.0, 0.0, 0.0, 0.0, 0.0, 1.0)
CAP = 5000


def reference(chi: float, green: str, scheme: str) -> dict:
    """Plan options for the reference medium of one run."""
    if chi >= 1e-3 or scheme == "CG":
        return {}
    if scheme == "DS":
        return {"ds_beta": 0.509}
    e0 = {"MS": 0.01, "W": 0.7 + math.sqrt(chi), "R": 0.12 + math.sqrt(chi)}[green]
    return {"ref_rule": "explicit", "E0": e0 * E1, "nu0": NU}


def runs():
    for chi in (100.0, 1e-6):
        for scheme in ("DS", "AS"):
            for green in ("MS", "W", "R"):
                yield chi, scheme, green
        for green in ("W", "R"):
            yield chi, "CG", green


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--cap", type=int, default=CAP)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    import torch

    import paper_1412_8398_amd as fe
    from microstructure import boolean_spheres

    phase_np, info = boolean_spheres((L, L, L), RADIUS, FRACTION, SEED)
    phase = torch.from_numpy(phase_np).cuda()
    f = float(phase_np.mean())
    print(json.dumps({"msg": "medium", "spheres": info.n_spheres, "fraction": f}), flush=True)
    rows = []
    e64 = torch.empty((6, L, L, L), dtype=torch.float64, device="cuda")
    e32 = torch.empty((6, L, L, L), dtype=torch.float32, device="cuda")
    for chi, scheme, green in runs():
        E = [E1, chi * E1]
        kw = reference(chi, green, scheme)
        for precision in ("fp64", "fp32"):
            eps = e64 if precision == "fp64" else e32
            with fe.Plan(L, green=green, scheme=scheme, precision=precision, max_iter=args.cap, **kw) as plan:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = plan.solve(phase, E, [NU, NU], SHEAR, args.tol, strain=eps, raise_on_error=False)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            row = {"chi": chi, "scheme": scheme, "green": green, "precision": precision,
                   "status": fe.status_string(r.status), "iterations": r.iterations, "seconds": round(dt, 3),
                   "eta": r.eta, "eta_verify_fp64": r.eta_verify_fp64, "refinements": r.refinements,
                   "C_12_12": float(r.mean_stress[5]) / 2.0, "reference": kw or "paper"}
            if precision == "fp32":
                row["strain_rel_l2_vs_fp64"] = float(torch.linalg.vector_norm(e32.double() - e64)
                                                     / torch.linalg.vector_norm(e64))
            rows.append(row)
            print(json.dumps(row), flush=True)
    rep = {"size": L, "spheres": info.n_spheres, "fraction": f, "tol": args.tol, "cap": args.cap, "runs": rows}
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(rep, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
