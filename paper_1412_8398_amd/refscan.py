"""Reference-medium study of §6.1 on the GPU: the iteration count N(E0) to
reach eta <= tol as a function of the reference Young modulus E0 (nu0 = 0.25),
and the paper's descent rule for the E0 that minimises it.

The medium is the paper's §6.1 Boolean model of spheres: L = 64, diameter 5
voxels (radius 2.5), volume fraction 17% (Poisson count with mean 746 for the
stated intensity), matrix E1 = 1.5, inclusions E2 = chi E1, nu = 0.25 in both
phases, macroscopic shear eps_12 = 1, float64 fields, tol 1e-8.

    python -m paper_1412_8398_amd.refscan --mode scan --chi 1e-5
    python -m paper_1412_8398_amd.refscan --mode descent --out d.json
    python -m paper_1412_8398_amd.refscan --mode scan --scheme CG --chi 10

Descent (§6.1): start from E0 = 0.51 (E1 + E2) for the direct scheme and
E0 = sqrt(E1 E2) for the accelerated one; at each step compare N(E0) with
N(E0 + dE0), dE0 = 0.01 E0, and move towards the smaller count, or, when the
counts are equal, towards the smaller eta after that many iterations; stop
when N(E0) is unchanged after two descent steps.  The paper does not state
how far a step moves E0: here E0 is multiplied or divided by a factor that
starts at 1.1, is squared (up to 2) while the direction holds until the
first reversal and square-rooted at every reversal; the two unchanged steps
of the stop rule count once the factor is below 1.05 (plateaus are crossed
first).  A run whose eta becomes non-finite counts as worse than the
iteration cap; when both runs of a comparison diverge the step goes to the
stiffer reference medium.
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

E1 = 1.5
NU = 0.25
MACRO = (0.0, 0.0, 0.0, 0.0, 0.0, 1.0)
OPS = ("MS", "C", "W", "R")


def descend(count, E0_start, max_steps=30, factor=1.1, max_factor=2.0, settle=1.05):
    """The descent rule on a counting function ``count(E0) -> (N, eta_N)``
    (N: first iteration with eta <= tol or the cap; eta_N: eta after N
    iterations).  Returns (best E0, best N, visited list of (E0, N, eta))."""
    E = float(E0_start)
    N, eta = count(E)
    visited = [(E, N, eta)]
    best = (E, N, eta)
    unchanged, last_dir, bracketed = 0, 0, False
    for _ in range(max_steps):
        Nd, etad = count(E * 1.01)
        visited.append((E * 1.01, Nd, etad))
        if Nd != N:
            direction = 1 if Nd < N else -1
        elif math.isinf(eta) and math.isinf(etad):
            direction = 1  # both diverge: a stiffer reference medium restores convergence (beta < 1/2, §6.1)
        else:
            direction = 1 if etad < eta else -1
        if last_dir and direction != last_dir:
            factor = math.sqrt(factor)
            bracketed = True
        elif last_dir and not bracketed:
            factor = min(factor * factor, max_factor)
        last_dir = direction
        E = E * factor ** direction
        Nn, etan = count(E)
        visited.append((E, Nn, etan))
        unchanged = unchanged + 1 if (Nn == N and factor < settle) else 0
        N, eta = Nn, etan
        if (N, eta) < (best[1], best[2]):
            best = (E, N, eta)
        if unchanged >= 2:
            break
    return best[0], best[1], visited


class Counter:
    """N(E0) on one GPU for a fixed medium, operator and scheme (float64)."""

    def __init__(self, phase, chi, op, scheme, tol=1e-8, cap=3000):
        import paper_1412_8398_amd as fe

        self.fe = fe
        self.phase = phase
        self.E = [E1, chi * E1]
        self.nu = [NU, NU]
        self.op, self.scheme, self.tol, self.cap = op, scheme, tol, cap
        self.L = int(phase.shape[0])
        self.calls = 0
        self.iterations = 0

    def __call__(self, E0):
        with self.fe.Plan(self.L, green=self.op, scheme=self.scheme, precision="fp64", max_iter=self.cap,
                          ref_rule="explicit", E0=float(E0), nu0=NU, diverge_window=0) as plan:
            r = plan.solve(self.phase, self.E, self.nu, MACRO, self.tol, history=self.cap + 1,
                           raise_on_error=False)
        self.calls += 1
        self.iterations += r.iterations
        eta = float(r.eta_history[r.iterations]) if len(r.eta_history) > r.iterations else float(r.eta)
        if r.status == self.fe.FE_DIVERGED or not math.isfinite(eta):
            return self.cap + 1, math.inf  # worse than any run that stays finite
        return int(r.iterations), eta


def medium(L=64, seed=1412):
    from microstructure import boolean_spheres

    phase, info = boolean_spheres((L, L, L), 2.5, 0.17, seed)
    return phase, info


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", choices=("scan", "descent", "both"), default="both")
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--seed", type=int, default=1412)
    ap.add_argument("--chi", type=float, default=1e-5, help="contrast of the scan")
    ap.add_argument("--scheme", choices=("AS", "DS", "CG"), default="AS",
                    help="scheme of the scan (CG: conjugate gradients, WP and rotated operators)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--cap", type=int, default=3000)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    import torch

    ph_np, info = medium(args.L, args.seed)
    phase = torch.from_numpy(ph_np).cuda()
    out = {"L": args.L, "seed": args.seed, "spheres": info.n_spheres, "fraction": info.volume_fraction,
           "E1": E1, "nu": NU, "nu0": NU, "tol": args.tol, "cap": args.cap, "macro": list(MACRO)}
    print(json.dumps({"msg": "medium", "spheres": info.n_spheres, "fraction": info.volume_fraction}), flush=True)
    t0 = time.time()
    if args.mode in ("scan", "both"):
        grid = [0.005, 0.01, 0.02, 0.03, 0.04, 0.05, 0.06, 0.07, 0.08, 0.09, 0.1, 0.12, 0.14, 0.17, 0.2, 0.25,
                0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0]
        scan = {}
        ops = ("W", "R") if args.scheme == "CG" else OPS
        for op in ops:
            cnt = Counter(phase, args.chi, op, args.scheme, args.tol, args.cap)
            scan[op] = []
            for E0 in grid:
                n, eta = cnt(E0)
                scan[op].append([E0, n, eta])
            best = min(scan[op], key=lambda r: (r[1], r[2]))
            print(json.dumps({"msg": "scan", "op": op, "scheme": args.scheme, "chi": args.chi, "best_E0": best[0],
                              "best_N": best[1], "N": [r[1] for r in scan[op]],
                              "seconds": round(time.time() - t0, 1)}), flush=True)
        out["scan"] = {"chi": args.chi, "scheme": args.scheme, "E0": grid,
                       "N": {op: [r[1] for r in scan[op]] for op in ops},
                       "eta": {op: [r[2] for r in scan[op]] for op in ops}}
    if args.mode in ("descent", "both"):
        cases = [("AS", chi) for chi in (1e-5, 1e-3, 1e-1, 1e1, 1e3, 1e5)] + [("DS", chi) for chi in (1e-2, 1e2)]
        rows = []
        for scheme, chi in cases:
            E2 = chi * E1
            start = 0.51 * (E1 + E2) if scheme == "DS" else math.sqrt(E1 * E2)
            cap = args.cap if 1e-4 < chi < 1e4 else 4 * args.cap  # slow extremes (AS ~ 1/sqrt(chi), sqrt(chi))
            for op in OPS:
                cnt = Counter(phase, chi, op, scheme, args.tol, cap)
                E0, n, visited = descend(cnt, start, max_steps=20)
                row = {"scheme": scheme, "op": op, "chi": chi, "cap": cap, "E0_start": start, "N_start": visited[0][1],
                       "E0": E0, "N": n, "beta": E0 / (E1 + E2), "E0_over_sqrt": E0 / math.sqrt(E1 * E2),
                       "solves": cnt.calls, "iterations": cnt.iterations}
                rows.append(row)
                print(json.dumps(dict(row, msg="descent", seconds=round(time.time() - t0, 1))), flush=True)
        out["descent"] = rows
    out["seconds"] = round(time.time() - t0, 1)
    print(json.dumps({"msg": "done", "seconds": out["seconds"]}), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
