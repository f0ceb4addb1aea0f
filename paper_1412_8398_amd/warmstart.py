"""Learned warm start versus the plain start eps^0 = eps_bar.

Both runs solve the same cell with the accelerated scheme and the rotated
operator (float32 fields, float64 reductions and re-anchoring) to the same
equilibrium tolerance; the learned run starts from the network's prediction
and its time includes the prediction.

    python -m paper_1412_8398_amd.warmstart --weights w.npy --size 128 --count 16 [--scaled]

Break-even model, per cell.  The scheme contracts the error of its iterate by
a factor rho per iteration (measured: rho = (eta_end / eta_0)^(1/k) of the
plain run), so a start whose error is e times that of eps_bar (e: the
prediction's relative L2 distance to the converged strain, against the
fluctuation eps - eps_bar) saves about log(e) / log(rho) iterations.  The
prediction costs C = t_predict / t_iteration iterations, so the learned start
pays only if e < rho^C (e_breakeven).
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

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_warmstart.npy")


def load_net(path=DEFAULT_WEIGHTS):
    import paper_1412_8398_amd as fe

    net = fe.UNet()
    net.set_params(np.load(path))
    return net


def solve_from_prediction(plan, net, phase, E, nu, macro, tol, strain, pred, history=1):
    """The learned warm start with the applied strain as its fallback: the
    network's prediction (written to ``pred``, device float32 (1, 6, nz, ny, nx))
    starts the plan's solve; a start the scheme cannot bring to equilibrium
    (FE_DIVERGED: eta not finite, or rising for the divergence window) is
    dropped and the solve restarts from eps^0 = eps_bar.  Returns
    (result, predict_seconds, fell_back)."""
    import paper_1412_8398_amd as fe

    _, t_pred = net.predict(phase.unsqueeze(0), [E], [nu], [macro], out=pred)
    r = plan.solve(phase, E, nu, macro, tol, strain_init=pred[0], strain=strain, history=history,
                   raise_on_error=False)
    if r.status == fe.FE_DIVERGED:
        return plan.solve(phase, E, nu, macro, tol, strain=strain, history=history, raise_on_error=False), t_pred, True
    return r, t_pred, False


def scaled_starts(plan, phase, E, nu, macro, tol, eps_star, pred, scales=(0.5, 0.25, 0.1), shares=(0.5, 0.3, 0.1)):
    """Iterations from starts a better prediction could give, around the
    converged strain eps_star (6, nz, ny, nx):
      "pred_x<s>":  eps_star + s (pred - eps_star), the network's own error
                    scaled by s (same shape, e times s);
      "fluct_e<e>": eps_bar + (1 - e)(eps_star - eps_bar), the exact
                    fluctuation scaled down (relative error e, the shape of
                    the solution itself).
    Returns {label: iterations}."""
    import torch

    mac = torch.tensor(np.asarray(macro, dtype=np.float32), device=phase.device).view(6, 1, 1, 1)
    out = {}
    start = torch.empty_like(eps_star)
    eps = torch.empty_like(eps_star)
    for label, make in ([(f"pred_x{sc:g}", lambda sc=sc: eps_star + sc * (pred - eps_star)) for sc in scales] +
                        [(f"fluct_e{e:g}", lambda e=e: mac + (1.0 - e) * (eps_star - mac)) for e in shares]):
        start.copy_(make())
        r = plan.solve(phase, E, nu, macro, tol, strain_init=start, strain=eps, history=1, raise_on_error=False)
        out[label] = int(r.iterations) if r.status == 0 else None
    return out


def compare_one(net, phase, E, nu, macro, tol=1e-6, max_iter=3000, plan=None, scaled=False):
    """Plain and learned solves of one cell; returns a dict of measurements.
    ``phase`` is a device uint8 tensor (nz, ny, nx)."""
    import torch

    import paper_1412_8398_amd as fe

    nz, ny, nx = (int(v) for v in phase.shape)
    own = plan is None
    if own:
        plan = fe.Plan((nx, ny, nz), green="R", scheme="AS", precision="fp32", max_iter=max_iter)
    eps_p = torch.empty((6, nz, ny, nx), dtype=torch.float32, device=phase.device)
    eps_l = torch.empty_like(eps_p)
    pred = torch.empty((1, 6, nz, ny, nx), dtype=torch.float32, device=phase.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rp = plan.solve(phase, E, nu, macro, tol, strain=eps_p, history=1, raise_on_error=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rl, t_pred, fell_back = solve_from_prediction(plan, net, phase, E, nu, macro, tol, eps_l, pred)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    mac = torch.tensor(np.asarray(macro, dtype=np.float32), device=phase.device).view(6, 1, 1, 1)
    fluct = torch.linalg.vector_norm((eps_p - mac).double()).item()
    pred_err = torch.linalg.vector_norm((pred[0] - eps_p).double()).item() / max(fluct, 1e-300)
    sp, sl = np.asarray(rp.mean_stress), np.asarray(rl.mean_stress)
    hist = np.asarray(rp.eta_history, dtype=np.float64)
    k = max(int(rp.iterations), 1)
    rho = float((rp.eta_verify_fp64 / hist[0]) ** (1.0 / k)) if hist.size and hist[0] > 0 else float("nan")
    t_iter = (t1 - t0) / k
    cost = t_pred / t_iter
    out = {
        "plain": {"iterations": rp.iterations, "seconds": t1 - t0, "eta0": float(rp.eta_history[0]),
                  "eta": rp.eta_verify_fp64, "status": rp.status},
        "learned": {"iterations": rl.iterations, "seconds": t2 - t1, "predict_seconds": t_pred,
                    "eta0": float(rl.eta_history[0]), "eta": rl.eta_verify_fp64, "status": rl.status,
                    "fell_back": fell_back},
        "prediction_rel_l2": pred_err,
        "mean_stress_rel_diff": float(np.linalg.norm(sl - sp) / max(np.linalg.norm(sp), 1e-300)),
        "rho": rho,
        "iteration_seconds": t_iter,
        "prediction_cost_iterations": cost,
        "iterations_saved": int(rp.iterations) - int(rl.iterations),
        "iterations_saved_model": float(np.log(pred_err) / np.log(rho)) if 0 < rho < 1 else float("nan"),
        "e_breakeven": float(rho ** cost) if 0 < rho < 1 else float("nan"),
    }
    if scaled:
        out["scaled_starts"] = scaled_starts(plan, phase, E, nu, macro, tol, eps_p, pred[0])
    if own:
        plan.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--count", type=int, default=16)
    ap.add_argument("--seed", type=int, default=5141230)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--out", default=None)
    ap.add_argument("--scaled", action="store_true",
                    help="also solve from the network's error scaled down and from scaled exact fluctuations")
    args = ap.parse_args(argv)

    from microstructure import batch_samples

    samples = batch_samples(args.count, args.seed, sizes=(args.size,))
    import torch

    import paper_1412_8398_amd as fe

    net = load_net(args.weights)
    rows = []
    with fe.Plan(args.size, green="R", scheme="AS", precision="fp32", max_iter=3000) as plan:
        s = samples[0]  # warm-up: first launches and workspace, not reported
        compare_one(net, torch.from_numpy(s.phase).cuda(), [1.0, s.contrast], [s.nu, s.nu], s.macro_strain,
                    args.tol, plan=plan)
        for i, s in enumerate(samples):
            ph = torch.from_numpy(s.phase).cuda()
            r = compare_one(net, ph, [1.0, s.contrast], [s.nu, s.nu], s.macro_strain, args.tol, plan=plan,
                            scaled=args.scaled)
            r.update({"sample": i, "L": s.L, "contrast": s.contrast, "fraction": s.volume_fraction, "radius": s.radius,
                      "nu": s.nu, "load": s.load, "seed": s.seed})
            rows.append(r)
            print(json.dumps(r), flush=True)
    it_p = np.array([r["plain"]["iterations"] for r in rows])
    it_l = np.array([r["learned"]["iterations"] for r in rows])
    t_p = np.array([r["plain"]["seconds"] for r in rows])
    t_l = np.array([r["learned"]["seconds"] for r in rows])
    summ = {"size": args.size, "count": args.count, "tol": args.tol,
            "iterations_plain_mean": float(it_p.mean()), "iterations_learned_mean": float(it_l.mean()),
            "seconds_plain_total": float(t_p.sum()), "seconds_learned_total": float(t_l.sum()),
            "prediction_rel_l2_median": float(np.median([r["prediction_rel_l2"] for r in rows])),
            "eta0_plain_median": float(np.median([r["plain"]["eta0"] for r in rows])),
            "eta0_learned_median": float(np.median([r["learned"]["eta0"] for r in rows])),
            "mean_stress_rel_diff_max": float(max(r["mean_stress_rel_diff"] for r in rows)),
            "speedup": float(t_p.sum() / t_l.sum()),
            "rho_median": float(np.median([r["rho"] for r in rows])),
            "prediction_cost_iterations_median": float(np.median([r["prediction_cost_iterations"] for r in rows])),
            "iterations_saved_mean": float(np.mean([r["iterations_saved"] for r in rows])),
            "iterations_saved_model_mean": float(np.mean([r["iterations_saved_model"] for r in rows])),
            "e_breakeven_median": float(np.median([r["e_breakeven"] for r in rows]))}
    if args.scaled:
        # iterations saved against the plain start, per start family, over all
        # cells and over the slow ones (rho > 0.8), beside the prediction's cost
        labels = list(rows[0]["scaled_starts"])
        slow = [r for r in rows if r["rho"] > 0.8]
        saved = {}
        for lab in labels:
            d_all = [r["plain"]["iterations"] - r["scaled_starts"][lab] for r in rows if r["scaled_starts"][lab] is not None]
            d_slow = [r["plain"]["iterations"] - r["scaled_starts"][lab] for r in slow
                      if r["scaled_starts"][lab] is not None]
            saved[lab] = {"mean": float(np.mean(d_all)) if d_all else None,
                          "mean_rho_gt_0.8": float(np.mean(d_slow)) if d_slow else None}
        summ["scaled_starts_saved"] = saved
    print(json.dumps({"summary": summ}), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump({"summary": summ, "rows": rows}, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
