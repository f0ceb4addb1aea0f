"""Solver-generated training data and training of the warm-start network.

    python -m paper_1412_8398_amd.train --samples 20000 --epochs 3 --out weights.npy

Samples follow the batched-solve distribution of ``microstructure.batch_samples``
(sphere-Boolean cells of edge 32, 48, 64 or 96 voxels, volume fraction
U[0.05, 0.4], log10 contrast U[-2, 3], one Poisson ratio U[0.2, 0.4], radius
U[3, 8], one unit macroscopic strain).  Their strain fields are computed by
``fe_solve_batched`` (accelerated scheme, rotated operator, float32 fields,
float64 reductions) and kept on the device in bfloat16; the network is then
trained on them with ``fe_unet_train_step`` (Adam, warm-up and cosine step-size decay).
Everything numerical runs in the library; this module only moves batches.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _log(msg, **kw):
    print(json.dumps({"t": round(time.time() - _T0, 1), "msg": msg, **kw}), flush=True)


_T0 = time.time()


def _phase_of(args):
    from microstructure import boolean_spheres

    L, r, f, seed = args
    return boolean_spheres((L, L, L), r, f, seed)[0]


def make_samples(n: int, seed: int, workers: int, sizes=(32, 48, 64, 96)):
    """Config-4 samples with their phase maps (generated in worker processes;
    call before the GPU is initialised)."""
    from microstructure import batch_samples

    smp = batch_samples(n, seed, sizes=sizes, with_phase=False)
    jobs = [(s.L, s.radius, s.volume_fraction, s.seed) for s in smp]
    if workers > 1:
        with mp.get_context("fork").Pool(workers) as pool:
            phases = pool.map(_phase_of, jobs, chunksize=8)
    else:
        phases = [_phase_of(j) for j in jobs]
    for s, p in zip(smp, phases):
        s.phase = p
    return smp


class Dataset:
    """Phase maps (uint8) and solver strains (bfloat16) per grid size, on the device."""

    def __init__(self, samples):
        import torch

        self.samples = samples
        self.classes = {}
        self.where = {}
        for L in sorted({s.L for s in samples}):
            idx = [i for i, s in enumerate(samples) if s.L == L]
            ph = torch.empty((len(idx), L, L, L), dtype=torch.uint8, device="cuda")
            for k, i in enumerate(idx):
                ph[k].copy_(torch.from_numpy(samples[i].phase))
                self.where[i] = (L, k)
            self.classes[L] = {"idx": idx, "phase": ph,
                               "target": torch.empty((len(idx), 6, L, L, L), dtype=torch.bfloat16, device="cuda")}
        self.iterations = np.zeros(len(samples), dtype=np.int64)
        self.status = np.zeros(len(samples), dtype=np.int64)
        self.eta = np.zeros(len(samples))

    def voxels(self):
        return sum(s.L ** 3 for s in self.samples)

    def solve(self, tol=1e-6, max_iter=1500, chunk=512, launch="per_pass"):
        """Strain targets from batched solves of ``chunk`` samples at a time
        (``launch``: fe_plan_options.batch_launch, "per_pass" or "persistent")."""
        import torch

        import paper_1412_8398_amd as fe

        n = len(self.samples)
        t0 = time.time()
        vox_iter = 0
        for a in range(0, n, chunk):
            ids = list(range(a, min(n, a + chunk)))
            specs, outs = [], []
            for i in ids:
                s = self.samples[i]
                L, k = self.where[i]
                eps = torch.empty((6, L, L, L), dtype=torch.float32, device="cuda")
                specs.append(fe.BatchSampleSpec(self.classes[L]["phase"][k], [1.0, s.contrast], [s.nu, s.nu],
                                                s.macro_strain, eps))
                outs.append((i, L, k, eps))
            res, status, sec = fe.solve_batched(specs, tol, green="R", scheme="AS", precision="fp32", max_iter=max_iter,
                                                launch=launch)
            for (i, L, k, eps), r in zip(outs, res):
                self.classes[L]["target"][k].copy_(eps.to(torch.bfloat16))
                self.iterations[i], self.status[i], self.eta[i] = r.iterations, r.status, r.eta
                vox_iter += self.samples[i].L ** 3 * r.iterations
            del specs, outs
            _log("solved", done=ids[-1] + 1, of=n, batch_seconds=round(sec, 2),
                 gvox_iter_per_s=round(sum(self.samples[i].L ** 3 * self.iterations[i] for i in ids) / max(sec, 1e-9) / 1e9, 2),
                 not_converged=int(np.sum(self.status[ids] != 0)))
        nc = self.status != 0
        return {"seconds": time.time() - t0, "voxel_iterations": int(vox_iter),
                "iterations_mean": float(self.iterations.mean()), "iterations_max": int(self.iterations.max()),
                "not_converged": int(np.sum(nc)),
                "eta_not_converged_median": float(np.median(self.eta[nc])) if nc.any() else None,
                "eta_not_converged_max": float(np.max(self.eta[nc])) if nc.any() else None,
                "eta_max": float(np.max(self.eta))}

    def batch(self, L, ks):
        import torch

        c = self.classes[L]
        kt = torch.as_tensor(ks, dtype=torch.long, device="cuda")
        ph = c["phase"].index_select(0, kt).contiguous()
        tg = c["target"].index_select(0, kt).contiguous()
        smp = [self.samples[c["idx"][k]] for k in ks]
        E = [[1.0, s.contrast] for s in smp]
        nu = [[s.nu, s.nu] for s in smp]
        macro = np.stack([s.macro_strain for s in smp])
        return ph, E, nu, macro, tg

    def batches(self, batch_voxels, rng):
        out = []
        for L, c in self.classes.items():
            B = max(1, batch_voxels // L ** 3)
            perm = rng.permutation(len(c["idx"]))
            out += [(L, perm[i:i + B]) for i in range(0, len(perm), B)]
        order = rng.permutation(len(out))
        return [out[i] for i in order]


def evaluate_loss(net, data: Dataset, batch_voxels=1 << 20):
    tot, w = 0.0, 0
    for L, c in data.classes.items():
        B = max(1, batch_voxels // L ** 3)
        for a in range(0, len(c["idx"]), B):
            ks = list(range(a, min(len(c["idx"]), a + B)))
            ph, E, nu, macro, tg = data.batch(L, ks)
            tot += net.loss_grad(ph, E, nu, macro, tg) * len(ks) * L ** 3
            w += len(ks) * L ** 3
    return tot / w


def train(net, data: Dataset, epochs: float, lr=1e-4, batch_voxels=1 << 20, seed=0, val=None, time_budget=None,
          warmup=300):
    """Adam with a linear warm-up over ``warmup`` steps and cosine decay to 2%
    of ``lr``.  Without normalisation layers the relu network dies at larger
    step sizes (1e-3 left every unit of the last block inactive within one
    epoch); 1e-4 trains steadily."""
    rng = np.random.default_rng(seed)
    per_epoch = len(data.batches(batch_voxels, np.random.default_rng(0)))
    total = max(1, int(round(epochs * per_epoch)))
    step, t0, hist = 0, time.time(), []
    last_log = t0
    while step < total:
        for L, ks in data.batches(batch_voxels, rng):
            if step >= total or (time_budget and time.time() - t0 > time_budget):
                break
            warm = min(1.0, (step + 1) / warmup)
            net.set_learning_rate(lr * warm * (0.02 + 0.98 * 0.5 * (1.0 + math.cos(math.pi * step / total))))
            ph, E, nu, macro, tg = data.batch(L, list(ks))
            loss = net.train_step(ph, E, nu, macro, tg)
            hist.append(loss)
            step += 1
            if time.time() - last_log > 20:
                last_log = time.time()
                _log("train", step=step, of=total, loss=round(float(np.mean(hist[-50:])), 6),
                     steps_per_s=round(step / (time.time() - t0), 2))
        if time_budget and time.time() - t0 > time_budget:
            _log("time budget reached", step=step, of=total)
            break
        if val is not None:
            _log("validation", step=step, loss=round(evaluate_loss(net, val, batch_voxels), 6))
    return {"steps": step, "planned_steps": total, "seconds": time.time() - t0,
            "final_train_loss": float(np.mean(hist[-50:])) if hist else None}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=20000)
    ap.add_argument("--val-samples", type=int, default=256)
    ap.add_argument("--seed", type=int, default=20141230)
    ap.add_argument("--epochs", type=float, default=3.0)
    ap.add_argument("--lr", type=float, default=1e-4)
    ap.add_argument("--batch-voxels", type=int, default=1 << 20)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=1500)
    ap.add_argument("--launch", choices=["per_pass", "persistent"], default="per_pass",
                    help="batched-solve launch of the data generation (per_pass is the faster on MI355X)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--time-budget", type=float, default=None, help="seconds of training at most")
    ap.add_argument("--init", default=None, help="start from these parameters (.npy)")
    ap.add_argument("--out", required=True, help="trained parameters (.npy, float32, canonical order)")
    ap.add_argument("--report", default=None, help="JSON summary")
    args = ap.parse_args(argv)

    # inputs first: the generator runs in forked workers, before any GPU use
    train_s = make_samples(args.samples, args.seed, args.workers)
    val_s = make_samples(args.val_samples, args.seed + 1, args.workers)
    _log("microstructures", train=len(train_s), val=len(val_s),
         voxels=int(sum(s.L ** 3 for s in train_s)))

    import torch

    import paper_1412_8398_amd as fe

    assert torch.cuda.is_available(), "training needs a GPU"
    data = Dataset(train_s)
    rep = {"data": data.solve(args.tol, args.max_iter, launch=args.launch)}
    val = Dataset(val_s)
    rep["val_data"] = val.solve(args.tol, args.max_iter, launch=args.launch)
    net = fe.UNet(lr=args.lr)
    if args.init:
        net.set_params(np.load(args.init))
    rep["val_loss_initial"] = evaluate_loss(net, val, args.batch_voxels)
    _log("validation", step=0, loss=round(rep["val_loss_initial"], 6))
    rep["train"] = train(net, data, args.epochs, args.lr, args.batch_voxels, args.seed, val, args.time_budget)
    rep["val_loss_final"] = evaluate_loss(net, val, args.batch_voxels)
    np.save(args.out, net.get_params())
    rep.update({"samples": args.samples, "val_samples": args.val_samples, "seed": args.seed, "epochs": args.epochs,
                "lr": args.lr, "batch_voxels": args.batch_voxels, "tol": args.tol, "max_iter": args.max_iter,
                "out": args.out})
    _log("done", **{k: v for k, v in rep.items() if not isinstance(v, dict)})
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(rep, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
