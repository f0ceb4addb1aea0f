"""Benchmark of the Lippmann-Schwinger FFT iteration on one MI355X.

Workload (one "step" = one full iteration: divergence stencil, forward 3D
transform, Green operator, inverse 3D transform, strain update, float64
equilibrium-norm reduction):
  512^3 sphere-Boolean microstructure (Poisson spheres of radius 6 voxels,
  target volume fraction 0.25, seed 20141230), inclusion/matrix Young's
  moduli 10 / 1, nu = 0.3 in both phases, macroscopic shear eps_12 = 1,
  accelerated scheme with the rotated-grid Green operator, float32 fields,
  float64 reductions; reference medium by the geometric-mean rule.

Prints one JSON line.  Also reports the time to eta <= 1e-6 from the plain
start (eps^0 = eps_bar) and from the learned warm start (the U-Net prediction,
inference time included), and the FP64 CPU oracle's rate on a bounded sample
of the same recipe.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "voxel-iter/s & time to 1e-6 equilibrium at 512^3: plain vs learned warm start"
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E peak

RECIPE = dict(radius=6.0, fraction=0.25, E=(1.0, 10.0), nu=(0.3, 0.3), seed=20141230)
MACRO = (0.0, 0.0, 0.0, 0.0, 0.0, 1.0)  # eps_12 = 1 (tensor Voigt order)


def make_phase(L: int):
    from microstructure import boolean_spheres

    phase, info = boolean_spheres((L, L, L), RECIPE["radius"], RECIPE["fraction"], RECIPE["seed"])
    return phase, info


def pass_bytes(L: int, elem: int = 4):
    """Algorithmic HBM bytes of one launch of each pass (displacement form,
    3-component spectra, accelerated scheme), for an L^3 grid.  "pointwise"
    (the stand-alone divergence) runs once per solve and after each float64
    re-anchor; every other iteration gets it from the fused "update"."""
    N = L ** 3
    H = L // 2 + 1
    spec = 3 * H * L * L * 2 * elem        # 3 half spectra along z, complex
    real3 = 3 * N * elem                   # 3 real planes (divergence / displacement)
    strain = 6 * N * elem
    return {
        "pointwise": strain + N + real3,              # read eps, phase; write D
        "zfwd": real3 + spec,                         # read D; write half spectra
        "yfwd": 2 * spec,                             # read + write in place
        "xgreen": 2 * spec,
        "yinv": 2 * spec,
        "zinv": spec + real3,                         # read half spectra; write U
        # fused strain update and divergence: read U, eps^k, phase; write eps^(k+1), D
        "update": real3 + strain + N + strain + real3,
    }


def traffic_file(L: int) -> str:
    """The committed per-pass traffic record of an L^3 run (paper_1412_8398_amd.traffic)."""
    return os.path.join(ROOT, "profiles", f"traffic_ASR_fp32_{L}.json")


def measured_traffic(pass_name: str, L: int):
    """HBM bytes per launch of a pass from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE counters (scaled by a 1 GiB copy's readings), or None when the
    counters were taken on another grid or the kernel's sources changed since."""
    import hashlib

    if not os.path.exists(traffic_file(L)):
        return None
    with open(traffic_file(L)) as fh:
        rec = json.load(fh).get("kernels", {}).get(pass_name)
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, "paper_1412_8398_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return int(round(rec["bytes"]))


def time_to_tolerance(fe, torch, np, phase, E, nu, L, weights):
    """Time to eta <= 1e-6 from the plain start (eps^0 = eps_bar) and from the
    learned warm start (network prediction, its time included), same plan,
    same tolerance; float64 re-anchoring as the plan's default.  The plan's
    first solve allocates the re-anchoring workspace: it is timed separately
    (first_call_seconds) and the reported times are those of a warm plan.  A
    learned start the scheme cannot bring to equilibrium falls back to eps_bar
    (``warmstart.solve_from_prediction``), inside the timed region."""
    from paper_1412_8398_amd.warmstart import solve_from_prediction

    tol = 1e-6
    eps = torch.empty((6, L, L, L), dtype=torch.float32, device="cuda")
    out = {"tol": tol}
    with fe.Plan(L, green="R", scheme="AS", precision="fp32", max_iter=2000) as plan:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.solve(phase, E, nu, MACRO, tol, strain=eps, history=1)
        torch.cuda.synchronize()
        t_first = time.perf_counter() - t0
        t0 = time.perf_counter()
        r = plan.solve(phase, E, nu, MACRO, tol, strain=eps, history=1)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        out["plain"] = {"seconds": round(t_plain, 4), "first_call_seconds": round(t_first, 4),
                        "iterations": r.iterations, "status": r.status,
                        "eta0": float(r.eta_history[0]), "eta": r.eta, "eta_verify_fp64": r.eta_verify_fp64,
                        "refinements": r.refinements, "C_12_12": float(r.mean_stress[5]) / 2.0}
        out["learned"] = None
        if weights and os.path.exists(weights):
            net = fe.UNet()
            net.set_params(np.load(weights))
            pred = torch.empty((1, 6, L, L, L), dtype=torch.float32, device="cuda")
            net.predict(phase.unsqueeze(0), [E], [nu], [MACRO], out=pred)  # workspace and first launches
            eps_l = torch.empty_like(eps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rl, t_pred, fell_back = solve_from_prediction(plan, net, phase, E, nu, MACRO, tol, eps_l, pred)
            torch.cuda.synchronize()
            t_learned = time.perf_counter() - t0
            mac = torch.tensor(MACRO, dtype=torch.float32, device="cuda").view(6, 1, 1, 1)
            err = (torch.linalg.vector_norm((pred[0] - eps).double())
                   / torch.linalg.vector_norm((eps - mac).double())).item()
            out["learned"] = {"seconds": round(t_learned, 4), "predict_seconds": round(t_pred, 4),
                              "iterations": rl.iterations, "status": rl.status, "eta0": float(rl.eta_history[0]),
                              "eta": rl.eta, "eta_verify_fp64": rl.eta_verify_fp64, "refinements": rl.refinements,
                              "C_12_12": float(rl.mean_stress[5]) / 2.0, "prediction_rel_l2": round(err, 4),
                              "fell_back_to_applied_strain": fell_back, "weights": os.path.relpath(weights, ROOT)}
            out["speedup"] = round(t_plain / t_learned, 3)
            net.close()
    return out


def spectrum_bytes(L):
    """Bytes of the three float32 half spectra of an L^3 cell as the solver
    stores them (H = L/2 + 1 planes rounded up to the z blocking of 8)."""
    zs = 3
    while zs > 0 and L % (1 << zs):
        zs -= 1
    hp = ((L // 2 + 1 + (1 << zs) - 1) >> zs) << zs
    return 3 * hp * L * L * 8


def device_inplace(fe, torch, nbytes, reps=5):
    """Bandwidth of the library's streaming kernel rewriting one buffer in
    place (fe_stream_copy with dst == src), the access pattern of the in-place
    transform passes, over ``nbytes`` (the workload's half spectra): read +
    write counted, best of ``reps`` per variant."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    out = {"bytes": nbytes}

    def best_of(nt):
        fe.stream_copy(a, a, nt, st.cuda_stream)
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fe.stream_copy(a, a, nt, st.cuda_stream)
            e1.record(st)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3)
        return 2 * nbytes / best / 1e9

    out["plain_gbs"] = round(best_of(False), 1)
    out["nontemporal_gbs"] = round(best_of(True), 1)
    out["gbs"] = max(out["plain_gbs"], out["nontemporal_gbs"])
    out["kernel"] = "fe_stream_copy in place (dst == src) over the half spectra, best variant, best of 5"
    del a
    torch.cuda.empty_cache()
    return out


def device_copy(fe, torch, nbytes=1 << 31, reps=5):
    """Bandwidth of the library's streaming copy kernel (fe_stream_copy) on
    2 GiB, read + write counted, best of ``reps`` per variant (plain and
    non-temporal), timed with events on the stream it runs on; torch's copy_
    beside it for reference."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    out = {}

    def best_of(fn):
        fn()
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fn()
            e1.record(st)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3)
        return 2 * nbytes / best / 1e9

    out["plain_gbs"] = round(best_of(lambda: fe.stream_copy(b, a, False, st.cuda_stream)), 1)
    out["nontemporal_gbs"] = round(best_of(lambda: fe.stream_copy(b, a, True, st.cuda_stream)), 1)
    out["torch_copy_gbs"] = round(best_of(lambda: b.copy_(a)), 1)
    out["gbs"] = max(out["plain_gbs"], out["nontemporal_gbs"])
    out["kernel"] = "fe_stream_copy of 2 GiB (read + write), best variant, best of 5"
    del a, b
    torch.cuda.empty_cache()
    return out


def fp64_rate(fe, torch, phase, E, nu, L, K, warmup, tti):
    """The same workload with float64 fields (the paper's precision): K timed
    iterations, and the time to eta <= 1e-6 from the plain start."""
    eps = torch.empty((6, L, L, L), dtype=torch.float64, device="cuda")
    with fe.Plan(L, green="R", scheme="AS", precision="fp64", max_iter=max(warmup, 1)) as plan:
        plan.solve(phase, E, nu, MACRO, 1e-300, strain=eps)
    torch.cuda.synchronize()
    with fe.Plan(L, green="R", scheme="AS", precision="fp64", max_iter=K) as plan:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.solve(phase, E, nu, MACRO, 1e-300, strain=eps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    out = {"value": round(L ** 3 * K / wall, 1), "unit": "voxel-iter/s", "ms_per_step": round(wall / K * 1e3, 4),
           "steps": K, "dtype": "f64"}
    if tti:
        with fe.Plan(L, green="R", scheme="AS", precision="fp64", max_iter=2000) as plan:
            plan.solve(phase, E, nu, MACRO, 1e-6, strain=eps, history=1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = plan.solve(phase, E, nu, MACRO, 1e-6, strain=eps, history=1)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        out["time_to_tol_1e-6"] = {"seconds": round(dt, 4), "iterations": r.iterations, "status": r.status,
                                   "eta": r.eta, "C_12_12": float(r.mean_stress[5]) / 2.0}
    del eps
    torch.cuda.empty_cache()
    return out


def cpu_baseline(L_sample: int, iters: int):
    """The FP64 oracle on the host cores: AS with the rotated operator on an
    L_sample^3 sample of the same recipe, `iters` iterations."""
    workers = min(16, os.cpu_count() or 1)
    os.environ["ORACLE_WORKERS"] = str(workers)
    import oracle as O
    from microstructure import boolean_spheres

    phase, _ = boolean_spheres((L_sample,) * 3, RECIPE["radius"], RECIPE["fraction"], RECIPE["seed"])
    O.solve(phase, list(RECIPE["E"]), list(RECIPE["nu"]), MACRO, op="R", scheme="AS", tol=1e-300, max_iter=1)
    t0 = time.perf_counter()
    O.solve(phase, list(RECIPE["E"]), list(RECIPE["nu"]), MACRO, op="R", scheme="AS", tol=1e-300, max_iter=iters)
    dt = time.perf_counter() - t0
    return {
        "value": L_sample ** 3 * iters / dt,
        "unit": "voxel-iter/s",
        "cores": workers,
        "kind": "oracle",
        "sample": f"{L_sample}^3 of the same recipe, {iters} iterations (+1 eta evaluation), FP64 NumPy/SciPy, "
                  f"{dt:.1f} s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tti", action="store_true", help="skip the time-to-tolerance solve")
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 leg")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1412_8398_amd", "weights", "unet_warmstart.npy"),
                    help="trained warm-start network (.npy); the learned leg is skipped if absent")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference kernel for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not "
                                   "supported (one solve per GPU, no inter-GPU exchange)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1412_8398_amd as fe

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    L = args.size
    phase_np, info = make_phase(L)
    phase = torch.from_numpy(phase_np).cuda()
    eps = torch.empty((6, L, L, L), dtype=torch.float32, device="cuda")
    N = L ** 3
    E, nu = list(RECIPE["E"]), list(RECIPE["nu"])

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # warmup
    with fe.Plan(L, green="R", scheme="AS", precision="fp32", max_iter=max(args.warmup, 1), refine=False) as plan:
        plan.solve(phase, E, nu, MACRO, 1e-300, strain=eps)
    torch.cuda.synchronize()

    # timed: exactly K float32 iterations (tol below reach), per-pass HIP-event
    # timing on the plan's stream.  No float64 re-anchoring here: once the
    # float32 iterate stalls it would insert float64 passes that are not
    # iterations; the time-to-tolerance leg below runs with it.
    K = args.steps
    with fe.Plan(L, green="R", scheme="AS", precision="fp32", max_iter=K, timing=True, refine=False) as plan:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = plan.solve(phase, E, nu, MACRO, 1e-300, strain=eps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    wall = t1 - t0
    value = N * K / wall

    pb = pass_bytes(L)
    passes = {}
    for name, nbytes in pb.items():
        launches = res.pass_launches[name]
        if launches:
            avg = res.pass_seconds[name] / launches
            passes[name] = {"avg_ms": avg * 1e3, "launches": launches, "gbs": nbytes / avg / 1e9,
                            "bytes_per_launch": nbytes}
    dom = max(passes, key=lambda n: passes[n]["avg_ms"] * passes[n]["launches"])
    roof = {
        "bound": "hbm",
        "kernel": dom,
        "achieved": round(passes[dom]["gbs"], 1),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(passes[dom]["gbs"] / PEAK_HBM_GBS, 4),
        "traffic": measured_traffic(dom, L),
    }
    # one iteration: the five transform passes and the fused update (the
    # stand-alone divergence runs once per solve)
    step_bytes = sum(v for k, v in pb.items() if k != "pointwise")
    iter_gbs = step_bytes * K / wall / 1e9

    # context for the roofline: the bandwidth a plain copy attains on this GPU
    copy = device_copy(fe, torch)
    # and an in-place rewrite of a buffer the size of the half spectra (the
    # transform passes read and write their buffer in place)
    inplace = device_inplace(fe, torch, spectrum_bytes(L))

    # the paper's precision: the same K iterations with float64 fields
    fp64 = None
    if not args.no_fp64:
        del eps
        torch.cuda.empty_cache()
        fp64 = fp64_rate(fe, torch, phase, E, nu, L, K, args.warmup, not args.no_tti)
        eps = None

    tti = None
    if not args.no_tti:
        tti = time_to_tolerance(fe, torch, np, phase, E, nu, L, args.weights)
        ref = (fp64 or {}).get("time_to_tol_1e-6")
        if ref:  # each float32 result's effective modulus against the float64 solve's
            for leg in ("plain", "learned"):
                if tti.get(leg):
                    tti[leg]["C_12_12_rel_diff_vs_fp64"] = abs(tti[leg]["C_12_12"] - ref["C_12_12"]) / abs(ref["C_12_12"])

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_sample, args.cpu_iters)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "voxel-iter/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(wall / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{L}^3 sphere-Boolean (r={RECIPE['radius']:g}, f={info.volume_fraction:.4f}, "
                        f"{info.n_spheres} spheres, seed {RECIPE['seed']}), E 10/1, nu 0.3, eps_12=1, "
                        "AS + rotated Green operator, f32 fields / f64 reductions",
            "grid": L,
            "scheme": "AS",
            "green": "rotated",
            "parallelism": "single-gpu",
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "time_to_tol_1e-6": tti,
        "iteration_bytes_model": step_bytes,
        "iteration_gbs_model": round(iter_gbs, 1),
        "iteration_hbm_frac_model": round(iter_gbs / PEAK_HBM_GBS, 4),
        "device_copy": dict(copy, dominant_kernel_frac=round(passes[dom]["gbs"] / copy["gbs"], 4),
                            iteration_frac=round(iter_gbs / copy["gbs"], 4)),
        "device_inplace": dict(inplace, iteration_frac=round(iter_gbs / inplace["gbs"], 4)),
        "fp64": fp64,
        "passes": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                   for k, v in passes.items()},
        "library_seconds": round(res.seconds, 4),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
