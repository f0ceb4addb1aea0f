"""Full-size checks in the configuration bench.py times (AS, rotated operator,
float32 fields, float64 reductions and re-anchoring) at 512^3 and 1024^3:
closed forms compared voxel by voxel on sampled outputs, and properties that
hold at any size.

Tolerances: a float32 field stored after the iteration reached eta <= tol has
a relative error of about tol times the contrast plus the float32 storage
rounding (6e-8); 1e-5 of the largest strain component covers both for the
tolerances used here (1e-7, contrast <= 10).
"""
import numpy as np
import pytest

import oracle as O
from microstructure import laminate

torch = pytest.importorskip("torch")
import paper_1412_8398_amd as fe  # noqa: E402

pytestmark = pytest.mark.gpu

MACRO = [0.7, -0.3, 0.4, 0.2, -0.5, 0.6]


def _layers(L, seed):
    r = np.random.default_rng(seed)
    cuts = np.sort(r.choice(np.arange(1, L), size=6, replace=False))
    widths = np.diff(np.concatenate([[0], cuts, [L]]))
    return np.concatenate([np.full(w, i % 3, dtype=np.uint8) for i, w in enumerate(widths)])


@pytest.mark.parametrize("L", [512, 1024])
def test_laminate_matches_the_closed_form_at_full_size(L):
    print(f"laminate L={L}", flush=True)
    labels = _layers(L, L)
    E, nu = [1.0, 10.0, 3.0], [0.3, 0.2, 0.35]
    phase = torch.from_numpy(laminate((L, L, L), labels)).cuda()
    eps = torch.empty((6, L, L, L), dtype=torch.float32, device="cuda")
    with fe.Plan(L, green="R", scheme="AS", precision="fp32", max_iter=500) as plan:
        r = plan.solve(phase, E, nu, MACRO, 1e-7, strain=eps)
    torch.cuda.synchronize()
    assert r.status == fe.FE_OK and r.eta_verify_fp64 <= 1.2e-7
    exact = O.tensor_to_voigt(O.laminate_exact(labels, E, nu, MACRO))  # (6, L)
    rng = np.random.default_rng(3)
    n = 8192
    z, y, x = (rng.integers(0, L, n) for _ in range(3))
    got = eps[:, torch.from_numpy(z).cuda(), torch.from_numpy(y).cuda(), torch.from_numpy(x).cuda()]
    got = got.double().cpu().numpy()
    scale = np.abs(exact).max()
    assert np.max(np.abs(got - exact[:, x])) <= 1e-5 * scale
    # every voxel: the field depends on x only
    dev = (eps - eps[:, :1, :1, :]).abs().max().item()
    assert dev <= 1e-5 * scale
    del eps, phase
    torch.cuda.empty_cache()


def _corner_div_rms(sig):
    """RMS over the interior corners of a window of the rotated-grid divergence
    of sigma (eq. (38)): div_j(c) = 1/4 sum_{a in {0,1}^3} sum_i (2 a_i - 1)
    sigma_ij(c - a); sig is (3, 3, nz, ny, nx) float64."""
    nz, ny, nx = sig.shape[2:]
    d = np.zeros((3, nz - 1, ny - 1, nx - 1))
    for az in (0, 1):
        for ay in (0, 1):
            for ax in (0, 1):
                a = (ax, ay, az)
                w = sig[:, :, 1 - az:nz - az, 1 - ay:ny - ay, 1 - ax:nx - ax]
                for i in range(3):
                    d += 0.25 * (2 * a[i] - 1) * w[i]
    return float(np.sqrt(np.mean(np.sum(d * d, axis=0))))


def test_bench_workload_properties():
    """The 512^3 benchmark cell: converged in float64 verification, mean strain
    eps_bar, effective shear modulus between the Reuss and Voigt bounds, the
    direct scheme reaching the same mean stress, and a local equilibrium check
    of the returned field consistent with the reported eta."""
    import bench

    L = 512
    print("bench workload 512^3", flush=True)
    phase_np, _ = bench.make_phase(L)
    phase = torch.from_numpy(phase_np).cuda()
    E, nu = list(bench.RECIPE["E"]), list(bench.RECIPE["nu"])
    macro = list(bench.MACRO)
    eps = torch.empty((6, L, L, L), dtype=torch.float32, device="cuda")
    with fe.Plan(L, green="R", scheme="AS", precision="fp32", max_iter=2000) as plan:
        ra = plan.solve(phase, E, nu, macro, 1e-6, strain=eps)
    torch.cuda.synchronize()
    assert ra.status == fe.FE_OK and ra.eta_verify_fp64 <= 1.2e-6
    mean = eps.double().mean(dim=(1, 2, 3)).cpu().numpy()
    assert np.allclose(mean, macro, atol=1e-6)
    f = float(phase_np.mean())
    lam, mu = O.lame_from_young(E, nu)
    mu_eff = ra.mean_stress[5] / 2.0  # eps_12 = 1: <sigma_12> = 2 mu_eff
    assert 1.0 / ((1 - f) / mu[0] + f / mu[1]) <= mu_eff <= (1 - f) * mu[0] + f * mu[1]
    # local equilibrium on a 40^3 window
    w = eps[:, 100:140, 200:240, 300:340].double().cpu().numpy()
    ph = phase_np[100:140, 200:240, 300:340]
    e3 = O.voigt_to_tensor(w)
    tr = e3[0, 0] + e3[1, 1] + e3[2, 2]
    sig = 2 * mu[ph] * e3 + lam[ph] * tr * np.eye(3)[:, :, None, None, None]
    s_norm = np.linalg.norm(O.voigt_to_tensor(np.asarray(ra.mean_stress)))
    assert _corner_div_rms(sig) <= 5.0 * ra.eta_verify_fp64 * s_norm
    with fe.Plan(L, green="R", scheme="DS", precision="fp32", max_iter=3000) as plan:
        rd = plan.solve(phase, E, nu, macro, 1e-6)
    assert rd.status == fe.FE_OK
    assert np.allclose(rd.mean_stress, ra.mean_stress, rtol=1e-4, atol=1e-6)
    del eps, phase
    torch.cuda.empty_cache()
