"""Mixed-precision refinement: float32 fields with float64 re-anchoring reach
tolerances below the float32 floor and the float64 solution.

Tolerance: at eta <= 1e-7 the float32-stored strain agrees with the float64
solution to relative L2 <= 1e-5 (the remaining equilibrium error times the
conditioning of a contrast-10 medium; float32 storage rounding alone leaves
eta ~ 3e-8 on this sample, so tolerances below that are out of reach and
end as FE_NOT_CONVERGED)."""
import numpy as np
import pytest

from microstructure import boolean_spheres

torch = pytest.importorskip("torch")
import paper_1412_8398_amd as fe  # noqa: E402

pytestmark = pytest.mark.gpu


def _case(L=48):
    phase, _ = boolean_spheres((L, L, L), 4.0, 0.25, 99)
    return phase, [1.0, 10.0], [0.3, 0.3], [0.2, -0.1, 0.3, 0.0, 0.4, 1.0]


def _solve(phase, E, nu, macro, op, scheme, precision, tol, max_iter, refine=True):
    L = phase.shape[0]
    dt = torch.float64 if precision == "fp64" else torch.float32
    with fe.Plan(L, green=op, scheme=scheme, precision=precision, max_iter=max_iter, refine=refine) as plan:
        eps = torch.empty((6, L, L, L), dtype=dt, device="cuda")
        r = plan.solve(torch.from_numpy(phase).cuda(), E, nu, macro, tol, strain=eps, raise_on_error=False)
        torch.cuda.synchronize()
    return r, eps.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("op,scheme", [("R", "AS"), ("R", "DS"), ("W", "AS"), ("MS", "AS"), ("MS", "DS"), ("C", "AS"),
                                       ("MSS", "AS")])
def test_refinement_reaches_the_float64_solution(op, scheme):
    """Displacement form (R, W): float64 displacement and divergences at each
    anchor; six-component form (MS, C): the anchor's iterate, strain residual
    and divergence spectrum in float64, the float32 iterations on the
    correction."""
    phase, E, nu, macro = _case()
    # the float32 storage floor of the returned strain is higher for the
    # continuous and centered operators (their eta weighs the rounding noise
    # of the stored strain with |k| up to pi sqrt(3) at the Nyquist corner,
    # twice the rotated operator's): 1.05e-7 measured for MS-DS on this cell
    tol = 1e-7 if op in ("R", "W") else 3e-7
    r64, e64 = _solve(phase, E, nu, macro, op, scheme, "fp64", 1e-11, 3000)
    assert r64.status == fe.FE_OK
    r32, e32 = _solve(phase, E, nu, macro, op, scheme, "fp32", tol, 3000)
    assert r32.status == fe.FE_OK, (r32.status, r32.eta, r32.eta_verify_fp64)
    assert r32.refinements >= 1
    assert r32.eta_verify_fp64 <= 1.2 * tol
    assert np.linalg.norm(e32 - e64) / np.linalg.norm(e64) < 1e-5
    assert np.allclose(r32.mean_stress, r64.mean_stress, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("op", ["R", "MS"])
def test_plain_float32_stalls_above_the_refined_tolerance(op):
    phase, E, nu, macro = _case()
    r, _ = _solve(phase, E, nu, macro, op, "AS", "fp32", 1e-7, 400, refine=False)
    assert r.status == fe.FE_NOT_CONVERGED
    assert r.refinements == 0
    assert r.eta_verify_fp64 > 1e-7


def test_tolerance_below_the_float32_storage_floor_stops_early():
    phase, E, nu, macro = _case()
    r, _ = _solve(phase, E, nu, macro, "R", "AS", "fp32", 1e-12, 3000)
    assert r.status == fe.FE_NOT_CONVERGED
    assert r.iterations < 3000
    assert r.eta_verify_fp64 < 1e-6


def test_refinement_costs_at_most_two_iterations_over_float64():
    """The float32 floor is caught as it shows (the eta ratio rising), so the
    refined float32 solve to 1e-6 on a 256^3 cell of the benchmark recipe
    (spheres of radius 6, fraction 0.25, contrast 10, shear) needs at most two
    iterations more than float64, with one or two re-anchors, and no re-anchor
    at a tolerance above the floor."""
    import bench

    phase, _ = bench.make_phase(256)
    E, nu, macro = list(bench.RECIPE["E"]), list(bench.RECIPE["nu"]), list(bench.MACRO)
    r64, _ = _solve(phase, E, nu, macro, "R", "AS", "fp64", 1e-6, 500)
    r32, _ = _solve(phase, E, nu, macro, "R", "AS", "fp32", 1e-6, 500)
    print(r64.iterations, r32.iterations, r32.refinements, r32.eta_verify_fp64, flush=True)
    assert r64.status == fe.FE_OK and r32.status == fe.FE_OK and r32.eta_verify_fp64 <= 1e-6
    assert r32.iterations <= r64.iterations + 2 and 1 <= r32.refinements <= 2
    coarse, _ = _solve(phase, E, nu, macro, "R", "AS", "fp32", 1e-4, 500)
    assert coarse.status == fe.FE_OK and coarse.refinements == 0
