"""Conjugate gradients on the GPU (FE_CONJUGATE_GRADIENT: WP and ROT on the
corner displacement, MS and centered on the six-component strain): the
iterates equal the oracle's conjugate gradients at equal iteration index
(float64: strain to 1e-10 relative L2, eta^k to 1e-9 relative of eta^0 -- a
recursive residual in another summation order carries rounding that the
fixed-point schemes do not), the converged solution equals the accelerated
scheme's, float32 reaches a tolerance with float64 verification, and the
error paths (other operators, a start strain, batched solves)."""
import numpy as np
import pytest

import oracle as O
from microstructure import voronoi_cells

torch = pytest.importorskip("torch")
import paper_1412_8398_amd as fe  # noqa: E402

pytestmark = pytest.mark.gpu

MACRO = [0.7, -0.2, 0.3, 0.15, -0.4, 0.25]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _three_phase(shape, seed=7):
    ph, _, _ = voronoi_cells(shape, 10, 3, seed)
    return ph, [1.0, 5.0, 50.0], [0.2, 0.3, 0.35]


def _cg(phase, E, nu, op, precision, max_iter, tol=1e-300, scheme="CG", refine=True):
    nz, ny, nx = phase.shape
    dt = torch.float64 if precision == "fp64" else torch.float32
    with fe.Plan((nx, ny, nz), green=op, scheme=scheme, precision=precision, max_iter=max_iter,
                 refine=refine) as plan:
        eps = torch.empty((6, nz, ny, nx), dtype=dt, device="cuda")
        res = plan.solve(_dev(phase), E, nu, MACRO, tol, strain=eps, history=max_iter + 1, raise_on_error=False)
        torch.cuda.synchronize()
    return res, eps.cpu().numpy().astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("op", ["W", "R", "MS", "C"])
@pytest.mark.parametrize("shape", [(8, 12, 16), (12, 24, 256)])
def test_cg_iterates_match_the_oracle_fp64(op, shape):
    """Equal iterates at k = 10 on a small cell and on one spanning several
    tiles along x (256 = two 128-wide tiles) with a ragged y (24 = 3 rows of 8)."""
    phase, E, nu = _three_phase(shape, seed=11)
    k = 10
    ref = O.solve_cg(phase, E, nu, MACRO, op=op, tol=1e-300, max_iter=k)
    res, eps = _cg(phase, E, nu, op, "fp64", k)
    print(op, shape, res.status, res.iterations, ref.eta_history[-1], flush=True)
    assert res.iterations == k
    assert _rel(eps, O.tensor_to_voigt(ref.eps)) < 1e-10
    h = np.asarray(res.eta_history[: k + 1])
    assert np.allclose(h, ref.eta_history, rtol=0, atol=1e-9 * ref.eta_history[0])
    assert np.allclose(res.mean_stress, O.tensor_to_voigt(ref.mean_stress), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("op", ["W", "R", "MS", "C"])
def test_cg_converges_with_the_oracle_and_to_the_accelerated_solution(op):
    shape = (16, 16, 16)
    phase, E, nu = _three_phase(shape, seed=3)
    tol = 1e-10
    ref = O.solve_cg(phase, E, nu, MACRO, op=op, tol=tol, max_iter=2000)
    res, eps = _cg(phase, E, nu, op, "fp64", 2000, tol)
    assert res.status == fe.FE_OK and res.iterations == ref.iterations
    asr, eps_as = _cg(phase, E, nu, op, "fp64", 2000, 1e-12, scheme="AS")
    assert asr.status == fe.FE_OK
    assert _rel(eps, eps_as) < 1e-8
    assert np.allclose(res.mean_stress, asr.mean_stress, rtol=1e-8, atol=1e-10)


def test_cg_fp32_reaches_tolerance_with_fp64_verification():
    """Float32 conjugate gradients without refinement reach 1e-5 (float64
    verification agrees) and stop at the float32 floor of this contrast-50
    cell (about 2.5e-6) with FE_NOT_CONVERGED; with float64 refinement (the
    default) they reach 1e-6 and 1e-7, the returned float32 strain verifying
    to tol, and report FE_NOT_CONVERGED below what a float32 strain can hold."""
    shape = (32, 32, 32)
    phase, E, nu = _three_phase(shape, seed=5)
    ref, _ = _cg(phase, E, nu, "R", "fp64", 2000, 1e-10)
    res, eps = _cg(phase, E, nu, "R", "fp32", 2000, 1e-5, refine=False)
    assert res.status == fe.FE_OK and res.eta_verify_fp64 <= 1.2e-5
    assert np.allclose(res.mean_stress, ref.mean_stress, rtol=1e-4, atol=1e-5)
    low, _ = _cg(phase, E, nu, "R", "fp32", 2000, 1e-8, refine=False)
    assert low.status == fe.FE_NOT_CONVERGED and 1e-8 < low.eta_verify_fp64 < 1e-5
    assert abs(low.eta - low.eta_verify_fp64) <= 0.05 * low.eta_verify_fp64
    for tol in (1e-6, 1e-7):
        rr, _ = _cg(phase, E, nu, "R", "fp32", 2000, tol)
        print(tol, rr, flush=True)
        assert rr.status == fe.FE_OK and rr.eta <= tol and rr.eta_verify_fp64 <= tol
        assert np.allclose(rr.mean_stress, ref.mean_stress, rtol=1e-6, atol=1e-7)
    tiny, _ = _cg(phase, E, nu, "R", "fp32", 2000, 1e-11)
    assert tiny.status == fe.FE_NOT_CONVERGED and tiny.eta_verify_fp64 > 1e-11


def test_cg_six_component_fp32():
    """Float32 conjugate gradients in the six-component form (no refinement)
    reach 1e-5 with the float64 verification agreeing, and the float64
    solution's mean stress."""
    phase, E, nu = _three_phase((32, 32, 32), seed=5)
    ref, _ = _cg(phase, E, nu, "MS", "fp64", 2000, 1e-10)
    res, _ = _cg(phase, E, nu, "MS", "fp32", 2000, 1e-5)
    assert res.status == fe.FE_OK and res.eta_verify_fp64 <= 1.2e-5
    assert np.allclose(res.mean_stress, ref.mean_stress, rtol=1e-4, atol=1e-5)


def test_cg_error_paths():
    phase, E, nu = _three_phase((8, 8, 8))
    with pytest.raises(fe.FeError) as ei:
        fe.Plan(8, green="MSS", scheme="CG", precision="fp64")
    assert ei.value.status == fe.FE_ERR_UNSUPPORTED
    with fe.Plan(8, green="R", scheme="CG", precision="fp64") as plan:
        init = torch.zeros((6, 8, 8, 8), dtype=torch.float64, device="cuda")
        with pytest.raises(fe.FeError) as ei:
            plan.solve(_dev(phase), E, nu, MACRO, 1e-8, strain_init=init)
        assert ei.value.status == fe.FE_ERR_UNSUPPORTED
    with pytest.raises(fe.FeError) as ei:
        fe.solve_batched([fe.BatchSampleSpec(_dev(phase), E, nu, MACRO)], 1e-6, green="R", scheme="CG")
    assert ei.value.status == fe.FE_ERR_UNSUPPORTED


def test_cg_iteration_count_does_not_depend_on_the_reference_scale():
    """Scaling C0 scales the preconditioner and the inner product together:
    the conjugate-gradient iterates, hence N(E0) at fixed nu0, do not depend
    on E0 (unlike the fixed-point schemes of §6.1); the count equals the
    oracle's.  Porous Boolean medium, contrast 1e-3, tol 1e-8, float64."""
    from microstructure import boolean_spheres

    phase, _ = boolean_spheres((16, 16, 16), 2.5, 0.17, 1412)
    E, nu = [1.5, 1.5e-3], [0.25, 0.25]
    macro = [0.0, 0.0, 0.0, 0.0, 0.0, 1.0]
    counts = []
    for E0 in (0.05, 0.5, 5.0):
        with fe.Plan(16, green="R", scheme="CG", precision="fp64", max_iter=3000, ref_rule="explicit", E0=E0,
                     nu0=0.25) as plan:
            r = plan.solve(_dev(phase), E, nu, macro, 1e-8, raise_on_error=False)
        assert r.status == fe.FE_OK
        counts.append(r.iterations)
    ref = O.solve_cg(phase, E, nu, macro, op="R", tol=1e-8, max_iter=3000,
                     ref=O.reference_medium(None, None, "AS", E0=0.5, nu0=0.25))
    print(counts, ref.iterations, flush=True)
    assert counts[0] == counts[1] == counts[2] == ref.iterations


def test_cg_one_plane_cell_and_effective_stiffness():
    """A one-plane (2D, plane strain) cell: float64 iterates equal to the
    oracle's; the effective stiffness from six conjugate-gradient solves
    equals the accelerated scheme's."""
    shape = (1, 32, 48)
    phase, E, nu = _three_phase(shape, seed=21)
    k = 12
    ref = O.solve_cg(phase, E, nu, MACRO, op="R", tol=1e-300, max_iter=k)
    res, eps = _cg(phase, E, nu, "R", "fp64", k)
    assert res.iterations == k and _rel(eps, O.tensor_to_voigt(ref.eps)) < 1e-10
    ph3, E3, nu3 = _three_phase((12, 16, 8), seed=4)
    C = {}
    for scheme in ("CG", "AS"):
        with fe.Plan((8, 16, 12), green="W", scheme=scheme, precision="fp64", max_iter=3000) as plan:
            C[scheme], its, st = plan.effective_stiffness(_dev(ph3), E3, nu3, 1e-11)
        assert st == fe.FE_OK
    assert np.allclose(C["CG"], C["AS"], rtol=1e-8, atol=1e-9)
