"""Batched solves of uneven samples (fe_solve_batched).

Each sample of a batch must follow exactly the iteration a single-sample
fe_solve of the same plan options performs (same kernels, same constants,
same fixed-order reductions), with either float32 launch (one per pass, or
one cooperative persistent launch): iteration counts, eta and the strain
field are compared bit for bit against single solves with refinement off.  One float64
sample is also compared with the oracle at its converged iteration count
(relative L2 <= 1e-12, the single-solve float64 bar).
"""
import numpy as np
import pytest

import oracle as O
from microstructure import boolean_spheres, laminate, sphere_inclusion

torch = pytest.importorskip("torch")
import paper_1412_8398_amd as fe  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _samples():
    """Four samples over three grid classes, two contrasts, two phase counts."""
    a, _ = boolean_spheres((32, 32, 32), 3.0, 0.2, 11)
    b, _ = boolean_spheres((24, 32, 48), 3.0, 0.3, 12)  # (nz, ny, nx)
    c, _ = boolean_spheres((32, 32, 32), 4.0, 0.15, 13)
    d = laminate((16, 16, 16), [0] * 4 + [1] * 8 + [2] * 4)  # three layers along x
    d[sphere_inclusion((16, 16, 16), (8, 8, 8), 3.0) == 1] = 3   # and a fourth phase
    n_d = 4
    specs = [
        (a, [1.0, 10.0], [0.3, 0.3], [0, 0, 0, 0, 0, 1.0]),
        (b, [1.0, 10.0], [0.3, 0.25], [0.5, -0.2, 0.1, 0.0, 0.3, 0.0]),
        (c, [1.0, 100.0], [0.2, 0.35], [1.0, 0, 0, 0, 0, 0]),
        (d, list(np.linspace(1.0, 20.0, n_d)), [0.3] * n_d, [0.2, 0.2, -0.1, 0.4, 0.0, 0.1]),
    ]
    return specs


def _single(phase, E, nu, macro, op, scheme, precision, tol, max_iter):
    nz, ny, nx = phase.shape
    dt = torch.float64 if precision == "fp64" else torch.float32
    with fe.Plan((nx, ny, nz), green=op, scheme=scheme, precision=precision, max_iter=max_iter,
                 refine=False) as plan:
        eps = torch.empty((6, nz, ny, nx), dtype=dt, device="cuda")
        r = plan.solve(_dev(phase), E, nu, macro, tol, strain=eps, raise_on_error=False)
        torch.cuda.synchronize()
    return r, eps.cpu().numpy()


def _batched(specs, op, scheme, precision, tol, max_iter, launch="per_pass"):
    dt = torch.float64 if precision == "fp64" else torch.float32
    samples, outs = [], []
    for ph, E, nu, macro in specs:
        nz, ny, nx = ph.shape
        eps = torch.empty((6, nz, ny, nx), dtype=dt, device="cuda")
        outs.append(eps)
        samples.append(fe.BatchSampleSpec(_dev(ph), E, nu, macro, eps))
    res, status, sec = fe.solve_batched(samples, tol, green=op, scheme=scheme, precision=precision,
                                        max_iter=max_iter, launch=launch)
    torch.cuda.synchronize()
    return res, status, sec, [e.cpu().numpy() for e in outs]


@pytest.mark.parametrize("op,scheme,precision,tol,launch", [
    ("R", "AS", "fp32", 1e-5, "per_pass"),
    ("R", "AS", "fp32", 1e-5, "persistent"),
    ("W", "DS", "fp32", 1e-3, "per_pass"),  # float32 DS at contrast 100 stalls near 1.4e-4 (float32 tau)
    ("W", "DS", "fp32", 1e-3, "persistent"),
    ("R", "DS", "fp64", 1e-8, "per_pass"),
    ("W", "AS", "fp64", 1e-9, "per_pass"),
])
def test_batched_samples_match_single_solves_bitwise(op, scheme, precision, tol, launch):
    """Both float32 launches (one per pass, one persistent) and float64."""
    specs = _samples()
    res, status, sec, eps = _batched(specs, op, scheme, precision, tol, 3000, launch)
    assert status == fe.FE_OK, [(r.status, r.iterations, r.eta) for r in res]
    assert sec > 0
    its = []
    for (ph, E, nu, macro), rb, eb in zip(specs, res, eps):
        rs, es = _single(ph, E, nu, macro, op, scheme, precision, tol, 3000)
        assert rs.status == fe.FE_OK and rb.status == fe.FE_OK
        assert rb.iterations == rs.iterations
        assert rb.eta == rs.eta
        assert rb.eta <= tol
        assert np.array_equal(eb, es)
        assert np.array_equal(rb.mean_stress, rs.mean_stress)
        assert np.isclose(rb.eta_verify_fp64, rs.eta_verify_fp64, rtol=1e-12, atol=0)
        its.append(rb.iterations)
    assert len(set(its)) > 1  # uneven: samples retire at different iterations


def test_batched_float64_sample_matches_the_oracle():
    specs = _samples()
    res, status, _, eps = _batched(specs, "R", "AS", "fp64", 1e-8, 3000)
    assert status == fe.FE_OK
    ph, E, nu, macro = specs[1]
    k = res[1].iterations
    ref = O.solve(ph, E, nu, macro, op="R", scheme="AS", tol=1e-300, max_iter=k)
    assert ref.iterations == k
    rel = np.linalg.norm(eps[1] - O.tensor_to_voigt(ref.eps)) / np.linalg.norm(O.tensor_to_voigt(ref.eps))
    assert rel < 1e-12
    assert np.isclose(res[1].eta, ref.eta_history[k], rtol=1e-10, atol=1e-14)


def test_iteration_cap_retires_only_the_capped_samples():
    """The high-contrast sample needs many more direct-scheme iterations; with
    a cap between the counts it alone ends FE_NOT_CONVERGED at the cap."""
    specs = _samples()
    free, _, _, _ = _batched(specs, "R", "DS", "fp64", 1e-6, 5000)
    its = sorted(r.iterations for r in free)
    cap = (its[-2] + its[-1]) // 2
    assert its[-2] < cap < its[-1]
    res, status, _, eps = _batched(specs, "R", "DS", "fp64", 1e-6, cap)
    assert status == fe.FE_NOT_CONVERGED
    for rf, rc, (ph, E, nu, macro), ec in zip(free, res, specs, eps):
        if rf.iterations <= cap:
            assert rc.status == fe.FE_OK and rc.iterations == rf.iterations
        else:
            assert rc.status == fe.FE_NOT_CONVERGED and rc.iterations == cap
            rs, es = _single(ph, E, nu, macro, "R", "DS", "fp64", 1e-6, cap)
            assert rs.status == fe.FE_NOT_CONVERGED and rs.iterations == cap
            assert np.array_equal(ec, es)


def test_batched_rejects_bad_labels():
    specs = _samples()
    ph, E, nu, macro = specs[0]
    bad = ph.copy()
    bad[3, 4, 5] = 2  # two phases declared
    samples = [fe.BatchSampleSpec(_dev(bad), E, nu, macro)]
    _, status, _ = fe.solve_batched(samples, 1e-6, raise_on_error=False)
    assert status == fe.FE_ERR_INVALID_ARG
    assert "label" in fe.last_error()


def test_batch_outside_the_persistent_lengths_matches_single_solves():
    """A persistent batch with a grid length the persistent kernel is not
    built for (8) runs one launch per pass; samples still equal single solves
    bit for bit."""
    a, _ = boolean_spheres((8, 16, 16), 2.0, 0.2, 21)
    b, _ = boolean_spheres((16, 16, 16), 3.0, 0.25, 22)
    specs = [(a, [1.0, 10.0], [0.3, 0.3], [0, 0, 0, 0, 0, 1.0]), (b, [1.0, 5.0], [0.3, 0.3], [1.0, 0, 0, 0, 0, 0])]
    res, status, _, eps = _batched(specs, "R", "AS", "fp32", 1e-5, 2000, "persistent")
    assert status == fe.FE_OK
    for (ph, E, nu, macro), rb, eb in zip(specs, res, eps):
        rs, es = _single(ph, E, nu, macro, "R", "AS", "fp32", 1e-5, 2000)
        assert rb.iterations == rs.iterations and rb.eta == rs.eta and np.array_equal(eb, es)


@pytest.mark.parametrize("launch", ["per_pass", "persistent"])
def test_float64_continuation_reaches_the_tolerance(launch):
    """High-contrast samples whose float32 iteration stalls above 1e-6 (the
    float32 floor) continue in float64 from their float32 iterate: every
    returned strain verifies to 1e-6 in float64, and without the
    continuation some do not."""
    from microstructure import batch_samples

    samples = [s for s in batch_samples(24, 7001, sizes=(32, 48))]
    specs = [(s.phase, [1.0, s.contrast], [s.nu, s.nu], s.macro_strain) for s in samples]
    plain, _, _, _ = _batched_opts(specs, "R", "AS", 1e-6, 2000, refine=False, launch=launch)
    res, status, _, eps = _batched_opts(specs, "R", "AS", 1e-6, 2000, refine=True, launch=launch)
    assert status == fe.FE_OK, [(r.status, r.iterations, r.eta_verify_fp64) for r in res]
    assert all(r.eta_verify_fp64 <= 1e-6 for r in res)
    assert any(r.eta_verify_fp64 > 1e-6 for r in plain)
    for rp, rr, e in zip(plain, res, eps):
        assert rr.iterations >= rp.iterations and np.isfinite(e).all()


def _batched_opts(specs, op, scheme, tol, max_iter, refine, launch="per_pass"):
    samples, outs = [], []
    for ph, E, nu, macro in specs:
        nz, ny, nx = ph.shape
        eps = torch.empty((6, nz, ny, nx), dtype=torch.float32, device="cuda")
        outs.append(eps)
        samples.append(fe.BatchSampleSpec(_dev(ph), E, nu, macro, eps))
    res, status, sec = fe.solve_batched(samples, tol, green=op, scheme=scheme, precision="fp32", max_iter=max_iter,
                                        refine=refine, raise_on_error=False, launch=launch)
    torch.cuda.synchronize()
    return res, status, sec, [e.cpu().numpy() for e in outs]


def test_persistent_launch_with_more_grid_classes_than_it_holds_falls_back():
    """Nine distinct grids (the persistent kernel holds eight classes): the
    batch runs one launch per pass, and still equals single solves."""
    shapes = [(16, 16, 16), (16, 16, 24), (16, 24, 16), (24, 16, 16), (16, 16, 32), (16, 32, 16), (32, 16, 16),
              (24, 24, 16), (16, 24, 24)]
    specs = []
    for i, shp in enumerate(shapes):
        ph, _ = boolean_spheres(shp, 2.5, 0.2, 40 + i)
        specs.append((ph, [1.0, 8.0], [0.3, 0.3], [0, 0, 0, 0, 0, 1.0]))
    res, status, _, eps = _batched(specs, "R", "AS", "fp32", 1e-4, 500, "persistent")
    assert status == fe.FE_OK
    for (ph, E, nu, macro), rb, eb in zip(specs, res, eps):
        rs, es = _single(ph, E, nu, macro, "R", "AS", "fp32", 1e-4, 500)
        assert rb.iterations == rs.iterations and rb.eta == rs.eta and np.array_equal(eb, es)


@pytest.mark.parametrize("max_iter", [0, 3])
def test_both_launches_agree_at_a_small_iteration_cap(max_iter):
    """At caps of 0 and 3 iterations every sample ends FE_NOT_CONVERGED at the
    cap, with the same iterate and eta from either launch."""
    specs = _samples()
    a, sa, _, ea = _batched(specs, "R", "AS", "fp32", 1e-12, max_iter, "per_pass")
    b, sb, _, eb = _batched(specs, "R", "AS", "fp32", 1e-12, max_iter, "persistent")
    assert sa == sb == fe.FE_NOT_CONVERGED
    for ra, rb, xa, xb in zip(a, b, ea, eb):
        assert ra.status == rb.status == fe.FE_NOT_CONVERGED
        assert ra.iterations == rb.iterations == max_iter
        assert ra.eta == rb.eta and np.array_equal(xa, xb)
