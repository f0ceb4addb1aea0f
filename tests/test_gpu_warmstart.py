"""The trained warm-start network (paper_1412_8398_amd/weights) on held-out
cells of its training distribution: its prediction is closer to the
converged strain than the plain start eps^0 = eps_bar (relative L2 1 by
definition), the solve from it reaches the same equilibrium, and it saves
iterations, no more than the contraction model allows: a start whose error
is e times that of eps_bar saves at most about log(e) / log(rho) iterations
(rho: the plain run's contraction per iteration).  Measured on 16 cells at
512^3: 0.94 iterations saved per cell against a prediction that costs 5.4."""
import os

import numpy as np
import pytest

from microstructure import batch_samples

torch = pytest.importorskip("torch")
import paper_1412_8398_amd as fe  # noqa: E402
from paper_1412_8398_amd.warmstart import DEFAULT_WEIGHTS, compare_one, load_net, scaled_starts  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.skipif(not os.path.exists(DEFAULT_WEIGHTS), reason="no trained weights in the tree")
def test_learned_start_is_closer_and_converges_to_the_same_answer():
    net = load_net()
    samples = batch_samples(6, 777, sizes=(64,))  # seed outside the training and validation sets
    rows = []
    with fe.Plan(64, green="R", scheme="AS", precision="fp32", max_iter=3000) as plan:
        for s in samples:
            ph = torch.from_numpy(s.phase).cuda()
            r = compare_one(net, ph, [1.0, s.contrast], [s.nu, s.nu], s.macro_strain, 1e-6, plan=plan)
            rows.append(r)
            print(s.contrast, s.volume_fraction, r["plain"]["iterations"], r["learned"]["iterations"],
                  r["prediction_rel_l2"], flush=True)
    net.close()
    for r in rows:
        assert r["plain"]["status"] == fe.FE_OK and r["learned"]["status"] == fe.FE_OK
        assert r["mean_stress_rel_diff"] <= 1e-5
    err = np.array([r["prediction_rel_l2"] for r in rows])
    assert np.median(err) < 0.6, err
    it_p = sum(r["plain"]["iterations"] for r in rows)
    it_l = sum(r["learned"]["iterations"] for r in rows)
    assert it_l < it_p, (it_p, it_l)  # the gain: fewer iterations in total
    saved = sum(r["iterations_saved"] for r in rows)
    bound = sum(max(r["iterations_saved_model"], 0.0) + 1.0 for r in rows)
    assert saved <= bound, (saved, bound)


def test_a_start_that_cannot_converge_falls_back_to_the_applied_strain():
    """A prediction the scheme cannot bring to equilibrium (here: not finite)
    ends FE_DIVERGED; the warm-start solve then restarts from eps_bar and
    returns the plain solution."""
    from paper_1412_8398_amd.warmstart import solve_from_prediction

    class _NaNNet:  # stands in for the network: predicts a non-finite strain
        def predict(self, phase, E, nu, macro, out):
            out.fill_(float("nan"))
            return out, 0.0

    s = batch_samples(1, 778, sizes=(32,))[0]
    ph = torch.from_numpy(s.phase).cuda()
    E, nu = [1.0, s.contrast], [s.nu, s.nu]
    with fe.Plan(32, green="R", scheme="AS", precision="fp32", max_iter=3000) as plan:
        plain = plan.solve(ph, E, nu, s.macro_strain, 1e-6, history=1, raise_on_error=False)
        pred = torch.empty((1, 6, 32, 32, 32), dtype=torch.float32, device="cuda")
        eps = torch.empty((6, 32, 32, 32), dtype=torch.float32, device="cuda")
        r, _, fell_back = solve_from_prediction(plan, _NaNNet(), ph, E, nu, s.macro_strain, 1e-6, eps, pred)
    assert fell_back
    assert r.status == fe.FE_OK == plain.status and r.iterations == plain.iterations
    assert np.array_equal(np.asarray(r.mean_stress), np.asarray(plain.mean_stress))


def test_starts_between_the_applied_strain_and_the_solution():
    """The starts that bound what a better prediction could save: the
    network's error scaled by 0 is the converged strain itself, from which the
    solve stops at once (at most one iteration: its float32 eta^0 may sit at
    the tolerance the float64 check met); from eps_bar plus 90% of the exact
    fluctuation it needs fewer iterations than from eps_bar, and from eps_bar
    plus half of it no fewer than from 90%."""
    s = batch_samples(1, 4242, sizes=(48,))[0]
    ph = torch.from_numpy(s.phase).cuda()
    E, nu = [1.0, 50.0], [s.nu, s.nu]
    with fe.Plan(48, green="R", scheme="AS", precision="fp32", max_iter=3000) as plan:
        eps = torch.empty((6, 48, 48, 48), dtype=torch.float32, device="cuda")
        plain = plan.solve(ph, E, nu, s.macro_strain, 1e-6, strain=eps, raise_on_error=False)
        assert plain.status == fe.FE_OK
        pred = eps + 0.01 * torch.randn_like(eps)  # a stand-in prediction near the solution
        its = scaled_starts(plan, ph, E, nu, s.macro_strain, 1e-6, eps, pred, scales=(0.0,), shares=(0.5, 0.1))
    print(plain.iterations, its, flush=True)
    assert its["pred_x0"] <= 1
    assert its["fluct_e0.1"] < plain.iterations
    assert its["fluct_e0.1"] <= its["fluct_e0.5"] <= plain.iterations
