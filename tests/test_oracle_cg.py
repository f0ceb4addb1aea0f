"""Pins of the oracle's conjugate-gradient solver (``solve_cg``): the discrete
problem of eq. (19) has one solution, so conjugate gradients must end where
the accelerated scheme ends; the laminate's exact solution; a homogeneous
medium is solved by the applied strain; and the properties that make the
iteration conjugate gradients in the C0-weighted inner product (strain energy
decreasing at every step, C0-orthogonal residuals)."""
import numpy as np
import pytest

import oracle as O
from microstructure import laminate

E3, NU3 = [1.0, 10.0, 0.3], [0.3, 0.25, 0.35]
MACRO = [0.1, -0.2, 0.05, 0.3, 0.0, 0.5]


def _cell(shape=(6, 8, 10), seed=5):
    return np.random.default_rng(seed).integers(0, 3, size=shape).astype(np.uint8)


@pytest.mark.parametrize("op", ["MS", "C", "W", "R"])
def test_cg_ends_at_the_accelerated_scheme_solution(op):
    ph = _cell()
    a = O.solve(ph, E3, NU3, MACRO, op=op, scheme="AS", tol=1e-12, max_iter=3000)
    c = O.solve_cg(ph, E3, NU3, MACRO, op=op, tol=1e-12, max_iter=3000)
    assert a.converged and c.converged
    assert np.abs(c.eps - a.eps).max() <= 1e-9 * np.abs(a.eps).max()
    assert np.allclose(c.mean_stress, a.mean_stress, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("op", ["W", "R"])
def test_cg_laminate_exact_solution(op):
    labels = np.array([1] * 3 + [0] * 7, dtype=np.uint8)
    phase = laminate((4, 6, 10), labels)
    E, nu = np.array([1.0, 7.0]), np.array([0.3, 0.2])
    macro = np.array([0.7, -0.3, 0.4, 0.2, -0.5, 0.6])
    r = O.solve_cg(phase, E, nu, macro, op=op, tol=1e-13, max_iter=500)
    assert r.converged
    assert np.allclose(r.eps[:, :, 0, 0, :], O.laminate_exact(labels, E, nu, macro), atol=1e-10)


def test_cg_homogeneous_medium_needs_no_iteration():
    ph = np.zeros((4, 6, 8), dtype=np.uint8)
    r = O.solve_cg(ph, [2.0], [0.3], MACRO, op="R", tol=1e-14)
    assert r.iterations == 0 and r.eta_history[0] < 1e-15


def _B(op, ph, E, nu, ref, x):
    lam, mu = O.lame_from_young(np.asarray(E), np.asarray(nu))
    C = [O.stiffness_tensor(l, m) for l, m in zip(lam, mu)]
    sig = O.apply_phasewise(C, ph, x)
    return np.real(O.inverse_dft(O.green_apply(op, ref, O.forward_dft(sig), ph.shape))), sig


@pytest.mark.parametrize("op", ["W", "R"])
def test_cg_energy_decreases_and_residuals_are_c0_orthogonal(op):
    ph = _cell((6, 6, 8), seed=9)
    lam, mu = O.lame_from_young(np.asarray(E3), np.asarray(NU3))
    ref = O.reference_medium(lam, mu, "AS")
    C0 = O.stiffness_tensor(ref.lam0, ref.mu0)
    r = O.solve_cg(ph, E3, NU3, MACRO, op=op, tol=1e-300, max_iter=8, keep_iterates=True)
    energies, res = [], []
    for eps in r.iterates:
        Bx, sig = _B(op, ph, E3, NU3, ref, eps)
        energies.append(float(np.sum(eps * sig)))
        res.append(-Bx)
    assert all(b < a for a, b in zip(energies, energies[1:])), energies
    dot = lambda a, b: float(np.sum(a * O.contract(C0, b)))  # noqa: E731
    for i in range(len(res)):
        for j in range(i):
            assert abs(dot(res[i], res[j])) <= 1e-9 * np.sqrt(dot(res[i], res[i]) * dot(res[j], res[j]))
