"""Pins of the oracle's iterative solve against closed forms, a direct
finite-difference solve, invariants and the paper's printed values (no GPU)."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as O
from microstructure import laminate, sphere_inclusion, sphere_array

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_sym(rng, shape):
    e = rng.standard_normal((3, 3) + shape)
    return 0.5 * (e + e.transpose(1, 0, 2, 3, 4))


# --- homogeneous medium: one step to the applied strain ----------------------------

@pytest.mark.parametrize("scheme", ["DS", "AS"])
@pytest.mark.parametrize("op", ["MS", "W", "R"])
def test_homogeneous_medium_one_step(op, scheme, rng):
    """C(x) = C0 gives tau = 0, so e^0 = eps_bar and both eq. (9) and eq. (16)
    return exactly eps_bar after one iteration from any start."""
    shape = (6, 8, 4)
    phase = (rng.random(shape) < 0.5).astype(np.uint8)
    E, nu = [2.0, 2.0], [0.3, 0.3]
    macro = np.array([0.3, -0.2, 0.1, 0.05, -0.4, 0.25])
    start = _rand_sym(rng, shape)
    r = O.solve(phase, E, nu, macro, op=op, scheme=scheme, tol=1e-300, max_iter=1,
                eps_init=start)
    assert r.iterations == 1
    assert np.allclose(r.eps, O.voigt_to_tensor(macro)[:, :, None, None, None], atol=1e-14)
    # and from eps_bar: converged at k = 0
    r0 = O.solve(phase, E, nu, macro, op=op, scheme=scheme, tol=1e-12)
    assert r0.iterations == 0


# --- laminates: exact piecewise-constant solution -------------------------------------

def _laminate_exact(phase_x, E, nu, macro):
    return O.laminate_exact(phase_x, E, nu, macro)


def test_laminate_closed_form_balances_tractions_and_strains():
    """sigma_11, sigma_12, sigma_13 equal in every layer and the mean strain is
    eps_bar: the two conditions that define the laminate solution."""
    labels = np.array([0, 0, 1, 2, 2, 2, 1], dtype=np.uint8)
    E, nu = np.array([1.0, 7.0, 3.0]), np.array([0.3, 0.2, 0.45])
    macro = np.array([0.7, -0.3, 0.4, 0.2, -0.5, 0.6])
    eps = O.laminate_exact(labels, E, nu, macro)
    lam, mu = O.lame_from_young(E, nu)
    tr = eps[0, 0] + eps[1, 1] + eps[2, 2]
    s11 = lam[labels] * tr + 2 * mu[labels] * eps[0, 0]
    assert np.allclose(s11, s11[0], rtol=1e-14)
    assert np.allclose(2 * mu[labels] * eps[0, 1], 2 * mu[0] * eps[0, 1, 0], rtol=1e-14)
    assert np.allclose(2 * mu[labels] * eps[0, 2], 2 * mu[0] * eps[0, 2, 0], rtol=1e-14)
    assert np.allclose(eps.mean(axis=-1), O.voigt_to_tensor(macro), atol=1e-14)


@pytest.mark.parametrize("op,layers", [("R", [3, 7]), ("W", [3, 7]), ("MS", [4, 6]), ("C", [4, 6])])
@pytest.mark.parametrize("scheme", ["DS", "AS"])
def test_laminate_exact_solution(op, layers, scheme):
    """Phase depending on x only: traction continuity makes sigma_11,
    sigma_12, sigma_13 uniform and compatibility makes eps_22, eps_33, eps_23
    uniform (eqs. (1), (2), (4)); the discrete schemes reproduce this exactly
    (R, W for any layer thickness; MS and C when the layering has no Nyquist
    content, i.e. even thicknesses)."""
    nx = sum(layers)
    labels = np.array([1] * layers[0] + [0] * layers[1], dtype=np.uint8)
    shape = (4, 6, nx)
    phase = laminate(shape, labels)
    E, nu = np.array([1.0, 7.0]), np.array([0.3, 0.2])
    macro = np.array([0.7, -0.3, 0.4, 0.2, -0.5, 0.6])
    r = O.solve(phase, E, nu, macro, op=op, scheme=scheme, tol=1e-13, max_iter=2000)
    assert r.converged
    exact = _laminate_exact(labels, E, nu, macro)
    got = r.eps[:, :, 0, 0, :]
    assert np.allclose(r.eps, r.eps[:, :, :1, :1, :], atol=1e-10)  # depends on x only
    assert np.allclose(got, exact, atol=1e-10)


# --- direct finite-difference solve on tiny grids (W, R) --------------------------------

def _grad_R(U):
    def shift(f, a):
        return np.roll(f, shift=(-a[2], -a[1], -a[0]), axis=(-3, -2, -1))
    d = np.zeros((3, 3) + U.shape[1:])
    for i in range(3):
        for comp in range(3):
            for a in itertools.product((0, 1), repeat=3):
                d[i, comp] += (1 if a[i] == 1 else -1) * shift(U[comp], a) / 4.0
    return 0.5 * (d + d.transpose(1, 0, 2, 3, 4))


def _div_R(S):
    def shift(f, a):
        return np.roll(f, shift=(a[2], a[1], a[0]), axis=(-3, -2, -1))
    div = np.zeros((3,) + S.shape[2:])
    for j in range(3):
        for i in range(3):
            for a in itertools.product((0, 1), repeat=3):
                div[j] += (1 if a[i] == 0 else -1) * shift(S[i, j], a)
    return div


_AX = (-1, -2, -3)


def _grad_W(U):
    d = np.zeros((3, 3) + U.shape[1:])
    for i in range(3):
        for comp in range(3):
            d[i, comp] = np.roll(U[comp], -1, axis=_AX[i]) - U[comp]
    return 0.5 * (d + d.transpose(1, 0, 2, 3, 4))


def _div_W(S):
    div = np.zeros((3,) + S.shape[2:])
    for j in range(3):
        for i in range(3):
            div[j] += S[i, j] - np.roll(S[i, j], 1, axis=_AX[i])
    return div


@pytest.mark.parametrize("op", ["R", "W"])
def test_converged_iteration_equals_direct_finite_difference_solve(op, rng):
    """Assemble the finite-difference elasticity problem straight from the
    paper's stencils (R: eqs. (37)-(38); W: eq. (23)), solve it densely, and
    compare with the oracle's converged strain."""
    shape = (4, 6, 4)
    phase = (rng.random(shape) < 0.4).astype(np.uint8)
    E, nu = np.array([1.0, 5.0]), np.array([0.3, 0.25])
    lam, mu = O.lame_from_young(E, nu)
    C = [O.stiffness_tensor(l, m) for l, m in zip(lam, mu)]
    macro = np.array([1.0, 0.2, -0.3, 0.1, 0.4, -0.2])
    grad, div = (_grad_R, _div_R) if op == "R" else (_grad_W, _div_W)
    ebar = O.voigt_to_tensor(macro)[:, :, None, None, None] * np.ones((1, 1) + shape)

    def residual(u_flat, with_macro):
        U = u_flat.reshape((3,) + shape)
        eps = grad(U) + (ebar if with_macro else 0.0)
        return div(O.homogenization.apply_phasewise(C, phase, eps)).ravel()

    n = 3 * int(np.prod(shape))
    K = np.stack([residual(np.eye(n)[c], False) for c in range(n)], axis=1)
    f = -residual(np.zeros(n), True)
    u = np.linalg.lstsq(K, f, rcond=None)[0]
    eps_fd = grad(u.reshape((3,) + shape)) + ebar
    r = O.solve(phase, E, nu, macro, op=op, scheme="AS", tol=1e-13, max_iter=3000)
    assert r.converged
    assert np.max(np.abs(r.eps - eps_fd)) < 1e-10


@pytest.mark.parametrize("op", ["MS", "C"])
def test_converged_iteration_is_fixed_point_of_lippmann_schwinger(op, rng):
    """For the spectral operators, the converged strain solves eq. (6)
    (eps = eps_bar - G * (C - C0) : eps), assembled densely on a tiny grid."""
    shape = (4, 4, 6)
    phase = (rng.random(shape) < 0.4).astype(np.uint8)
    E, nu = np.array([1.0, 4.0]), np.array([0.3, 0.3])
    lam, mu = O.lame_from_young(E, nu)
    ref = O.reference_medium(lam, mu, "DS")
    C0 = O.stiffness_tensor(ref.lam0, ref.mu0)
    dC = [O.stiffness_tensor(l, m) - C0 for l, m in zip(lam, mu)]
    macro = np.array([0.3, 1.0, -0.2, 0.0, 0.5, 0.1])
    N = int(np.prod(shape))

    def lhs(eps6):
        eps = O.voigt_to_tensor(eps6.reshape((6,) + shape))
        tau = O.homogenization.apply_phasewise(dC, phase, eps)
        g = np.real(O.inverse_dft(O.green_apply(op, ref, O.forward_dft(tau), shape)))
        return O.tensor_to_voigt(eps + g).ravel()

    n = 6 * N
    M = np.stack([lhs(np.eye(n)[c]) for c in range(n)], axis=1)
    rhs = np.repeat(macro, N)
    sol = np.linalg.solve(M, rhs).reshape((6,) + shape)
    r = O.solve(phase, E, nu, macro, op=op, scheme="DS", tol=1e-14, max_iter=3000)
    assert np.max(np.abs(O.tensor_to_voigt(r.eps) - sol)) < 1e-10


# --- invariants -------------------------------------------------------------------

def test_direct_and_accelerated_schemes_reach_the_same_fields():
    """§4.2: for a given Green operator DS and AS give the same fields."""
    phase = sphere_inclusion((12, 12, 12), (6, 6, 6), 3.5)
    for op in ("R", "MS"):
        a = O.solve(phase, [1.0, 10.0], [0.3, 0.3], [1, 0, 0, 0, 0, 0], op=op, scheme="DS", tol=1e-12)
        b = O.solve(phase, [1.0, 10.0], [0.3, 0.3], [1, 0, 0, 0, 0, 0], op=op, scheme="AS", tol=1e-12)
        assert np.max(np.abs(a.eps - b.eps)) < 1e-9


def test_mirror_symmetry_R_and_MS_but_not_W():
    """A centred sphere under eps_bar = e1 (x) e1 is symmetric under x -> -x:
    eps_12, eps_13 are odd and the other components even.  G and G^R keep the
    symmetry, G^W breaks it (§4.1, §5)."""
    L = 12
    phase = sphere_inclusion((L, L, L), (L / 2, L / 2, L / 2), 3.5)
    sign = np.array([[1, -1, -1], [-1, 1, 1], [-1, 1, 1]])
    asym = {}
    for op in ("R", "MS", "W"):
        r = O.solve(phase, [1.0, 10.0], [0.3, 0.3], [1, 0, 0, 0, 0, 0], op=op, scheme="AS", tol=1e-12)
        mirrored = r.eps[:, :, :, :, ::-1] * sign[:, :, None, None, None]
        asym[op] = np.max(np.abs(mirrored - r.eps)) / np.max(np.abs(r.eps))
    assert asym["R"] < 1e-10 and asym["MS"] < 1e-10
    assert asym["W"] > 1e-3


def _mandel_from_voigt(Cv):
    w = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])
    return Cv * w[:, None] * w[None, :]


def test_effective_stiffness_within_voigt_reuss_bounds():
    """<C^-1>^-1 <= C_eff <= <C> as quadratic forms (discrete variational
    principles), C_eff from the six unit loads of eq. (5)."""
    phase = sphere_inclusion((10, 10, 10), (5, 5, 5), 3.0)
    E, nu = np.array([1.0, 20.0]), np.array([0.3, 0.2])
    Cv, its = O.effective_stiffness(phase, E, nu, op="R", scheme="AS", tol=1e-11)
    lam, mu = O.lame_from_young(E, nu)
    f = np.array([1 - phase.mean(), phase.mean()])
    M = [O.mandel_matrix(O.stiffness_tensor(l, m)) for l, m in zip(lam, mu)]
    voigt = f[0] * M[0] + f[1] * M[1]
    reuss = np.linalg.inv(f[0] * np.linalg.inv(M[0]) + f[1] * np.linalg.inv(M[1]))
    Ce = _mandel_from_voigt(Cv)
    assert np.allclose(Ce, Ce.T, atol=1e-8)
    assert np.linalg.eigvalsh(voigt - 0.5 * (Ce + Ce.T)).min() > -1e-9
    assert np.linalg.eigvalsh(0.5 * (Ce + Ce.T) - reuss).min() > -1e-9


def test_direct_scheme_below_half_diverges():
    """§6.1: beta < 1/2 in eq. (18) leads to non-converging direct schemes."""
    phase = sphere_inclusion((8, 8, 8), (4, 4, 4), 2.6)
    r = O.solve(phase, [1.0, 50.0], [0.3, 0.3], [1, 0, 0, 0, 0, 0], op="R", scheme="DS",
                tol=1e-12, max_iter=400, beta=0.45)
    assert not r.converged
    h = r.eta_history
    assert h[-1] > h[-50] > h[-100]


def test_periodic_sphere_array_approaches_printed_limit():
    """§5.3 prints C_11,11 -> 1.208 +- 0.001 as L grows (f = 20%,
    chi = 1e-4, kappa1 = 1, mu1 = 0.6).  At L = 32 the rotated scheme must sit
    below that limit and within 3% of it, and above its L = 16 value."""
    with open(os.path.join(GOLDEN, "paper_values.json")) as fh:
        gold = json.load(fh)["periodic_sphere_array_C1111_limit"]
    E1 = 1.5  # kappa1 = 1, mu1 = 0.6 -> E1 = 9 kappa mu / (3 kappa + mu)
    ref = O.reference_medium(None, None, "AS", E0=0.12 + np.sqrt(1e-4), nu0=0.25)
    vals = []
    for L in (16, 32):
        ph = sphere_array(L, 0.2)
        r = O.solve(ph, [E1, 1e-4 * E1], [0.25, 0.25], [1, 0, 0, 0, 0, 0], op="R", scheme="AS",
                    tol=1e-8, max_iter=2000, ref=ref)
        assert r.converged
        vals.append(O.tensor_to_voigt(r.mean_stress)[0])
    limit, tol = gold["value"], gold["tolerance"]
    assert vals[0] < vals[1] < limit + tol
    assert vals[1] > 0.97 * limit
