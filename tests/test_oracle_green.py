"""Pins of the oracle's transforms, wave vectors and Green operators against
what the paper and the mathematics fix (no GPU)."""
import itertools

import numpy as np
import pytest

import oracle as O


def _ref():
    return O.Reference(lam0=0.6, mu0=0.6)  # paper units: kappa=1, mu=0.6 (§2)


# --- discrete Fourier transform, eqs. (10)-(12) ------------------------------

@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 4, 10), (5, 6, 7)])
def test_forward_dft_matches_brute_force_sum(shape, rng):
    f = rng.standard_normal(shape)
    assert np.allclose(O.forward_dft(f), O.brute_force_dft(f), rtol=0, atol=1e-11)


def test_inverse_dft_normalisation(rng):
    f = rng.standard_normal((6, 4, 10))
    F = O.brute_force_dft(f)
    assert np.allclose(np.real(O.inverse_dft(F)), f, atol=1e-13)


def test_signed_modes_even_and_odd():
    assert list(O.signed_modes(8)) == [0, 1, 2, 3, 4, -3, -2, -1]  # Nyquist at +L/2
    assert list(O.signed_modes(7)) == [0, 1, 2, 3, -3, -2, -1]


# --- wave vectors (§4) ---------------------------------------------------------

def test_rotated_wave_vector_equals_literal_eq36(rng):
    shape = (12, 10, 14)
    k = O.wave_vector("R", shape)
    (mx, my, mz), (nx, ny, nz) = O.homogenization.mode_grid(shape)
    for _ in range(40):
        iz, iy, ix = rng.integers(0, shape[0]), rng.integers(0, shape[1]), rng.integers(0, shape[2])
        m = (O.signed_modes(nx)[ix], O.signed_modes(ny)[iy], O.signed_modes(nz)[iz])
        if any(2 * mm == L for mm, L in zip(m, (nx, ny, nz))):
            continue
        q = 2 * np.pi * np.array(m) / np.array([nx, ny, nz])
        assert np.allclose(k[:, iz, iy, ix], O.wave_vector_r_literal(q), atol=1e-14)


def _corner_strain_stencil(U):
    """Strain at voxel centres from corner displacements, eq. (37): corner
    index c sits at position c - 1/2; voxel v has corners v + a, a in {0,1}^3.
    U has shape (3, nz, ny, nx) with component 0 = x."""
    def shift(f, a):  # f(v + a) with periodic wrap; a = (ax, ay, az)
        return np.roll(f, shift=(-a[2], -a[1], -a[0]), axis=(-3, -2, -1))

    def d(i, comp):  # (1/4) [sum_{a_i=1} - sum_{a_i=0}] U_comp(v + a)
        acc = 0.0
        for a in itertools.product((0, 1), repeat=3):
            acc = acc + (1 if a[i] == 1 else -1) * shift(U[comp], a)
        return acc / 4.0

    eps = np.zeros((3, 3) + U.shape[1:])
    for i in range(3):
        for j in range(3):
            eps[i, j] = 0.5 * (d(i, j) + d(j, i))
    return eps


def _corner_divergence_stencil(S):
    """Eq. (38) at corner c (position c - 1/2): the voxels around the corner are
    c - a, a in {0,1}^3; the i-th term is sum over the voxels on the far side
    (a_i = 0) minus the near side (a_i = 1).  No 1/4 factor, as printed."""
    def shift(f, a):  # f(c - a)
        return np.roll(f, shift=(a[2], a[1], a[0]), axis=(-3, -2, -1))

    div = np.zeros((3,) + S.shape[2:])
    for j in range(3):
        for i in range(3):
            for a in itertools.product((0, 1), repeat=3):
                div[j] += (1 if a[i] == 0 else -1) * shift(S[i, j], a)
    return div


def test_rotated_k_is_the_symbol_of_the_corner_strain_stencil(rng):
    shape = (6, 8, 10)
    U = rng.standard_normal((3,) + shape)
    eps_stencil = _corner_strain_stencil(U)
    k = O.wave_vector("R", shape)
    Uh = O.forward_dft(U)
    eh = 0.5 * (np.einsum("i...,j...->ij...", k, Uh) + np.einsum("j...,i...->ij...", k, Uh))
    assert np.allclose(np.real(O.inverse_dft(eh)), eps_stencil, atol=1e-13)


def test_rotated_conj_k_is_the_symbol_of_the_corner_divergence(rng):
    shape = (6, 8, 10)
    S = rng.standard_normal((3, 3) + shape)
    S = 0.5 * (S + S.transpose(1, 0, 2, 3, 4))
    div = _corner_divergence_stencil(S)
    kc = np.conj(O.wave_vector("R", shape))
    spectral = np.einsum("i...,ij...->j...", kc, O.forward_dft(S))
    assert np.allclose(O.forward_dft(div) / -4.0, spectral, atol=1e-11)


def test_willot_pellegrini_k_is_forward_difference_symbol(rng):
    shape = (5, 6, 8)
    u = rng.standard_normal(shape)
    kW = O.wave_vector("W", shape)
    # d/dx u ~ u(x+e1) - u(x), eq. (23)
    fd = np.roll(u, -1, axis=-1) - u
    assert np.allclose(O.forward_dft(fd), kW[0] * O.forward_dft(u), atol=1e-12)
    # backward difference sigma(x) - sigma(x - e3) has symbol -conj(k_3)
    bd = u - np.roll(u, 1, axis=-3)
    assert np.allclose(O.forward_dft(bd), -np.conj(kW[2]) * O.forward_dft(u), atol=1e-12)


def test_centered_k_is_centered_difference_symbol(rng):
    shape = (6, 5, 8)
    u = rng.standard_normal(shape)
    kC = O.wave_vector("C", shape)
    cd = 0.5 * (np.roll(u, -1, axis=-2) - np.roll(u, 1, axis=-2))  # eq. (22)
    assert np.allclose(O.forward_dft(cd), kC[1] * O.forward_dft(u), atol=1e-12)


# --- Green operators (§3, §4) ----------------------------------------------------

def _ordinary_indices(op, shape, rng, n):
    special = O.special_modes(op, shape)
    out = []
    while len(out) < n:
        idx = tuple(int(rng.integers(0, s)) for s in shape)
        if idx == (0, 0, 0) or special[idx]:
            continue
        out.append(idx)
    return out


def _q_at(shape, idx):
    nz, ny, nx = shape
    iz, iy, ix = idx
    m = np.array([O.signed_modes(nx)[ix], O.signed_modes(ny)[iy], O.signed_modes(nz)[iz]])
    return 2 * np.pi * m / np.array([nx, ny, nz])


def test_ms_general_solve_matches_closed_form_eq8(rng):
    shape = (8, 6, 10)
    ref = O.Reference(0.37, 1.3)
    for idx in _ordinary_indices("MS", shape, rng, 12):
        G = O.green_tensor_at("MS", ref, shape, idx)
        assert np.allclose(G, O.green_continuous_closed_form(ref, _q_at(shape, idx)), atol=1e-14)


@pytest.mark.parametrize("op", ["C", "W", "R", "MS"])
def test_general_solve_matches_eq39(op, rng):
    shape = (8, 6, 10)
    ref = O.Reference(0.9, 0.45)
    k = O.wave_vector(op, shape)
    for idx in _ordinary_indices(op, shape, rng, 12):
        G = O.green_tensor_at(op, ref, shape, idx)
        kk = k[(slice(None),) + idx]
        assert np.allclose(G, O.green3_closed_form(ref, kk), atol=1e-13)


@pytest.mark.parametrize("op", ["MS", "C", "W", "R"])
def test_green_minor_and_hermitian_major_symmetry_eq26(op, rng):
    shape = (6, 8, 4)
    for idx in _ordinary_indices(op, shape, rng, 6):
        G = O.green_tensor_at(op, _ref(), shape, idx)
        assert np.allclose(G, G.transpose(1, 0, 2, 3), atol=1e-15)
        assert np.allclose(G, G.transpose(0, 1, 3, 2), atol=1e-15)
        assert np.allclose(G, np.conj(G.transpose(2, 3, 0, 1)), atol=1e-14)


def _mirror(shape, idx):
    return tuple((-i) % s for i, s in zip(idx, shape))


@pytest.mark.parametrize("op", ["C", "W"])
def test_conjugate_symmetry_eq27_including_nyquist(op):
    shape = (4, 6, 8)
    for idx in itertools.product(range(4), range(6), range(8)):
        if idx == (0, 0, 0) or O.special_modes(op, shape)[idx]:
            continue
        G = O.green_tensor_at(op, _ref(), shape, idx)
        Gm = O.green_tensor_at(op, _ref(), shape, _mirror(shape, idx))
        assert np.allclose(np.conj(G), Gm, atol=1e-14)


def test_rotated_green_is_real_and_even_eq34():
    shape = (4, 6, 8)
    for idx in itertools.product(range(4), range(6), range(8)):
        if idx == (0, 0, 0):
            continue
        G = O.green_tensor_at("R", _ref(), shape, idx)
        assert np.max(np.abs(G.imag)) < 1e-14
        Gm = O.green_tensor_at("R", _ref(), shape, _mirror(shape, idx))
        assert np.allclose(G, Gm, atol=1e-14)


def test_rotated_green_is_continuous_operator_of_t():
    """G^R(q) is eq. (8) evaluated at the real vector t_i = sin(q_i/2) prod cos(q_j/2)."""
    shape = (6, 10, 8)
    ref = O.Reference(0.2, 0.8)
    rng = np.random.default_rng(5)
    for idx in _ordinary_indices("R", shape, rng, 10):
        q = _q_at(shape, idx)
        t = np.array([np.sin(q[a] / 2) * np.cos(q[(a + 1) % 3] / 2) * np.cos(q[(a + 2) % 3] / 2)
                      for a in range(3)])
        G = O.green_tensor_at("R", ref, shape, idx)
        assert np.allclose(G, O.green_continuous_closed_form(ref, t), atol=1e-13)


def _mandel(G):
    return O.mandel_matrix(G)


@pytest.mark.parametrize("op", ["MS", "C", "W", "R"])
def test_projection_properties(op, rng):
    """G'C0G' = G' and G'C0 has eigenvalues {0, 1} with rank 3 at ordinary
    frequencies; conj(k).C0:G':tau = conj(k).tau (the discrete equilibrium)."""
    shape = (6, 8, 4)
    ref = O.Reference(0.9, 0.45)
    M0 = _mandel(O.stiffness_tensor(ref.lam0, ref.mu0))
    k = O.wave_vector(op, shape)
    for idx in _ordinary_indices(op, shape, rng, 6):
        G = O.green_tensor_at(op, ref, shape, idx)
        M = _mandel(G)
        assert np.allclose(M @ M0 @ M, M, atol=1e-13)
        ev = np.sort(np.abs(np.linalg.eigvals(M @ M0)))
        assert np.allclose(ev, [0, 0, 0, 1, 1, 1], atol=1e-12)
        tau = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        tau = 0.5 * (tau + tau.T)
        kk = k[(slice(None),) + idx]
        lhs = np.conj(kk) @ O.homogenization.contract(O.stiffness_tensor(ref.lam0, ref.mu0),
                                                      np.einsum("ijkl,kl->ij", G, tau))
        assert np.allclose(lhs, np.conj(kk) @ tau, atol=1e-13)


def test_special_modes_values():
    ref = O.Reference(0.9, 0.45)
    shape = (4, 6, 8)
    M0 = _mandel(O.stiffness_tensor(ref.lam0, ref.mu0))
    # MS at a Nyquist mode: G = (C0)^-1, eq. (14)
    G = O.green_tensor_at("MS", ref, shape, (1, 3, 2))
    assert np.allclose(_mandel(G) @ M0, np.eye(6), atol=1e-13)
    # R with two Nyquist indices: 0, eq. (41); with one: ordinary, rank 3
    assert np.allclose(O.green_tensor_at("R", ref, shape, (2, 3, 1)), 0)
    G1 = O.green_tensor_at("R", ref, shape, (2, 1, 1))
    assert np.linalg.matrix_rank(_mandel(G1) @ M0, tol=1e-10) == 3
    # C where every q_i is 0 or pi: 0, eq. (29)
    assert np.allclose(O.green_tensor_at("C", ref, shape, (2, 0, 4)), 0)
    # W: no special mode
    assert not O.special_modes("W", shape).any()


@pytest.mark.parametrize("op", ["C", "W", "R"])
def test_discrete_operators_tend_to_continuous_as_q_to_0(op):
    """G^{C,W,R} -> G as q -> 0 (§4.1): the gap shrinks linearly with |q|."""
    ref = _ref()
    gaps = []
    for L in (256, 512, 1024):
        shape = (L, L, L)
        idx = (1, 2, 1)
        q = _q_at(shape, idx)
        k = O.homogenization.wave_vector_at(op, shape, idx)
        G = O.green3_closed_form(ref, k)
        gaps.append(np.max(np.abs(G - O.green_continuous_closed_form(ref, q))))
    assert gaps[2] < gaps[1] < gaps[0] < 0.05
    assert gaps[0] / gaps[2] > 3.0


# --- equilibrium norm, eq. (43) -----------------------------------------------------

def _stress_like(rng, shape):
    S = rng.standard_normal((3, 3) + shape)
    S = 0.5 * (S + S.transpose(1, 0, 2, 3, 4))
    S[0, 0] += 3.0
    return S


def test_equilibrium_norm_matches_real_space_corner_stencil(rng):
    shape = (6, 8, 10)
    S = _stress_like(rng, shape)
    div = _corner_divergence_stencil(S) / 4.0
    eta_real = np.sqrt(np.mean(np.sum(div ** 2, axis=0))) / np.linalg.norm(S.mean(axis=(2, 3, 4)))
    assert abs(O.equilibrium_norm("R", S) - eta_real) < 1e-13 * eta_real


def test_equilibrium_norm_matches_backward_difference_for_W(rng):
    shape = (5, 8, 6)
    S = _stress_like(rng, shape)
    div = np.zeros((3,) + shape)
    for j in range(3):
        for i, ax in zip(range(3), (-1, -2, -3)):
            div[j] += S[i, j] - np.roll(S[i, j], 1, axis=ax)
    eta_real = np.sqrt(np.mean(np.sum(div ** 2, axis=0))) / np.linalg.norm(S.mean(axis=(2, 3, 4)))
    assert abs(O.equilibrium_norm("W", S) - eta_real) < 1e-13 * eta_real
