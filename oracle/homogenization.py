"""FP64 CPU oracle of the Lippmann-Schwinger FFT iteration.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the GPU library and never imports it.

Source: F. Willot, "Fourier-based schemes for computing the mechanical
response of composites with accurate local fields" (arXiv 1412.8398).
Equation numbers below are the paper's.

Everything is plain NumPy in float64/complex128, written to be checked by
eye against the paper:

* fields are full 3x3 tensors, arrays of shape (3, 3, nz, ny, nx); tensor
  index 0/1/2 is the x/y/z direction (array axes 4/3/2);
* the discrete Fourier transform is the unnormalised forward sum of eq. (11)
  and the 1/N-normalised inverse of eq. (10), i.e. ``scipy.fft.fftn`` /
  ``ifftn`` over the three grid axes, on all host cores;
* the Green operator is applied by solving, per frequency, the defining
  linear system of the discrete equations, eq. (19), with a general complex
  3x3 solve (no closed form);
* the direct and accelerated schemes, eqs. (9) and (16), are run step by step
  so that iterates can be compared at equal iteration index.

Readings of the paper taken here:
  R1  eq. (24) is read with gradient k and divergence conj(k): the operator
      is sym[k_i (A^-1)_jk conj(k_l)] with A = lam0 conj(k) k^T
      + mu0 k conj(k)^T + mu0 |k|^2 I.  This is the operator that eq. (19)
      defines and it agrees with eq. (39).
  R2  in eq. (40) the off-diagonal entries of s are read as
      s_ij = -4 Im(r_k conj r_j) Im(r_k conj r_i) (k the third index), the
      symmetric form; see ``green3_closed_form``.
  R3  eq. (43): the middle (real-space mean) expression is authoritative; with
      the unnormalised forward transform of eq. (11) it equals
      sqrt(sum_q |conj(k).sigma(q)|^2) / ||sigma(q=0)||_F.
  R4  the divergence in eq. (43) is conj(k) . sigma (the divergence the
      discrete scheme enforces, eq. (19)); for MS, C and R this has the same
      modulus as k . sigma.
  R5  the convergence test of the accelerated scheme uses sigma^k = C:eps^k
      of the scheme's own iterate.
  R6  positions are in voxel units (spacing 1).
  R7  with more than two phases, or unequal Poisson ratios, eqs. (17)/(18)
      take the smallest and largest phase bulk and shear moduli.
  R9  eq. (15), the symmetrised alternative to eq. (14) for the continuous
      operator, is read with -q the grid partner of q: the mode whose DFT
      coefficient is the conjugate of q's for a real field, i.e. -q with
      every Nyquist component kept at +pi (a component -pi is not a grid
      mode).  At a mode with some q_i = pi the operator is the mean of the
      continuous operator of eq. (8) at q and at that partner (real, so the
      conjugate in eq. (15) changes nothing); the inverse transform is then
      real.  Read literally, with -q the negated vector, eq. (15) would equal
      G(q) (eq. (8) is real and even) and change nothing.  This variant is
      operator "MSS"; everywhere else it is "MS".  This operator does not
      impose equilibrium at those modes (its fixed point leaves
      conj(k).sigma(q) nonzero there: with every mode in eq. (43), eta
      stalls at 0.26 on a 6x8x10 Voronoi cell), so for "MSS" the sum of
      eq. (43) runs over the other modes, where it is the continuous operator.
  R8  the conjugate-gradient solver that §1 and §7 name as another use of
      the modified operators is read as plain (Hestenes-Stiefel) conjugate
      gradients on the discrete problem of eq. (19) for the strain
      fluctuation, in the inner product <a, b> = sum_x a : C0 : b, in which
      G'C is self-adjoint and positive on compatible zero-mean fields
      (G'C0G' = G'); the reference medium is that of the accelerated scheme,
      eq. (17); see ``solve_cg``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import os

import numpy as np
import scipy.fft as _sfft

OPERATORS = ("MS", "C", "W", "R", "MSS")
SCHEMES = ("DS", "AS")

# ----------------------------------------------------------------------------
# Isotropic elasticity (§2, eq. (2))
# ----------------------------------------------------------------------------

_I3 = np.eye(3)


def lame_from_young(E, nu):
    """lambda = E nu / ((1+nu)(1-2nu)), mu = E / (2(1+nu))."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def bulk_modulus(lam, mu):
    """kappa = lambda + (2/d) mu with d = 3 (§2)."""
    return lam + 2.0 * mu / 3.0


def stiffness_tensor(lam, mu):
    """C_ijkl = lambda d_ij d_kl + mu (d_ik d_jl + d_il d_jk), eq. (2)."""
    d = _I3
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def contract(C, eps):
    """(C:eps)_ij = sum_kl C_ijkl eps_kl for a constant tensor C."""
    return np.einsum("ijkl,kl...->ij...", C, eps)


def apply_phasewise(tables, phase, eps):
    """sum_kl C(x)_ijkl eps_kl(x), with C(x) = tables[phase(x)]."""
    out = np.zeros_like(eps)
    for p, C in enumerate(tables):
        m = phase == p
        if m.any():
            out[:, :, m] = np.einsum("ijkl,klv->ijv", C, eps[:, :, m])
    return out


# Mandel basis: an orthonormal basis of symmetric 3x3 tensors.
_MANDEL_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def _mandel_basis():
    B = np.zeros((6, 3, 3))
    for a, (i, j) in enumerate(_MANDEL_PAIRS):
        if i == j:
            B[a, i, i] = 1.0
        else:
            B[a, i, j] = B[a, j, i] = 1.0 / math.sqrt(2.0)
    return B


_MB = _mandel_basis()


def mandel_matrix(C):
    """6x6 matrix of a minor-symmetric 4th-order tensor in the Mandel basis."""
    return np.einsum("aij,ijkl,bkl->ab", _MB, C, _MB)


def tensor_from_mandel(M):
    return np.einsum("aij,ab,bkl->ijkl", _MB, M, _MB)


# ----------------------------------------------------------------------------
# Reference medium (§3, eqs. (17), (18); §6.1 for E0, nu0)
# ----------------------------------------------------------------------------


@dataclass
class Reference:
    lam0: float
    mu0: float

    @property
    def kappa0(self):
        return bulk_modulus(self.lam0, self.mu0)


def reference_medium(lam, mu, scheme, beta=0.5, E0=None, nu0=None):
    """Reference tensor C0.

    * explicit (E0, nu0): the parametrisation of §6.1;
    * accelerated scheme: kappa0 = sqrt(kappa1 kappa2), mu0 = sqrt(mu1 mu2),
      eq. (17);
    * direct scheme: kappa0 = beta (kappa1 + kappa2), mu0 = beta (mu1 + mu2),
      eq. (18), beta = 1/2 by default;
    with kappa1/kappa2 (mu1/mu2) the smallest and largest phase values (R7).
    """
    if E0 is not None:
        l0, m0 = lame_from_young(E0, nu0)
        return Reference(float(l0), float(m0))
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    kap = bulk_modulus(lam, mu)
    k1, k2 = kap.min(), kap.max()
    m1, m2 = mu.min(), mu.max()
    if scheme == "AS":
        k0, m0 = math.sqrt(k1 * k2), math.sqrt(m1 * m2)
    elif scheme == "DS":
        k0, m0 = beta * (k1 + k2), beta * (m1 + m2)
    else:
        raise ValueError(scheme)
    return Reference(float(k0 - 2.0 * m0 / 3.0), float(m0))


# ----------------------------------------------------------------------------
# Fourier modes (§3, eqs. (10)-(12)) and discrete wave vectors (§4)
# ----------------------------------------------------------------------------


def signed_modes(L):
    """m_i of eq. (12): 1-L/2 .. L/2 for even L (Nyquist at +L/2), and
    -(L-1)/2 .. (L-1)/2 for odd L, listed in DFT index order 0..L-1."""
    m = np.arange(L)
    return np.where(2 * m <= L, m, m - L)


def _cos_sin(num, den):
    """cos and sin of 2 pi num/den, exact at multiples of pi/2."""
    num = np.asarray(num)
    ang = 2.0 * np.pi * num / den
    c, s = np.cos(ang), np.sin(ang)
    quarter = (4 * num) % den == 0
    k = ((4 * num) // den) % 4
    c = np.where(quarter, np.choose(k, [1.0, 0.0, -1.0, 0.0]), c)
    s = np.where(quarter, np.choose(k, [0.0, 1.0, 0.0, -1.0]), s)
    return c, s


def mode_grid(shape):
    """Signed mode indices broadcastable over (nz, ny, nx): (mx, my, mz)."""
    nz, ny, nx = shape
    mx = signed_modes(nx)[None, None, :]
    my = signed_modes(ny)[None, :, None]
    mz = signed_modes(nz)[:, None, None]
    return (mx, my, mz), (nx, ny, nz)


def wave_vector(op, shape):
    """k(q) for every grid frequency, array of shape (3, nz, ny, nx), complex.

    MS: k = i q                        (continuous Green operator, eqs. (7)-(8))
    C : k = i sin(q)                   eq. (20)
    W : k = exp(i q) - 1               eq. (21)
    R : k = (i/4) tan(q_i/2) prod_j (1 + exp(i q_j)), eq. (36), evaluated as
        2 i exp(i (q1+q2+q3)/2) sin(q_i/2) prod_{j != i} cos(q_j/2),
        obtained with 1 + exp(i a) = 2 cos(a/2) exp(i a/2) and
        tan(a/2) cos(a/2) = sin(a/2); this form has no tan(pi/2).
    with q_i = 2 pi m_i / L_i (eq. (12)).
    """
    (mx, my, mz), (nx, ny, nz) = mode_grid(shape)
    return _wave_vector_from_modes(op, (mx, my, mz), (nx, ny, nz))


def wave_vector_at(op, shape, index):
    """k(q) at one grid frequency ``index`` = (iz, iy, ix)."""
    nz, ny, nx = shape
    iz, iy, ix = index
    ms = (np.array(signed_modes(nx)[ix]), np.array(signed_modes(ny)[iy]),
          np.array(signed_modes(nz)[iz]))
    return _wave_vector_from_modes(op, ms, (nx, ny, nz))


def _wave_vector_from_modes(op, ms, Ls):
    full = np.broadcast_shapes(*(np.shape(m) for m in ms))
    k = np.zeros((3,) + tuple(full), dtype=np.complex128)
    if op in ("MS", "MSS"):
        for a in range(3):
            k[a] = 1j * (2.0 * np.pi * ms[a] / Ls[a])
    elif op == "C":
        for a in range(3):
            _, s = _cos_sin(ms[a], Ls[a])
            k[a] = 1j * s
    elif op == "W":
        # exp(i q) - 1 written as -2 sin^2(q/2) + 2 i sin(q/2) cos(q/2), which
        # is the same number without the cancellation of cos(q) - 1 at small q
        for a in range(3):
            ch, sh = _cos_sin(ms[a], 2 * Ls[a])
            k[a] = -2.0 * sh * sh + 2j * sh * ch
    elif op == "R":
        # half angles q_a/2 = 2 pi m_a / (2 L_a)
        ch, sh = zip(*(_cos_sin(ms[a], 2 * Ls[a]) for a in range(3)))
        # exp(i (q1+q2+q3)/2) = prod_a (ch_a + i sh_a)
        phase = (ch[0] + 1j * sh[0]) * (ch[1] + 1j * sh[1]) * (ch[2] + 1j * sh[2])
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            t = sh[a] * ch[b] * ch[c]
            k[a] = 2j * phase * t
    else:
        raise ValueError(op)
    return k


def wave_vector_r_literal(q):
    """Eq. (36) typed literally, for a single frequency q (3 reals) with no
    q_i = pi: k_i = (i/4) tan(q_i/2) prod_j (1 + exp(i q_j))."""
    q = np.asarray(q, dtype=np.float64)
    prod = np.prod(1.0 + np.exp(1j * q))
    return 0.25j * np.tan(q / 2.0) * prod


def special_modes(op, shape):
    """Boolean mask of the nonzero frequencies where the paper replaces the
    Green operator:

    MS: (C0)^-1 where some q_i = pi with L_i even, eq. (14);
    C : 0 where every q_i is 0 or pi (L even), eq. (29), applied in 3D (§4.2);
    R : 0 where q_i = q_j = pi for two indices i != j (L even), eq. (41);
    W : none (k^W != 0 for q != 0, §4.1).
    """
    (mx, my, mz), (nx, ny, nz) = mode_grid(shape)
    ms, Ls = (mx, my, mz), (nx, ny, nz)
    full = np.broadcast_shapes(mx.shape, my.shape, mz.shape)
    nyq = [np.broadcast_to((L % 2 == 0) & (m == L // 2), full) for m, L in zip(ms, Ls)]
    zero = [np.broadcast_to(m == 0, full) for m in ms]
    nonzero_q = ~(zero[0] & zero[1] & zero[2])
    if op in ("MS", "MSS"):
        return (nyq[0] | nyq[1] | nyq[2]) & nonzero_q
    if op == "C":
        return (nyq[0] | zero[0]) & (nyq[1] | zero[1]) & (nyq[2] | zero[2]) & nonzero_q
    if op == "R":
        n = nyq[0].astype(int) + nyq[1].astype(int) + nyq[2].astype(int)
        return n >= 2
    if op == "W":
        return np.zeros(full, dtype=bool)
    raise ValueError(op)


# ----------------------------------------------------------------------------
# Green operator application (§3, §4)
# ----------------------------------------------------------------------------


def compliance_apply(ref: Reference, tau):
    """(C0)^-1 : tau for isotropic C0, obtained by inverting the Mandel matrix
    of C0 (the value of the Green operator at MS Nyquist modes, eq. (14))."""
    C0 = stiffness_tensor(ref.lam0, ref.mu0)
    S0 = tensor_from_mandel(np.linalg.inv(mandel_matrix(C0)))
    return np.einsum("ijkl,kl...->ij...", S0, tau)


_GREEN_CACHE = {}


def _green_plan(op, ref: Reference, shape):
    """Per-frequency data of the Green operator for one (operator, C0, grid):
    k(q), the special-mode mask and the inverse of A(q) (defined in
    ``green_apply``) at the ordinary frequencies.  A depends only on q and C0,
    so it is inverted once and reused across iterations."""
    key = (op, float(ref.lam0), float(ref.mu0), tuple(shape))
    plan = _GREEN_CACHE.get(key)
    if plan is not None:
        return plan
    if len(_GREEN_CACHE) > 8:
        _GREEN_CACHE.clear()
    k = wave_vector(op, shape)
    kc = np.conj(k)
    lam0, mu0 = ref.lam0, ref.mu0
    k2 = np.sum(np.abs(k) ** 2, axis=0)
    A = (lam0 * np.einsum("j...,l...->...jl", kc, k)
         + mu0 * np.einsum("j...,l...->...jl", k, kc)
         + mu0 * k2[..., None, None] * _I3)
    special = special_modes(op, shape)
    ordinary = ~special
    ordinary[0, 0, 0] = False
    Ainv = np.linalg.inv(A[ordinary])
    partner = None
    if op == "MSS" and special.any():
        # eq. (15) (R9): at the special modes, k at q and at the grid partner
        # of q (-q with the Nyquist components kept at +pi), and A^-1 at both
        (mx, my, mz), (nx, ny, nz) = mode_grid(shape)
        ms = [np.broadcast_to(m, shape) for m in (mx, my, mz)]
        Ls = (nx, ny, nz)
        kp = np.zeros((3,) + tuple(shape), dtype=np.complex128)
        for a in range(3):
            nyq_a = (Ls[a] % 2 == 0) & (ms[a] == Ls[a] // 2)
            mp = np.where(nyq_a, ms[a], -ms[a])
            kp[a] = 1j * (2.0 * np.pi * mp / Ls[a])
        kq, kpq = k[:, special], kp[:, special]

        def inv_a(kk):
            kkc = np.conj(kk)
            k2s = np.sum(np.abs(kk) ** 2, axis=0)
            Am = (lam0 * np.einsum("jm,lm->mjl", kkc, kk) + mu0 * np.einsum("jm,lm->mjl", kk, kkc)
                  + mu0 * k2s[:, None, None] * _I3)
            return np.linalg.inv(Am)

        partner = (kq, kpq, inv_a(kq), inv_a(kpq))
    plan = (k, kc, special, ordinary, Ainv, partner)
    _GREEN_CACHE[key] = plan
    return plan


def green_apply(op, ref: Reference, tau_hat, shape=None):
    """Return G'(q) : tau(q) at every nonzero frequency (q = 0 is set to 0).

    For an ordinary frequency the discrete equations (19),
        conj(k)_i sigma_ij = 0,  eps_ij = (k_i u_j + k_j u_i)/2,
        sigma = C0:eps + tau,
    give A u = -b with b_j = conj(k)_i tau_ij and
        A_jl = lam0 conj(k_j) k_l + mu0 k_j conj(k_l) + mu0 |k|^2 d_jl,
    and G':tau = -eps = -sym(k (x) u).  Special frequencies follow
    ``special_modes``.
    """
    if shape is None:
        shape = tau_hat.shape[2:]
    shape = tuple(shape)
    k, kc, special, ordinary, Ainv, partner = _green_plan(op, ref, shape)
    # b_j = sum_i conj(k_i) tau_ij
    b = np.einsum("i...,ij...->j...", kc, tau_hat)
    u = np.zeros(shape + (3,), dtype=np.complex128)
    rhs = np.moveaxis(b, 0, -1)
    u[ordinary] = -np.einsum("mjl,ml->mj", Ainv, rhs[ordinary])
    u = np.moveaxis(u, -1, 0)
    eps = 0.5 * (np.einsum("i...,j...->ij...", k, u) + np.einsum("j...,i...->ij...", k, u))
    out = -eps
    if op == "MS" and special.any():
        out[:, :, special] = compliance_apply(ref, tau_hat[:, :, special])
    if op == "MSS" and special.any():
        # eq. (15): the mean of the continuous operator at q and at its partner
        ts = tau_hat[:, :, special]  # (3, 3, M)
        g = np.zeros_like(ts)
        for kk, Ai in ((partner[0], partner[2]), (partner[1], partner[3])):
            b = np.einsum("im,ijm->jm", np.conj(kk), ts)
            u = -np.einsum("mjl,lm->jm", Ai, b)
            e = 0.5 * (np.einsum("im,jm->ijm", kk, u) + np.einsum("jm,im->ijm", kk, u))
            g += 0.5 * (-e)
        out[:, :, special] = g
    # C and R special modes: G' = 0 (already 0 since u = 0 there); q = 0: 0.
    out[:, :, 0, 0, 0] = 0.0
    return out


def green_tensor_at(op, ref: Reference, shape, index):
    """The 4th-order tensor G'_ijkl at one grid frequency ``index`` = (iz, iy, ix),
    built by applying ``green_apply`` to the symmetric unit tensors."""
    G = np.zeros((3, 3, 3, 3), dtype=np.complex128)
    for kk in range(3):
        for ll in range(3):
            E = np.zeros((3, 3) + tuple(shape), dtype=np.complex128)
            E[kk, ll][index] += 0.5
            E[ll, kk][index] += 0.5
            r = green_apply(op, ref, E, shape)
            G[:, :, kk, ll] = r[(slice(None), slice(None)) + tuple(index)]
    return G


def green_continuous_closed_form(ref: Reference, q):
    """Eq. (8): G_ijkl(q) = (1/mu0)[ (q_i q_l d_jk / |q|^2)_sym
    - (lam0+mu0)/(lam0+2mu0) q_i q_j q_k q_l / |q|^4 ], symmetrised over
    (i,j) and (k,l)."""
    q = np.asarray(q, dtype=np.float64)
    n = q / np.linalg.norm(q)
    lam0, mu0 = ref.lam0, ref.mu0
    T = np.einsum("i,l,jk->ijkl", n, n, _I3)
    Tsym = 0.25 * (T + T.transpose(1, 0, 2, 3) + T.transpose(0, 1, 3, 2)
                   + T.transpose(1, 0, 3, 2))
    return (Tsym - (lam0 + mu0) / (lam0 + 2 * mu0) * np.einsum("i,j,k,l->ijkl", n, n, n, n)) / mu0


def green3_closed_form(ref: Reference, k):
    """Eq. (39) for one complex wave vector k (3,), with r = k/|k| and the
    tensor s of eq. (40) read symmetrically (R2):
        s_jj = 4 Im(r_i conj r_k)^2,
        s_ij = -4 Im(r_k conj r_j) Im(r_k conj r_i)  (i, j, k distinct).
    Numerator terms are symmetrised over (i,j) and (k,l) like eq. (24)."""
    k = np.asarray(k, dtype=np.complex128)
    r = k / np.linalg.norm(k)
    rc = np.conj(r)
    lam0, mu0 = ref.lam0, ref.mu0
    s = np.zeros((3, 3))
    for j in range(3):
        i, kk = (j + 1) % 3, (j + 2) % 3
        s[j, j] = 4.0 * np.imag(r[i] * rc[kk]) ** 2
    for i in range(3):
        for j in range(3):
            if i != j:
                kk = 3 - i - j
                s[i, j] = -4.0 * np.imag(r[kk] * rc[j]) * np.imag(r[kk] * rc[i])

    def sym(T):
        return 0.25 * (T + T.transpose(1, 0, 2, 3) + T.transpose(0, 1, 3, 2)
                       + T.transpose(1, 0, 3, 2))

    t1 = sym(np.einsum("i,l,jk->ijkl", r, rc, _I3))
    t2 = sym(np.einsum("i,l,jk->ijkl", r, rc, s))
    ReRR = np.real(np.einsum("i,j->ij", r, rc))
    t3 = np.einsum("ij,kl->ijkl", ReRR, ReRR)
    t4 = np.einsum("i,j,k,l->ijkl", r, r, rc, rc)
    num = (lam0 + 2 * mu0) * t1 + lam0 * (t2 - t3) - mu0 * t4
    den = mu0 * (2 * (lam0 + mu0) - lam0 * abs(np.sum(r * r)) ** 2)
    return num / den


# ----------------------------------------------------------------------------
# Discrete Fourier transform (§3, eqs. (10)-(11))
# ----------------------------------------------------------------------------

_AXES = (-3, -2, -1)
_WORKERS = int(os.environ.get("ORACLE_WORKERS", os.cpu_count() or 1))


def forward_dft(f):
    """f(q) = sum_x f(x) exp(-i q.x), eq. (11), over the three grid axes."""
    return _sfft.fftn(f, axes=_AXES, workers=_WORKERS)


def inverse_dft(F):
    """f(x) = (1/L^d) sum_q f(q) exp(i q.x), eq. (10)."""
    return _sfft.ifftn(F, axes=_AXES, workers=_WORKERS)


def brute_force_dft(f):
    """Eq. (11) summed term by term (for tiny grids); f has shape (nz, ny, nx)."""
    nz, ny, nx = f.shape
    out = np.zeros(f.shape, dtype=np.complex128)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for a in range(nz):
        for b in range(ny):
            for c in range(nx):
                ph = 2 * np.pi * (a * z / nz + b * y / ny + c * x / nx)
                out[a, b, c] = np.sum(f * np.exp(-1j * ph))
    return out


# ----------------------------------------------------------------------------
# Equilibrium norm (§6.1, eq. (43))
# ----------------------------------------------------------------------------


def equilibrium_norm(op, sigma):
    """eta = sqrt(sum_q |conj(k(q)) . sigma(q)|^2) / ||sigma(q=0)||_F (R3, R4),
    where (conj(k).sigma)_j = sum_i conj(k_i) sigma_ij and the Frobenius norm
    runs over all nine tensor entries."""
    shape = sigma.shape[2:]
    s_hat = forward_dft(sigma)
    kc = np.conj(wave_vector(op, shape))
    div = np.einsum("i...,ij...->j...", kc, s_hat)
    if op == "MSS":  # R9: equilibrium is imposed off the Nyquist modes only
        div[:, special_modes(op, shape)] = 0.0
    num = math.sqrt(float(np.sum(np.abs(div) ** 2)))
    den = float(np.linalg.norm(s_hat[:, :, 0, 0, 0]))
    return num / den


# ----------------------------------------------------------------------------
# Iterative schemes (§3, eqs. (6), (9), (16))
# ----------------------------------------------------------------------------


def voigt_to_tensor(v):
    """Tensor Voigt order (11, 22, 33, 23, 13, 12) -> symmetric 3x3 (no factor
    2 on shear entries)."""
    v = np.asarray(v, dtype=np.float64)
    t = np.zeros((3, 3) + v.shape[1:])
    for a, (i, j) in enumerate(_MANDEL_PAIRS):
        t[i, j] = v[a]
        t[j, i] = v[a]
    return t


def tensor_to_voigt(t):
    return np.stack([t[i, j] for (i, j) in _MANDEL_PAIRS])


@dataclass
class SolveResult:
    iterations: int
    eps: np.ndarray            # (3,3,nz,ny,nx) at the returned iterate
    sigma: np.ndarray
    mean_stress: np.ndarray    # (3,3)
    eta: float
    eta_history: list = field(default_factory=list)
    mean_stress_history: list = field(default_factory=list)
    converged: bool = True
    iterates: list = field(default_factory=list)  # optional (3,3,...) per k


def laminate_exact(labels_x, E, nu, macro_strain):
    """Exact strain of a laminate whose phase depends on the x index only
    (labels_x[i] for every voxel of x index i): traction continuity across the
    layers (eqs. (1)-(2)) makes sigma_11, sigma_12, sigma_13 uniform and
    compatibility with the applied strain (eq. (4)) makes eps_22, eps_33,
    eps_23 equal to their averages.  Returns (3, 3, nx)."""
    lam, mu = lame_from_young(E, nu)
    lam_x, mu_x = lam[np.asarray(labels_x)], mu[np.asarray(labels_x)]
    e = voigt_to_tensor(np.asarray(macro_strain, dtype=np.float64))
    m = lambda f: float(np.mean(f))  # noqa: E731  (mean over the layers)
    S = (e[0, 0] + m(lam_x / (lam_x + 2 * mu_x)) * (e[1, 1] + e[2, 2])) / m(1 / (lam_x + 2 * mu_x))
    T12 = e[0, 1] / m(1 / (2 * mu_x))
    T13 = e[0, 2] / m(1 / (2 * mu_x))
    eps = np.zeros((3, 3, lam_x.size))
    eps[1, 1], eps[2, 2] = e[1, 1], e[2, 2]
    eps[1, 2] = eps[2, 1] = e[1, 2]
    eps[0, 0] = (S - lam_x * (e[1, 1] + e[2, 2])) / (lam_x + 2 * mu_x)
    eps[0, 1] = eps[1, 0] = T12 / (2 * mu_x)
    eps[0, 2] = eps[2, 0] = T13 / (2 * mu_x)
    return eps


def solve(phase, E, nu, macro_strain, op="R", scheme="DS", tol=1e-10, max_iter=1000,
          eps_init=None, ref: Reference | None = None, beta=0.5, keep_iterates=False):
    """Run the direct (eq. (9)) or accelerated (eq. (16)) scheme.

    Iteration k (k = 0, 1, ...):
      sigma^k = C : eps^k;  eta^k by eq. (43); stop at the first k with
      eta^k <= tol (or k = max_iter);
      tau^k = sigma^k - C0 : eps^k                           eq. (6)
      e^k   = eps_bar - G' * tau^k (mean eps_bar, G'(0) = 0)  eq. (6)
      DS: eps^{k+1} = e^k                                     eq. (9)
      AS: eps^{k+1} = eps^k + 2 (C + C0)^-1 : C0 : (e^k - eps^k)  eq. (16)
    eps^0 = eps_bar (eq. (9)) unless ``eps_init`` is given.
    ``macro_strain`` is in tensor Voigt order (11,22,33,23,13,12).
    """
    phase = np.asarray(phase)
    shape = phase.shape
    lam, mu = lame_from_young(E, nu)
    lam = np.atleast_1d(lam)
    mu = np.atleast_1d(mu)
    if ref is None:
        ref = reference_medium(lam, mu, scheme, beta=beta)
    C = [stiffness_tensor(l, m) for l, m in zip(lam, mu)]
    C0 = stiffness_tensor(ref.lam0, ref.mu0)
    dC = [Cp - C0 for Cp in C]
    eps_bar = voigt_to_tensor(np.asarray(macro_strain, dtype=np.float64))
    if scheme == "AS":
        # (C + C0)^-1 : C0 per phase, through 6x6 Mandel matrices
        P = [tensor_from_mandel(np.linalg.solve(mandel_matrix(Cp + C0), mandel_matrix(C0)))
             for Cp in C]
    if eps_init is None:
        eps = np.broadcast_to(eps_bar[:, :, None, None, None], (3, 3) + shape).copy()
    else:
        eps = np.array(eps_init, dtype=np.float64, copy=True)
    res = SolveResult(0, None, None, None, math.inf)
    N = float(np.prod(shape))
    for k in range(max_iter + 1):
        sigma = apply_phasewise(C, phase, eps)
        eta = equilibrium_norm(op, sigma)
        res.eta_history.append(eta)
        res.mean_stress_history.append(sigma.mean(axis=(2, 3, 4)))
        if keep_iterates:
            res.iterates.append(eps.copy())
        if not np.isfinite(eta):
            res.converged = False
            break
        if eta <= tol or k == max_iter:
            res.converged = eta <= tol
            break
        tau = apply_phasewise(dC, phase, eps)
        tau_hat = forward_dft(tau)
        e_hat = -green_apply(op, ref, tau_hat, shape)
        e_hat[:, :, 0, 0, 0] = N * eps_bar
        e = np.real(inverse_dft(e_hat))
        if scheme == "DS":
            eps = e
        else:
            eps = eps + 2.0 * apply_phasewise(P, phase, e - eps)
    res.iterations = k
    res.eps = eps
    res.sigma = sigma
    res.mean_stress = sigma.mean(axis=(2, 3, 4))
    res.eta = eta
    return res


def solve_cg(phase, E, nu, macro_strain, op="R", tol=1e-10, max_iter=1000, ref: Reference | None = None,
             keep_iterates=False):
    """Conjugate gradients on the discrete Lippmann-Schwinger problem (R8).

    The discrete solution is the strain eps = eps_bar + e, e compatible with
    zero mean, whose stress sigma = C:eps is equilibrated in the sense of
    eq. (19), i.e. G'(C:eps) = 0 at every nonzero frequency.  With
    B(x) = G' * (C:x) (a C0-orthogonal projection composed with C, hence
    self-adjoint and positive in <a, b> = sum_x a : C0 : b on compatible
    fields) the fluctuation solves B(e) = -B(eps_bar).  Iteration k
    (k = 0, 1, ...):
      sigma^k = C:eps^k; eta^k by eq. (43); stop at the first k with
      eta^k <= tol (or k = max_iter);
      r^0 = -B(eps_bar), p^0 = r^0;
      alpha = <r, r> / <p, B(p)>;  e += alpha p;  r -= alpha B(p);
      beta = <r, r>_new / <r, r>_old;  p = r + beta p.
    eps^0 = eps_bar.  The reference medium defaults to eq. (17).
    """
    phase = np.asarray(phase)
    shape = phase.shape
    lam, mu = lame_from_young(E, nu)
    lam = np.atleast_1d(lam)
    mu = np.atleast_1d(mu)
    if ref is None:
        ref = reference_medium(lam, mu, "AS")
    C = [stiffness_tensor(l, m) for l, m in zip(lam, mu)]
    C0 = stiffness_tensor(ref.lam0, ref.mu0)
    eps_bar = voigt_to_tensor(np.asarray(macro_strain, dtype=np.float64))

    def B(x):
        return np.real(inverse_dft(green_apply(op, ref, forward_dft(apply_phasewise(C, phase, x)), shape)))

    def dot(a, b):
        return float(np.sum(a * contract(C0, b)))

    eps = np.broadcast_to(eps_bar[:, :, None, None, None], (3, 3) + shape).copy()
    r = -B(eps)
    p = r.copy()
    rr = dot(r, r)
    res = SolveResult(0, None, None, None, math.inf)
    for k in range(max_iter + 1):
        sigma = apply_phasewise(C, phase, eps)
        eta = equilibrium_norm(op, sigma)
        res.eta_history.append(eta)
        res.mean_stress_history.append(sigma.mean(axis=(2, 3, 4)))
        if keep_iterates:
            res.iterates.append(eps.copy())
        if not np.isfinite(eta):
            res.converged = False
            break
        if eta <= tol or k == max_iter:
            res.converged = eta <= tol
            break
        q = B(p)
        alpha = rr / dot(p, q)
        eps = eps + alpha * p
        r = r - alpha * q
        rr_new = dot(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
    res.iterations = k
    res.eps = eps
    res.sigma = sigma
    res.mean_stress = sigma.mean(axis=(2, 3, 4))
    res.eta = eta
    return res


def effective_stiffness(phase, E, nu, op="R", scheme="AS", tol=1e-10, max_iter=1000, **kw):
    """Six unit macroscopic strains give the effective tensor (§2, eq. (5)),
    as a 6x6 matrix in Voigt notation: column J is <sigma_I> for a normal
    load J (eps_bar_JJ = 1) and <sigma_I>/2 for a shear load J
    (eps_bar_ab = eps_bar_ba = 1, engineering shear 2)."""
    Cv = np.zeros((6, 6))
    its = []
    for J in range(6):
        e = np.zeros(6)
        e[J] = 1.0
        r = solve(phase, E, nu, e, op=op, scheme=scheme, tol=tol, max_iter=max_iter, **kw)
        s = tensor_to_voigt(r.mean_stress)
        Cv[:, J] = s if J < 3 else s / 2.0
        its.append(r.iterations)
    return Cv, its
