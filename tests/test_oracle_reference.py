"""Pins of the oracle's reference medium (§3, eqs. (17) and (18)) through the
convergence of the schemes on a two-phase laminate, where the iteration can
be followed by hand (no GPU).

Laminate whose phase depends on x only, loaded in shear (eps_bar_12 = 1) or
in uniaxial strain (eps_bar_11 = 1), phases with the same Poisson ratio so
that C_p = s_p C0 when C0 follows the paper's rules.  The exact solution is
piecewise constant (``laminate_exact``) and so is every iterate of the
rotated and WP schemes from eps^0 = eps_bar: the error delta^k = eps^k -
eps* takes one value delta_p per phase, and along the loaded component the
schemes reduce to a scalar problem with modulus c (2 mu for shear, lambda +
2 mu for uniaxial strain) and reference c0:

  e - eps = -<delta> + (<c delta> - c delta) / c0          (Green step, 1D)
  DS (eq. (9)):  delta' = delta - (c delta - <c delta>)/c0 - <delta>
  AS (eq. (16)): delta' = r delta + 2 <(c - c0) delta> / (c + c0),
                 r_p = (c0 - c_p)/(c0 + c_p)

with volume fractions f_p.  For DS the zero-mean error (the start eps_bar
has the exact mean) is an eigenvector: delta' = lam delta with
lam = 1 - (f_1 c_2 + f_2 c_1)/c0.  For AS the 2x2 map has trace
r_1 (1 - 2 f_1) + r_2 (1 - 2 f_2) and determinant -r_1 r_2, so by
Cayley-Hamilton delta^(k+2) = tr delta^(k+1) + r_1 r_2 delta^k.  With the
geometric means of eq. (17), r_1 = -r_2 = rho = (sqrt(chi) - 1)/(sqrt(chi) + 1)
(chi the contrast): delta^(k+2) = 2 rho (f_2 - f_1) delta^(k+1) - rho^2 delta^k,
and the error decays as rho^k (complex pair of modulus rho).

The shear load pins mu0, the uniaxial load pins lambda0 + 2 mu0 (hence
kappa0); an arithmetic mean in eq. (17) breaks the AS recurrence (its rate
on this laminate is 0.56 instead of 0.82), a geometric mean in eq. (18)
makes DS diverge, a missing beta changes lam.
"""
import math

import numpy as np
import pytest

import oracle as O
from microstructure import laminate

CHI = 100.0
E = [1.0, CHI]       # phase 0 soft, phase 1 stiff: kappa and mu both in contrast CHI
NU = [0.25, 0.25]
LABELS = np.array([1] * 5 + [0] * 11, dtype=np.uint8)  # 5 stiff, 11 soft layers
F_SOFT, F_STIFF = 11 / 16, 5 / 16
SHAPE = (4, 4, 16)
SHEAR = [0, 0, 0, 0, 0, 1.0]
UNIAXIAL = [1.0, 0, 0, 0, 0, 0]


def _errors(op, scheme, macro, k, ref=None, beta=0.5):
    phase = laminate(SHAPE, LABELS)
    exact = O.laminate_exact(LABELS, E, NU, macro)  # (3, 3, nx)
    r = O.solve(phase, E, NU, macro, op=op, scheme=scheme, tol=1e-300, max_iter=k, ref=ref, beta=beta,
                keep_iterates=True)
    return [it - exact[:, :, None, None, :] for it in r.iterates]


@pytest.mark.parametrize("macro", [SHEAR, UNIAXIAL], ids=["shear", "uniaxial"])
@pytest.mark.parametrize("op", ["R", "W"])
def test_accelerated_scheme_recurrence_on_a_laminate(op, macro):
    """Eq. (17) gives rho = (sqrt(chi) - 1)/(sqrt(chi) + 1) = 9/11 and the
    three-term recurrence holds for every k (to rounding)."""
    rho = (math.sqrt(CHI) - 1.0) / (math.sqrt(CHI) + 1.0)
    a = 2.0 * rho * (F_STIFF - F_SOFT)
    d = _errors(op, "AS", macro, 40)
    for k in range(len(d) - 2):
        res = d[k + 2] - a * d[k + 1] + rho * rho * d[k]
        assert np.linalg.norm(res) <= 1e-9 * np.linalg.norm(d[0]), k
    # the decay rate: |delta^k| ~ rho^k (modulus of the complex pair)
    n = np.array([np.linalg.norm(x) for x in d])
    rate = (n[36] / n[4]) ** (1.0 / 32.0)
    assert abs(rate - rho) < 0.03


def test_arithmetic_mean_breaks_the_accelerated_recurrence():
    """The same recurrence with an arithmetic mean in place of eq. (17): the
    pin above would fail (the plausible slip it guards against)."""
    lam, mu = O.lame_from_young(E, NU)
    kap = lam + 2.0 * mu / 3.0
    k0, m0 = 0.5 * (kap[0] + kap[1]), 0.5 * (mu[0] + mu[1])
    ref = O.Reference(float(k0 - 2.0 * m0 / 3.0), float(m0))
    rho = (math.sqrt(CHI) - 1.0) / (math.sqrt(CHI) + 1.0)
    a = 2.0 * rho * (F_STIFF - F_SOFT)
    d = _errors("R", "AS", SHEAR, 12, ref=ref)
    worst = max(np.linalg.norm(d[k + 2] - a * d[k + 1] + rho * rho * d[k]) / np.linalg.norm(d[0])
                for k in range(len(d) - 2))
    assert worst > 1e-2
    # its decay rate is sqrt(|r_1 r_2|) = 0.56 on this laminate
    n = np.array([np.linalg.norm(x) for x in d])
    assert (n[12] / n[2]) ** 0.1 < 0.7


@pytest.mark.parametrize("macro", [SHEAR, UNIAXIAL], ids=["shear", "uniaxial"])
@pytest.mark.parametrize("beta", [0.5, 0.509])
def test_direct_scheme_ratio_on_a_laminate(macro, beta):
    """Eq. (18): c0 = beta (c_1 + c_2) for both moduli, so every iteration
    multiplies the error by lam = 1 - (f_1 c_2 + f_2 c_1)/(beta (c_1 + c_2)),
    with c_1 = 1 (soft), c_2 = chi in units of the soft phase."""
    lam_k = 1.0 - (F_SOFT * CHI + F_STIFF * 1.0) / (beta * (1.0 + CHI))
    d = _errors("R", "DS", macro, 8, beta=beta)
    for k in range(len(d) - 1):
        assert np.linalg.norm(d[k + 1] - lam_k * d[k]) <= 1e-10 * np.linalg.norm(d[0]), k


def test_geometric_mean_would_make_the_direct_scheme_diverge():
    """With eq. (17)'s geometric mean in the direct scheme the same ratio is
    1 - (f_1 chi + f_2)/sqrt(chi) = -5.9: the scheme diverges, so a swap of
    the two rules cannot pass the direct-scheme pin."""
    lam, mu = O.lame_from_young(E, NU)
    kap = lam + 2.0 * mu / 3.0
    k0, m0 = math.sqrt(kap[0] * kap[1]), math.sqrt(mu[0] * mu[1])
    ref = O.Reference(float(k0 - 2.0 * m0 / 3.0), float(m0))
    d = _errors("R", "DS", SHEAR, 3, ref=ref)
    lam_k = 1.0 - (F_SOFT * CHI + F_STIFF) / math.sqrt(CHI)
    assert np.linalg.norm(d[2] - lam_k * d[1]) <= 1e-10 * np.linalg.norm(d[1])
    assert abs(lam_k) > 1.0
