"""Reference-medium study (§6.1) on the GPU: the iteration counts N(E0) that
the descent compares are the oracle's, for explicit (E0, nu0) reference media
on a small sample of the paper's Boolean medium (float64, tol 1e-8)."""
import numpy as np
import pytest

import oracle as O
from microstructure import boolean_spheres

torch = pytest.importorskip("torch")
from paper_1412_8398_amd.refscan import E1, MACRO, NU, Counter  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("op,E0", [("R", 0.3), ("R", 0.9), ("W", 0.5), ("C", 0.4)])
def test_iteration_count_matches_the_oracle(op, E0):
    phase, _ = boolean_spheres((16, 16, 16), 2.5, 0.17, 7)
    chi = 0.1
    E, nu = [E1, chi * E1], [NU, NU]
    ref = O.solve(phase, E, nu, MACRO, op=op, scheme="AS", tol=1e-8, max_iter=3000,
                  ref=O.reference_medium(None, None, "AS", E0=E0, nu0=NU))
    cnt = Counter(torch.from_numpy(phase).cuda(), chi, op, "AS", tol=1e-8, cap=3000)
    n, eta = cnt(E0)
    print(op, E0, n, ref.iterations, eta, flush=True)
    assert n == ref.iterations
    assert np.isclose(eta, ref.eta_history[-1], rtol=1e-8, atol=1e-15)
