"""FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_1412_8398_amd``) and never imports it; the GPU path never
imports this package.

Parity status per function (what pins it, see tests/test_oracle_*.py):
  forward_dft / inverse_dft   brute-force DFT of eq. (11) on 8^3 and 6x4x10 grids
  wave_vector                 eq. (36) typed literally (R); real-space stencils
                              of eqs. (23), (37), (38) via their Fourier symbols
  green_apply                 closed form eq. (8) (MS), corrected eq. (39)
                              (C, W, R), symmetries eqs. (26), (27), (34),
                              projection properties, q -> 0 limit
  special_modes               eqs. (14), (29), (41) by construction + rank tests
  reference_medium            eqs. (17), (18) through the exact error recurrence
                              of AS and the exact error ratio of DS on a
                              two-phase laminate (shear pins mu0, uniaxial
                              strain pins lambda0 + 2 mu0)
  equilibrium_norm            real-space divergence stencils (Parseval)
  solve (DS, AS)              homogeneous one-step, laminate closed form,
                              direct finite-difference solve on tiny grids
                              (W, R), DS == AS fixed point
  solve_cg (R8)               ends at the accelerated scheme's solution (all
                              four operators), laminate closed form (W, R),
                              homogeneous start, strain energy decreasing and
                              C0-orthogonal residuals at every step
  laminate_exact              the oracle's own iterative solve on laminates
                              (R, W any thickness; MS, C even thickness),
                              and traction/compatibility checks
  effective_stiffness         Voigt/Reuss bounds, laminate closed form,
                              the paper's printed limit 1.208 (weak pin)
  unet (warm-start network, not part of the paper)
    conv3                     direct loop sum, FFT circular correlation
    conv3_backward            adjoint identities
    pool / up                 adjoint identities, values
    loss_and_grad             central finite differences of every tensor
    adam_step                 closed-form bias-corrected first step
No function is left unpinned.
"""
from .homogenization import *  # noqa: F401,F403
from .homogenization import (  # noqa: F401
    OPERATORS, SCHEMES, Reference, SolveResult, solve, solve_cg, effective_stiffness,
    reference_medium, green_apply, green_tensor_at, wave_vector, special_modes,
    equilibrium_norm, forward_dft, inverse_dft, brute_force_dft,
    voigt_to_tensor, tensor_to_voigt, stiffness_tensor, lame_from_young,
    green_continuous_closed_form, green3_closed_form, wave_vector_r_literal,
    signed_modes, mandel_matrix, compliance_apply, laminate_exact,
)
