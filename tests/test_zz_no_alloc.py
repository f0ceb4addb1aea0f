"""fe_solve_static (the solve that allocates nothing: its workspace is a
static device array) against fe_plan_create + fe_solve with the same
options, through the C ABI: bit-identical strain, eta history, mean stress
and iteration count, on two calls in a row (the second on a smaller grid, so
the array holds the first call's contents when the second starts), float32
and float64; and the size limit rejected before any device work."""
import ctypes as C

import numpy as np
import pytest

from microstructure import boolean_spheres

torch = pytest.importorskip("torch")
import paper_1412_8398_amd as fe  # noqa: E402

pytestmark = pytest.mark.gpu

MACRO = [0.3, -0.1, 0.2, 0.05, -0.2, 0.4]
E, NU = [1.0, 20.0], [0.3, 0.25]


def _lib():
    lib = fe.load_library()
    lib.fe_solve_static.argtypes = [fe.FeGrid, C.c_int, C.c_int, C.POINTER(fe.FePlanOptions), C.c_void_p,
                                    fe.FeMaterials, C.POINTER(C.c_double), C.c_double, C.c_void_p,
                                    C.POINTER(fe.FeResult)]
    lib.fe_solve_static.restype = C.c_int
    return lib


def _options(lib, precision, max_iter):
    opt = fe.FePlanOptions()
    lib.fe_plan_options_default(C.byref(opt))
    opt.precision = fe.PRECISION[precision]
    opt.max_iter = max_iter
    opt.refine = 0
    return opt


def _static_solve(lib, L, green, scheme, precision, phase, tol, max_iter, cap):
    dt = torch.float64 if precision == "fp64" else torch.float32
    eps = torch.full((6, L, L, L), float("nan"), dtype=dt, device="cuda")
    hist = np.zeros(cap)
    r = fe.FeResult()
    r.strain = eps.data_ptr()
    r.eta_history = hist.ctypes.data_as(C.POINTER(C.c_double))
    r.history_capacity = cap
    Ea, nua = np.array(E), np.array(NU)
    m = fe.FeMaterials(2, Ea.ctypes.data_as(C.POINTER(C.c_double)), nua.ctypes.data_as(C.POINTER(C.c_double)))
    macro = (C.c_double * 6)(*MACRO)
    opt = _options(lib, precision, max_iter)
    s = lib.fe_solve_static(fe.FeGrid(L, L, L), fe.GREEN[green], fe.SCHEME[scheme], C.byref(opt), phase.data_ptr(),
                            m, macro, tol, None, C.byref(r))
    torch.cuda.synchronize()
    return s, r, eps, hist


def _plan_solve(L, green, scheme, precision, phase, tol, max_iter, cap):
    dt = torch.float64 if precision == "fp64" else torch.float32
    eps = torch.empty((6, L, L, L), dtype=dt, device="cuda")
    with fe.Plan(L, green=green, scheme=scheme, precision=precision, max_iter=max_iter, refine=False) as plan:
        res = plan.solve(phase, E, NU, MACRO, tol, strain=eps, history=cap, raise_on_error=False)
    torch.cuda.synchronize()
    return res, eps


@pytest.mark.parametrize("precision,green,scheme,sizes", [("fp32", "R", "AS", (64, 32)),
                                                          ("fp64", "W", "DS", (48, 24))])
def test_static_solve_equals_plan_solve(precision, green, scheme, sizes):
    lib = _lib()
    tol, max_iter, cap = 1e-5, 400, 401
    for L in sizes:  # the second call is smaller: the array still holds the first one's values
        print(f"fe_solve_static {precision} {green} {scheme} {L}^3", flush=True)
        ph_np, _ = boolean_spheres((L, L, L), 3.0, 0.25, 900 + L)
        phase = torch.from_numpy(ph_np).cuda()
        s, r, eps_s, hist = _static_solve(lib, L, green, scheme, precision, phase, tol, max_iter, cap)
        ref, eps_p = _plan_solve(L, green, scheme, precision, phase, tol, max_iter, cap)
        assert s == ref.status == fe.FE_OK, (s, ref.status, fe.last_error())
        assert r.iterations == ref.iterations
        assert torch.equal(eps_s, eps_p)
        assert np.array_equal(hist[: r.iterations + 1], ref.eta_history)
        assert list(r.mean_stress) == list(ref.mean_stress)
        assert r.eta == ref.eta and r.eta_verify_fp64 == ref.eta_verify_fp64
        assert r.eta_verify_fp64 <= 1.5 * tol


def test_static_solve_rejects_grids_beyond_the_array():
    lib = _lib()
    L = 128  # float32 needs about 126 MiB of workspace, the array holds 64 MiB
    phase = torch.zeros((L, L, L), dtype=torch.uint8, device="cuda")
    s, r, eps, _ = _static_solve(lib, L, "R", "AS", "fp32", phase, 1e-6, 10, 1)
    assert s == fe.FE_ERR_UNSUPPORTED
    assert "static scratch" in fe.last_error()
    assert torch.isnan(eps).all()  # nothing was written
    s, *_ = _static_solve(lib, 16, "MS", "AS", "fp32", torch.zeros((16, 16, 16), dtype=torch.uint8, device="cuda"),
                          1e-6, 10, 1)
    assert s == fe.FE_ERR_UNSUPPORTED
