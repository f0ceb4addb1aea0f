"""The C-ABI library loads and exports every symbol include/fe.h declares;
argument checks that run before any device call (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

import paper_1412_8398_amd as fe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        with open(os.path.join(ROOT, "include", h)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(fe_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fe.library_path()):
        pytest.fail("libfe.so is not built (run `python -m paper_1412_8398_amd.build`)")
    return fe.load_library()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("fe_plan_create", "fe_plan_destroy", "fe_solve", "fe_effective_stiffness",
                 "fe_status_string", "fe_last_error", "fe_solve_batched", "fe_unet_create", "fe_unet_predict",
                 "fe_unet_train_step", "fe_nn_conv3_forward", "fe_nn_conv3_backward_data",
                 "fe_nn_conv3_backward_weight"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), f"libfe.so does not export {name}"


def test_status_strings(lib):
    assert fe.status_string(fe.FE_OK) == "FE_OK"
    assert fe.status_string(fe.FE_ERR_UNSUPPORTED) == "FE_ERR_UNSUPPORTED"
    assert fe.status_string(123) == "FE_UNKNOWN_STATUS"


def _create(lib, nx, ny, nz, disc=2, scheme=1, **kw):
    opt = fe.FePlanOptions()
    lib.fe_plan_options_default(C.byref(opt))
    for k, v in kw.items():
        setattr(opt, k, v)
    h = C.c_void_p()
    s = lib.fe_plan_create(fe.FeGrid(nx, ny, nz), disc, scheme, C.byref(opt), C.byref(h))
    return s, h


@pytest.mark.parametrize("dims,status", [
    ((14, 16, 16), fe.FE_ERR_UNSUPPORTED),   # 14 = 2 * 7
    ((16, 36, 16), fe.FE_ERR_UNSUPPORTED),   # 36 = 4 * 9: only 2^a and 3 * 2^a
    ((16, 15, 16), fe.FE_ERR_UNSUPPORTED),   # odd
    ((2048, 16, 16), fe.FE_ERR_UNSUPPORTED),  # above 1024
    ((2, 16, 16), fe.FE_ERR_UNSUPPORTED),
    ((0, 16, 16), fe.FE_ERR_INVALID_ARG),
    ((-8, 16, 16), fe.FE_ERR_INVALID_ARG),
])
def test_plan_rejects_bad_grids_before_device_work(lib, dims, status):
    s, h = _create(lib, *dims)
    assert s == status
    assert not h.value
    assert "grid dimension" in fe.last_error()


def test_plan_rejects_bad_options(lib):
    assert _create(lib, 16, 16, 16, disc=7)[0] == fe.FE_ERR_INVALID_ARG
    assert _create(lib, 16, 16, 16, scheme=3)[0] == fe.FE_ERR_INVALID_ARG
    assert _create(lib, 16, 16, 16, precision=5)[0] == fe.FE_ERR_INVALID_ARG
    assert _create(lib, 16, 16, 16, check_every=0)[0] == fe.FE_ERR_INVALID_ARG
    assert _create(lib, 16, 16, 16, ref_rule=1, E0=-1.0)[0] == fe.FE_ERR_INVALID_ARG
    assert _create(lib, 16, 16, 16, ref_rule=1, E0=1.0, nu0=0.5)[0] == fe.FE_ERR_INVALID_ARG
    assert _create(lib, 16, 16, 16, scheme=0, ds_beta=0.0)[0] == fe.FE_ERR_INVALID_ARG
    assert _create(lib, 16, 16, 16, struct_size=4)[0] == fe.FE_ERR_INVALID_ARG


def test_solve_rejects_null_plan_and_bad_arguments(lib):
    E = (C.c_double * 2)(1.0, 2.0)
    nu = (C.c_double * 2)(0.3, 0.3)
    m = fe.FeMaterials(2, E, nu)
    macro = (C.c_double * 6)(1, 0, 0, 0, 0, 0)
    r = fe.FeResult()
    assert lib.fe_solve(None, None, m, macro, 1e-6, None, C.byref(r)) == fe.FE_ERR_INVALID_ARG
    assert lib.fe_effective_stiffness(None, None, m, 1e-6, None, None) == fe.FE_ERR_INVALID_ARG


def _batch_desc(dims, n_phases=2):
    grids = (fe.FeGrid * 1)(fe.FeGrid(*dims))
    phase = (C.c_void_p * 1)(0x1000)  # never dereferenced: arguments fail first
    E = (C.c_double * n_phases)(*[1.0 + i for i in range(n_phases)])
    nu = (C.c_double * n_phases)(*[0.3] * n_phases)
    mats = (fe.FeMaterials * 1)(fe.FeMaterials(n_phases, E, nu))
    macro = (C.c_double * 6)(1, 0, 0, 0, 0, 0)
    desc = fe.FeBatchDesc(1, grids, phase, mats, macro, None)
    return desc, (grids, phase, E, nu, mats, macro)


def test_batched_solve_rejects_bad_arguments_before_device_work(lib):
    res = (fe.FeBatchResult * 1)()
    desc, keep = _batch_desc((16, 16, 16))
    call = lambda disc, scheme, d, tol: lib.fe_solve_batched(disc, scheme, None, d, tol, res, None)  # noqa: E731
    assert call(2, 1, None, 1e-6) == fe.FE_ERR_INVALID_ARG
    assert call(0, 1, C.byref(desc), 1e-6) == fe.FE_ERR_UNSUPPORTED  # MS: six-component form only
    assert "WP and ROT" in fe.last_error()
    assert call(7, 1, C.byref(desc), 1e-6) == fe.FE_ERR_INVALID_ARG
    assert call(2, 3, C.byref(desc), 1e-6) == fe.FE_ERR_INVALID_ARG
    assert call(2, 1, C.byref(desc), 0.0) == fe.FE_ERR_INVALID_ARG
    bad, keep2 = _batch_desc((16, 36, 16))
    assert call(2, 1, C.byref(bad), 1e-6) == fe.FE_ERR_UNSUPPORTED
    assert "grid dimension" in fe.last_error()
    empty, keep3 = _batch_desc((16, 16, 16))
    empty.n_samples = 0
    assert call(1, 0, C.byref(empty), 1e-6) == fe.FE_ERR_INVALID_ARG
    nomat, keep4 = _batch_desc((16, 16, 16))
    keep4[4][0].E[0] = -1.0
    assert call(1, 0, C.byref(nomat), 1e-6) == fe.FE_ERR_INVALID_ARG
    opt = fe.FePlanOptions()
    lib.fe_plan_options_default(C.byref(opt))
    assert opt.batch_launch == 0  # FE_BATCH_PER_PASS
    opt.batch_launch = 2
    assert lib.fe_solve_batched(2, 1, C.byref(opt), C.byref(desc), 1e-6, res, None) == fe.FE_ERR_INVALID_ARG
    assert "batch_launch" in fe.last_error()
    opt.batch_launch = 1
    opt.precision = 0  # float64: per-pass launches only
    assert lib.fe_solve_batched(2, 1, C.byref(opt), C.byref(desc), 1e-6, res, None) == fe.FE_ERR_UNSUPPORTED


def test_ctypes_structures_match_the_c_headers(tmp_path):
    """Every structure the binding passes through the ABI has the C layout:
    a C program built against include/*.h prints each size and field offset
    (a field missing in C fails the compile)."""
    import ctypes
    import shutil
    import subprocess

    import paper_1412_8398_amd as fe

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = [(fe.FeGrid, "fe_grid"), (fe.FePlanOptions, "fe_plan_options"), (fe.FeMaterials, "fe_materials"),
             (fe.FeResult, "fe_result"), (fe.FeBatchDesc, "fe_batch_desc"), (fe.FeBatchResult, "fe_batch_result"),
             (fe.FeUnetConfig, "fe_unet_config"), (fe.FeUnetBatch, "fe_unet_batch"),
             (fe.FeNNConvShape, "fe_nn_conv_shape")]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fe.h"', '#include "fe_nn.h"', "int main(void) {"]
    want = []
    for cls, cname in pairs:
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        want.append(ctypes.sizeof(cls))
        for name, _ in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {name}));')
            want.append(getattr(cls, name).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == want


def test_stream_copy_rejects_bad_arguments_before_device_work(lib):
    """Checked on the host before any launch: NULL, sizes that are not whole
    16-byte vectors, misalignment and partial overlap (dst == src is the
    in-place rewrite and allowed; these addresses are never dereferenced)."""
    call = lambda d, s, n: lib.fe_stream_copy(d, s, n, 0, None)  # noqa: E731
    assert call(None, 0x1000, 64) == fe.FE_ERR_INVALID_ARG
    assert call(0x1000, None, 64) == fe.FE_ERR_INVALID_ARG
    assert call(0x2000, 0x1000, 40) == fe.FE_ERR_INVALID_ARG
    assert call(0x2008, 0x1000, 64) == fe.FE_ERR_INVALID_ARG
    assert call(0x1010, 0x1000, 64) == fe.FE_ERR_INVALID_ARG
    assert call(0x1000, 0x1030, 64) == fe.FE_ERR_INVALID_ARG
    assert call(0x2000, 0x1000, 0) == fe.FE_OK
