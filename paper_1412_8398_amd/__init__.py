"""Python binding of ``libfe.so``: argument marshalling only.

Every step of the solve runs in the library's HIP kernels; PyTorch tensors
serve as device memory.  The binding raises if the library is not built --
there is no CPU fallback.

The C ABI is declared in ``include/fe.h``; names mirror it.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "FE_OK", "FE_NOT_CONVERGED", "FE_DIVERGED", "FE_ERR_INVALID_ARG", "FE_ERR_UNSUPPORTED",
    "FE_ERR_OOM", "FE_ERR_DEVICE", "GREEN", "SCHEME", "PRECISION", "FeError", "Plan", "Result",
    "load_library", "library_path", "status_string", "last_error", "BatchSampleSpec", "solve_batched",
    "UNet", "stream_copy", "conv3_forward", "conv3_backward_data", "conv3_backward_weight",
]

FE_OK, FE_NOT_CONVERGED, FE_DIVERGED = 0, 1, 2
FE_ERR_INVALID_ARG, FE_ERR_UNSUPPORTED, FE_ERR_OOM, FE_ERR_DEVICE = -1, -2, -3, -4

GREEN = {"MS": 0, "WP": 1, "W": 1, "ROT": 2, "R": 2, "C": 3, "CENTERED": 3, "MSS": 4, "MS_SYMMETRIZED": 4}
SCHEME = {"DS": 0, "direct": 0, "AS": 1, "accelerated": 1, "CG": 2, "conjugate_gradient": 2}
PRECISION = {"fp64": 0, "fp32": 1}
REF_RULE = {"paper": 0, "explicit": 1}
PASSES = ("pointwise", "zfwd", "yfwd", "xgreen", "yinv", "zinv", "update", "eta")

_PKG = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.environ.get("FE_LIBRARY", os.path.join(_PKG, "libfe.so"))


class FeGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32)]


class FePlanOptions(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("precision", C.c_int),
        ("max_iter", C.c_int32),
        ("ref_rule", C.c_int32),
        ("ds_beta", C.c_double),
        ("E0", C.c_double),
        ("nu0", C.c_double),
        ("check_every", C.c_int32),
        ("diverge_window", C.c_int32),
        ("timing", C.c_int32),
        ("refine", C.c_int32),
        ("hip_stream", C.c_void_p),
        ("batch_launch", C.c_int32),
    ]


BATCH_LAUNCH = {"per_pass": 0, "persistent": 1}


class FeMaterials(C.Structure):
    _fields_ = [("n_phases", C.c_int32), ("E", C.POINTER(C.c_double)), ("nu", C.POINTER(C.c_double))]


class FeResult(C.Structure):
    _fields_ = [
        ("strain", C.c_void_p),
        ("stress", C.c_void_p),
        ("eta_history", C.POINTER(C.c_double)),
        ("history_capacity", C.c_int32),
        ("mean_stress", C.c_double * 6),
        ("eta", C.c_double),
        ("eta_verify_fp64", C.c_double),
        ("iterations", C.c_int32),
        ("seconds", C.c_double),
        ("pass_seconds", C.c_double * 8),
        ("pass_launches", C.c_int32 * 8),
        ("refinements", C.c_int32),
        ("mean_stress_history", C.POINTER(C.c_double)),
    ]


_LIB = None


class FeBatchDesc(C.Structure):
    _fields_ = [("n_samples", C.c_int32), ("grids", C.POINTER(FeGrid)), ("phase", C.POINTER(C.c_void_p)),
                ("materials", C.POINTER(FeMaterials)), ("macro_strain", C.POINTER(C.c_double)),
                ("strain", C.POINTER(C.c_void_p))]


class FeBatchResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("eta", C.c_double),
                ("eta_verify_fp64", C.c_double), ("mean_stress", C.c_double * 6)]


def load_library():
    """Load libfe.so; raise if it has not been built (no fallback path)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: build it with "
                           "`python -m paper_1412_8398_amd.build`")
    lib = C.CDLL(path)
    lib.fe_plan_options_default.argtypes = [C.POINTER(FePlanOptions)]
    lib.fe_plan_options_default.restype = None
    lib.fe_plan_create.argtypes = [FeGrid, C.c_int, C.c_int, C.POINTER(FePlanOptions), C.POINTER(C.c_void_p)]
    lib.fe_plan_create.restype = C.c_int
    lib.fe_plan_destroy.argtypes = [C.c_void_p]
    lib.fe_plan_destroy.restype = None
    lib.fe_plan_workspace_bytes.argtypes = [C.c_void_p]
    lib.fe_plan_workspace_bytes.restype = C.c_size_t
    lib.fe_solve.argtypes = [C.c_void_p, C.c_void_p, FeMaterials, C.POINTER(C.c_double), C.c_double, C.c_void_p,
                             C.POINTER(FeResult)]
    lib.fe_solve.restype = C.c_int
    lib.fe_effective_stiffness.argtypes = [C.c_void_p, C.c_void_p, FeMaterials, C.c_double,
                                           C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    lib.fe_effective_stiffness.restype = C.c_int
    lib.fe_solve_batched.argtypes = [C.c_int, C.c_int, C.POINTER(FePlanOptions), C.POINTER(FeBatchDesc), C.c_double,
                                     C.POINTER(FeBatchResult), C.POINTER(C.c_double)]
    lib.fe_solve_batched.restype = C.c_int
    lib.fe_stream_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p]
    lib.fe_stream_copy.restype = C.c_int
    lib.fe_status_string.argtypes = [C.c_int]
    lib.fe_status_string.restype = C.c_char_p
    lib.fe_last_error.argtypes = []
    lib.fe_last_error.restype = C.c_char_p
    _LIB = lib
    return lib


def status_string(s: int) -> str:
    return load_library().fe_status_string(s).decode()


def last_error() -> str:
    return load_library().fe_last_error().decode()


class FeError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}: {last_error()}")


def _ptr(x) -> int | None:
    """Device address of a tensor already checked by ``_checked``; None for None."""
    return None if x is None else x.data_ptr()


def _checked(x, name, dtypes, shape, required=False):
    """Check a tensor handed to the library: dtype (one of ``dtypes``), exact
    shape and contiguity.  The library takes no sizes, so a mismatch here
    would make its kernels read or write out of bounds.  Every tensor of a
    call is checked before any is placed (``_addresses``) and before the
    library is called."""
    if x is None:
        if required:
            raise ValueError(f"{name} is required")
        return None
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(x).__name__}")
    dtypes = dtypes if isinstance(dtypes, tuple) else (dtypes,)
    if x.dtype not in dtypes:
        raise ValueError(f"{name}: dtype {x.dtype}, expected {' or '.join(str(d) for d in dtypes)}")
    if tuple(x.shape) != tuple(int(v) for v in shape):
        raise ValueError(f"{name}: shape {tuple(x.shape)}, expected {tuple(shape)}")
    if not x.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    return x


def _addresses(named, device=None):
    """Device addresses of checked tensors given as (name, tensor) pairs (None
    stays None); all must live on the GPU, on ``device`` if given, else on
    the device of the first one."""
    out = []
    for name, x in named:
        if x is None:
            out.append(None)
            continue
        if not x.is_cuda:
            raise ValueError(f"{name}: expected a device (cuda) tensor")
        if device is None:
            device = x.device.index
        elif x.device.index != device:
            raise ValueError(f"{name}: on cuda:{x.device.index}, expected cuda:{device}")
        out.append(x.data_ptr())
    return out


def _current_device():
    import torch
    return torch.cuda.current_device()


def _field_dtype(precision):
    import torch
    return torch.float64 if precision == "fp64" else torch.float32


def _materials(E, nu):
    E = np.ascontiguousarray(np.atleast_1d(np.asarray(E, dtype=np.float64)))
    nu = np.ascontiguousarray(np.atleast_1d(np.asarray(nu, dtype=np.float64)))
    if E.shape != nu.shape:
        raise ValueError("E and nu must have the same length")
    m = FeMaterials(int(E.size), E.ctypes.data_as(C.POINTER(C.c_double)), nu.ctypes.data_as(C.POINTER(C.c_double)))
    return m, (E, nu)  # keep the arrays alive


@dataclass
class Result:
    status: int
    iterations: int
    eta: float
    eta_verify_fp64: float
    mean_stress: np.ndarray
    seconds: float
    eta_history: np.ndarray = field(default=None, repr=False)
    mean_stress_history: np.ndarray = field(default=None, repr=False)  # (k, 6)
    pass_seconds: dict = field(default=None, repr=False)
    pass_launches: dict = field(default=None, repr=False)
    refinements: int = 0

    @property
    def converged(self) -> bool:
        return self.status == FE_OK


class Plan:
    """A solver plan for one grid, Green operator and scheme (fe_plan_create)."""

    def __init__(self, grid, green="R", scheme="AS", precision="fp32", max_iter=1000, ref_rule="paper",
                 ds_beta=0.5, E0=0.0, nu0=0.25, check_every=1, diverge_window=50, timing=False, refine=True,
                 stream=None):
        lib = load_library()
        nx, ny, nz = (grid, grid, grid) if isinstance(grid, int) else tuple(grid)
        self.shape = (nz, ny, nx)
        self.precision = precision
        opt = FePlanOptions()
        lib.fe_plan_options_default(C.byref(opt))
        opt.precision = PRECISION[precision]
        opt.max_iter = int(max_iter)
        opt.ref_rule = REF_RULE[ref_rule]
        opt.ds_beta = float(ds_beta)
        opt.E0 = float(E0)
        opt.nu0 = float(nu0)
        opt.check_every = int(check_every)
        opt.diverge_window = int(diverge_window)
        opt.timing = 1 if timing else 0
        opt.refine = 1 if refine else 0
        opt.hip_stream = stream
        h = C.c_void_p()
        s = lib.fe_plan_create(FeGrid(nx, ny, nz), GREEN[green], SCHEME[scheme], C.byref(opt), C.byref(h))
        if s != FE_OK:
            raise FeError(s, "fe_plan_create")
        self._h = h
        self._lib = lib
        self.device = _current_device()

    @property
    def n(self) -> int:
        nz, ny, nx = self.shape
        return nx * ny * nz

    @property
    def workspace_bytes(self) -> int:
        return int(self._lib.fe_plan_workspace_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fe_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def solve(self, phase, E, nu, macro_strain, tol, strain_init=None, strain=None, stress=None, history=0,
              raise_on_error=True, mean_history=False) -> Result:
        """fe_solve.  ``phase`` is a device uint8 tensor of the grid's shape;
        ``strain``/``stress`` optional device tensors (6, nz, ny, nx) of the
        plan precision that receive eps^n and sigma^n; ``history`` entries of
        eta^k (and of <sigma^k> with ``mean_history``)."""
        dt = _field_dtype(self.precision)
        fshape = (6,) + self.shape
        named = [("phase", _checked(phase, "phase", _uint8(), self.shape, required=True)),
                 ("strain", _checked(strain, "strain", dt, fshape)),
                 ("stress", _checked(stress, "stress", dt, fshape)),
                 ("strain_init", _checked(strain_init, "strain_init", dt, fshape))]
        mv = [float(v) for v in macro_strain]
        if len(mv) != 6:
            raise ValueError("macro_strain needs 6 components")
        p_phase, p_strain, p_stress, p_init = _addresses(named, self.device)
        m, keep = _materials(E, nu)
        macro = (C.c_double * 6)(*mv)
        r = FeResult()
        r.strain = p_strain
        r.stress = p_stress
        hist = None
        if history:
            hist = np.zeros(int(history), dtype=np.float64)
            r.eta_history = hist.ctypes.data_as(C.POINTER(C.c_double))
            r.history_capacity = int(history)
        mhist = None
        if history and mean_history:
            mhist = np.zeros((int(history), 6), dtype=np.float64)
            r.mean_stress_history = mhist.ctypes.data_as(C.POINTER(C.c_double))
        s = self._lib.fe_solve(self._h, p_phase, m, macro, float(tol), p_init, C.byref(r))
        if s < 0 and raise_on_error:
            raise FeError(s, "fe_solve")
        del keep
        res = Result(s, r.iterations, r.eta, r.eta_verify_fp64, np.array(r.mean_stress[:]), r.seconds)
        res.pass_seconds = {n: float(r.pass_seconds[i]) for i, n in enumerate(PASSES)}
        res.pass_launches = {n: int(r.pass_launches[i]) for i, n in enumerate(PASSES)}
        res.refinements = int(r.refinements)
        if hist is not None:
            res.eta_history = hist[: min(len(hist), r.iterations + 1)]
        if mhist is not None:
            res.mean_stress_history = mhist[: min(len(mhist), r.iterations + 1)]
        return res

    def effective_stiffness(self, phase, E, nu, tol):
        """fe_effective_stiffness: 6x6 Voigt matrix and the six iteration counts."""
        (p_phase,) = _addresses([("phase", _checked(phase, "phase", _uint8(), self.shape, required=True))],
                                self.device)
        m, keep = _materials(E, nu)
        Cv = (C.c_double * 36)()
        its = (C.c_int32 * 6)()
        s = self._lib.fe_effective_stiffness(self._h, p_phase, m, float(tol), Cv, its)
        if s < 0:
            raise FeError(s, "fe_effective_stiffness")
        del keep
        return np.array(Cv[:]).reshape(6, 6), list(its), s


def stream_copy(dst, src, nontemporal=False, stream=None):
    """fe_stream_copy between two device tensors of the same byte size (the
    measurement reference for attainable HBM bandwidth); ``dst is src``
    rewrites the tensor in place."""
    import torch
    for name, t in (("dst", dst), ("src", src)):
        if not isinstance(t, torch.Tensor) or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous tensor")
    nbytes = dst.numel() * dst.element_size()
    if src.numel() * src.element_size() != nbytes:
        raise ValueError("dst and src differ in size")
    pd, ps = _addresses([("dst", dst), ("src", src)])
    s = load_library().fe_stream_copy(pd, ps, nbytes, 1 if nontemporal else 0, stream)
    if s != FE_OK:
        raise FeError(s, "fe_stream_copy")


@dataclass
class BatchSampleSpec:
    """One sample of a batched solve: a device uint8 phase map (nz, ny, nx),
    its phases' moduli and the applied macroscopic strain; ``strain`` (optional)
    is a device tensor (6, nz, ny, nx) of the solve precision receiving eps^n."""
    phase: object
    E: object
    nu: object
    macro_strain: object
    strain: object = None


def _options(lib, precision, max_iter, ref_rule, ds_beta, E0, nu0, diverge_window, stream, refine=True):
    opt = FePlanOptions()
    lib.fe_plan_options_default(C.byref(opt))
    opt.refine = 1 if refine else 0
    opt.precision = PRECISION[precision]
    opt.max_iter = int(max_iter)
    opt.ref_rule = REF_RULE[ref_rule]
    opt.ds_beta = float(ds_beta)
    opt.E0 = float(E0)
    opt.nu0 = float(nu0)
    opt.diverge_window = int(diverge_window)
    opt.hip_stream = stream
    return opt


def solve_batched(samples, tol, green="R", scheme="AS", precision="fp32", max_iter=1000, ref_rule="paper",
                  ds_beta=0.5, E0=0.0, nu0=0.25, diverge_window=50, stream=None, raise_on_error=True, refine=True,
                  launch="per_pass"):
    """fe_solve_batched over a list of BatchSampleSpec; returns (results, status,
    seconds) with one Result per sample (eta_history, pass timings empty).
    ``refine``: float32 samples whose strain does not verify to tol continue
    in float64 (fe_plan_options.refine).  ``launch``: "per_pass" or
    "persistent" (fe_plan_options.batch_launch)."""
    if launch not in BATCH_LAUNCH:
        raise ValueError(f"launch must be one of {sorted(BATCH_LAUNCH)}")
    lib = load_library()
    n = len(samples)
    if n == 0:
        raise ValueError("no samples")
    grids = (FeGrid * n)()
    phases = (C.c_void_p * n)()
    mats = (FeMaterials * n)()
    macro = (C.c_double * (6 * n))()
    strains = (C.c_void_p * n)()
    keep = []
    dt = _field_dtype(precision)
    named = []
    for i, sp in enumerate(samples):
        if getattr(sp.phase, "ndim", None) != 3:
            raise ValueError(f"sample {i}: phase must be a 3D (nz, ny, nx) tensor")
        nz, ny, nx = (int(v) for v in sp.phase.shape)
        named.append((f"sample {i}: phase", _checked(sp.phase, f"sample {i}: phase", _uint8(), (nz, ny, nx),
                                                     required=True)))
        named.append((f"sample {i}: strain", _checked(sp.strain, f"sample {i}: strain", dt, (6, nz, ny, nx))))
    addr = _addresses(named)
    for i, sp in enumerate(samples):
        nz, ny, nx = (int(v) for v in sp.phase.shape)
        grids[i] = FeGrid(nx, ny, nz)
        phases[i] = addr[2 * i]
        strains[i] = addr[2 * i + 1]
        m, k = _materials(sp.E, sp.nu)
        keep.append(k)
        mats[i] = m
        mv = [float(v) for v in sp.macro_strain]
        if len(mv) != 6:
            raise ValueError("macro_strain needs 6 components")
        for q in range(6):
            macro[6 * i + q] = mv[q]
    desc = FeBatchDesc(n, grids, phases, mats, macro, strains)
    opt = _options(lib, precision, max_iter, ref_rule, ds_beta, E0, nu0, diverge_window, stream, refine)
    opt.batch_launch = BATCH_LAUNCH[launch]
    res = (FeBatchResult * n)()
    sec = C.c_double(0.0)
    s = lib.fe_solve_batched(GREEN[green], SCHEME[scheme], C.byref(opt), C.byref(desc), float(tol), res,
                             C.byref(sec))
    if s < 0 and raise_on_error:
        raise FeError(s, "fe_solve_batched")
    del keep
    out = [Result(r.status, r.iterations, r.eta, r.eta_verify_fp64, np.array(r.mean_stress[:]), sec.value)
           for r in res] if s >= 0 else []
    return out, s, sec.value


# ---------------------------------------------------------------------------
# warm-start U-Net (include/fe_nn.h)
# ---------------------------------------------------------------------------
class FeUnetConfig(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("seed", C.c_uint64), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("adam_eps", C.c_float), ("hip_stream", C.c_void_p)]


class FeUnetBatch(C.Structure):
    _fields_ = [("grid", FeGrid), ("batch", C.c_int32), ("phase", C.c_void_p), ("materials", C.POINTER(FeMaterials)),
                ("macro_strain", C.POINTER(C.c_double))]


class FeNNConvShape(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("batch", C.c_int32), ("c_in", C.c_int32),
                ("c_out", C.c_int32)]


_NN_BOUND = False


def _bind_nn(lib):
    global _NN_BOUND
    if _NN_BOUND:
        return lib
    P = C.c_void_p
    lib.fe_unet_config_default.argtypes = [C.POINTER(FeUnetConfig)]
    lib.fe_unet_config_default.restype = None
    lib.fe_unet_create.argtypes = [C.POINTER(FeUnetConfig), C.POINTER(P)]
    lib.fe_unet_create.restype = C.c_int
    lib.fe_unet_destroy.argtypes = [P]
    lib.fe_unet_destroy.restype = None
    lib.fe_unet_param_count.argtypes = []
    lib.fe_unet_param_count.restype = C.c_int64
    for f in ("fe_unet_get_params", "fe_unet_get_grads"):
        getattr(lib, f).argtypes = [P, C.POINTER(C.c_float)]
        getattr(lib, f).restype = C.c_int
    lib.fe_unet_set_learning_rate.argtypes = [P, C.c_float]
    lib.fe_unet_set_learning_rate.restype = C.c_int
    lib.fe_unet_set_params.argtypes = [P, C.POINTER(C.c_float)]
    lib.fe_unet_set_params.restype = C.c_int
    lib.fe_unet_predict.argtypes = [P, C.POINTER(FeUnetBatch), P, C.POINTER(C.c_double)]
    lib.fe_unet_predict.restype = C.c_int
    for f in ("fe_unet_loss_grad", "fe_unet_train_step"):
        getattr(lib, f).argtypes = [P, C.POINTER(FeUnetBatch), P, C.c_int32, C.POINTER(C.c_double)]
        getattr(lib, f).restype = C.c_int
    lib.fe_nn_conv3_forward.argtypes = [C.POINTER(FeNNConvShape), P, P, P, C.c_int32, P, P]
    lib.fe_nn_conv3_forward.restype = C.c_int
    lib.fe_nn_conv3_forward_cat.argtypes = [C.POINTER(FeNNConvShape), C.c_int32, P, P, P, P, C.c_int32, P, P]
    lib.fe_nn_conv3_forward_cat.restype = C.c_int
    lib.fe_nn_conv3_backward_data.argtypes = [C.POINTER(FeNNConvShape), P, P, P, P, P]
    lib.fe_nn_conv3_backward_data.restype = C.c_int
    lib.fe_nn_conv3_backward_weight.argtypes = [C.POINTER(FeNNConvShape), P, P, P, P, P, P]
    lib.fe_nn_conv3_backward_weight.restype = C.c_int
    _NN_BOUND = True
    return lib


def _check(s, where):
    if s < 0 or s == FE_DIVERGED:
        raise FeError(s, where)
    return s


def _shape(x, c_in, c_out):
    B, nz, ny, nx = (int(v) for v in x.shape[:4])
    return FeNNConvShape(nx, ny, nz, B, int(c_in), int(c_out))


def _uint8():
    import torch
    return torch.uint8


def _act5(x, name):
    """A channel-last activation (B, nz, ny, nx, C) in bfloat16: its leading
    shape and channel count (checked for rank and dtype)."""
    import torch
    if not isinstance(x, torch.Tensor) or x.ndim != 5:
        raise ValueError(f"{name}: expected a (B, nz, ny, nx, C) tensor")
    if x.dtype != torch.bfloat16:
        raise ValueError(f"{name}: dtype {x.dtype}, expected torch.bfloat16")
    return tuple(int(v) for v in x.shape[:4]), int(x.shape[4])


def _weights(w):
    import torch
    if not isinstance(w, torch.Tensor) or w.ndim != 3 or int(w.shape[0]) != 27:
        raise ValueError("w: expected a (27, c_in, c_out) tensor")
    return int(w.shape[1]), int(w.shape[2])


def conv3_forward(x, w, b=None, relu=True, stream=None):
    """fe_nn_conv3_forward on device tensors: x (B, nz, ny, nx, c_in) bfloat16,
    w (27, c_in, c_out) float32, b (c_out,) float32 -> y bfloat16."""
    import torch
    lead, c = _act5(x, "x")
    c_in, c_out = _weights(w)
    px, pw, pb = _addresses([("x", _checked(x, "x", torch.bfloat16, lead + (c_in,), required=True)),
                             ("w", _checked(w, "w", torch.float32, (27, c_in, c_out), required=True)),
                             ("b", _checked(b, "b", torch.float32, (c_out,)))])
    lib = _bind_nn(load_library())
    y = torch.empty(lead + (c_out,), dtype=torch.bfloat16, device=x.device)
    _check(lib.fe_nn_conv3_forward(C.byref(_shape(x, c_in, c_out)), px, pw, pb, 1 if relu else 0, _ptr(y), stream),
           "fe_nn_conv3_forward")
    return y


def conv3_forward_cat(coarse, skip, w, b=None, relu=True, stream=None):
    """fe_nn_conv3_forward_cat: conv3 of [nearest upsampling of coarse, skip]
    read in place; coarse (B, nz/2, ny/2, nx/2, c_coarse) and skip
    (B, nz, ny, nx, c_in - c_coarse) bfloat16 -> y (B, nz, ny, nx, c_out)."""
    import torch
    lead, c_skip = _act5(skip, "skip")
    c_in, c_out = _weights(w)
    c_coarse = c_in - c_skip
    B, nz, ny, nx = lead
    shp = (B, nz // 2, ny // 2, nx // 2, c_coarse)
    pc, ps, pw, pb = _addresses([("coarse", _checked(coarse, "coarse", torch.bfloat16, shp, required=True)),
                                 ("skip", _checked(skip, "skip", torch.bfloat16, lead + (c_skip,), required=True)),
                                 ("w", _checked(w, "w", torch.float32, (27, c_in, c_out), required=True)),
                                 ("b", _checked(b, "b", torch.float32, (c_out,)))])
    lib = _bind_nn(load_library())
    y = torch.empty(lead + (c_out,), dtype=torch.bfloat16, device=skip.device)
    _check(lib.fe_nn_conv3_forward_cat(C.byref(_shape(skip, c_in, c_out)), c_coarse, pc, ps, pw, pb,
                                       1 if relu else 0, _ptr(y), stream), "fe_nn_conv3_forward_cat")
    return y


def conv3_backward_data(dy, w, y_mask=None, stream=None):
    import torch
    lead, _ = _act5(dy, "dy")
    c_in, c_out = _weights(w)
    pdy, pm, pw = _addresses([("dy", _checked(dy, "dy", torch.bfloat16, lead + (c_out,), required=True)),
                              ("y_mask", _checked(y_mask, "y_mask", torch.bfloat16, lead + (c_out,))),
                              ("w", _checked(w, "w", torch.float32, (27, c_in, c_out), required=True))])
    lib = _bind_nn(load_library())
    dx = torch.empty(lead + (c_in,), dtype=torch.bfloat16, device=dy.device)
    _check(lib.fe_nn_conv3_backward_data(C.byref(_shape(dy, c_in, c_out)), pdy, pm, pw, _ptr(dx), stream),
           "fe_nn_conv3_backward_data")
    return dx


def conv3_backward_weight(x, dy, y_mask=None, stream=None):
    import torch
    lead, c_in = _act5(x, "x")
    _, c_out = _act5(dy, "dy")
    px, pdy, pm = _addresses([("x", _checked(x, "x", torch.bfloat16, lead + (c_in,), required=True)),
                              ("dy", _checked(dy, "dy", torch.bfloat16, lead + (c_out,), required=True)),
                              ("y_mask", _checked(y_mask, "y_mask", torch.bfloat16, lead + (c_out,)))])
    lib = _bind_nn(load_library())
    dw = torch.empty((27, c_in, c_out), dtype=torch.float32, device=x.device)
    db = torch.empty((c_out,), dtype=torch.float32, device=x.device)
    _check(lib.fe_nn_conv3_backward_weight(C.byref(_shape(x, c_in, c_out)), px, pdy, pm, _ptr(dw), _ptr(db), stream),
           "fe_nn_conv3_backward_weight")
    return dw, db


class UNet:
    """The warm-start network (fe_unet_*): predict, loss/gradient, Adam steps."""

    def __init__(self, seed=1412839801, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8, stream=None):
        lib = _bind_nn(load_library())
        cfg = FeUnetConfig()
        lib.fe_unet_config_default(C.byref(cfg))
        cfg.seed = int(seed)
        cfg.lr, cfg.beta1, cfg.beta2, cfg.adam_eps = float(lr), float(beta1), float(beta2), float(adam_eps)
        cfg.hip_stream = stream
        h = C.c_void_p()
        _check(lib.fe_unet_create(C.byref(cfg), C.byref(h)), "fe_unet_create")
        self._h, self._lib = h, lib
        self.n_params = int(lib.fe_unet_param_count())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fe_unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_learning_rate(self, lr):
        _check(self._lib.fe_unet_set_learning_rate(self._h, float(lr)), "fe_unet_set_learning_rate")

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        _check(self._lib.fe_unet_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float))), "fe_unet_get_params")
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        if p.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {p.size}")
        _check(self._lib.fe_unet_set_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float))), "fe_unet_set_params")

    def get_grads(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        _check(self._lib.fe_unet_get_grads(self._h, out.ctypes.data_as(C.POINTER(C.c_float))), "fe_unet_get_grads")
        return out

    @staticmethod
    def _batch(phase, E, nu, macro):
        """phase: device uint8 (B, nz, ny, nx); E, nu: per-sample phase tables; macro (B, 6)."""
        if getattr(phase, "ndim", None) != 4:
            raise ValueError("phase: expected a (B, nz, ny, nx) tensor")
        B, nz, ny, nx = (int(v) for v in phase.shape)
        _checked(phase, "phase", _uint8(), (B, nz, ny, nx), required=True)
        if len(E) != B or len(nu) != B:
            raise ValueError(f"E and nu need one phase table per sample ({B})")
        mats = (FeMaterials * B)()
        keep = []
        for s in range(B):
            m, k = _materials(E[s], nu[s])
            mats[s] = m
            keep.append(k)
        mac = np.ascontiguousarray(np.asarray(macro, dtype=np.float64).reshape(B, 6))
        keep.append(mac)
        b = FeUnetBatch(FeGrid(nx, ny, nz), B, None, mats, mac.ctypes.data_as(C.POINTER(C.c_double)))
        keep.append(mats)
        return b, keep

    def predict(self, phase, E, nu, macro, out=None):
        """Predicted strain, device float32 (B, 6, nz, ny, nx); returns (out, seconds)."""
        import torch
        b, keep = self._batch(phase, E, nu, macro)
        shape = (b.batch, 6) + tuple(int(v) for v in phase.shape[1:])
        _checked(out, "out", torch.float32, shape)
        b.phase, _ = _addresses([("phase", phase), ("out", out)])
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=phase.device)
        pout = out.data_ptr()
        sec = C.c_double(0.0)
        _check(self._lib.fe_unet_predict(self._h, C.byref(b), pout, C.byref(sec)), "fe_unet_predict")
        del keep
        return out, sec.value

    def _target(self, b, phase, target):
        import torch
        shape = (int(phase.shape[0]), 6) + tuple(int(v) for v in phase.shape[1:])
        _checked(target, "target", (torch.float32, torch.bfloat16), shape, required=True)
        b.phase, pt = _addresses([("phase", phase), ("target", target)])
        return pt, 1 if target.dtype == torch.bfloat16 else 0

    def loss_grad(self, phase, E, nu, macro, target):
        b, keep = self._batch(phase, E, nu, macro)
        pt, is_bf16 = self._target(b, phase, target)
        loss = C.c_double(0.0)
        _check(self._lib.fe_unet_loss_grad(self._h, C.byref(b), pt, is_bf16, C.byref(loss)), "fe_unet_loss_grad")
        del keep
        return loss.value

    def train_step(self, phase, E, nu, macro, target):
        b, keep = self._batch(phase, E, nu, macro)
        pt, is_bf16 = self._target(b, phase, target)
        loss = C.c_double(0.0)
        _check(self._lib.fe_unet_train_step(self._h, C.byref(b), pt, is_bf16, C.byref(loss)), "fe_unet_train_step")
        del keep
        return loss.value
