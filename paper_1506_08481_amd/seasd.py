"""Python binding of the C ABI in include/seasd.h (ctypes; marshalling only).

Every step of the mobility product and of the far-field solve runs in the HIP
library libseasd.so built by paper_1506_08481_amd.build. Importing this module
when the library has not been built raises at once; there is no other
implementation to fall back on.

PyTorch is used for device memory and streams: the functions take CUDA/HIP
tensors and pass their data pointers and torch's current stream.
"""
from __future__ import annotations

import ctypes
import math
import numbers
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libseasd.so")

SEASD_OK = 0
SEASD_E_INVALID_ARG = -1
SEASD_E_NONFINITE = -2
SEASD_E_OVERLAP = -3
SEASD_E_CUTOFF = -4
SEASD_E_SINGULAR = -5
SEASD_E_HIP = -6
SEASD_E_NOMEM = -7
SEASD_E_UNSUPPORTED = -8
SEASD_E_FORMAT = -9
SEASD_E_SCRATCH = -10
SEASD_W_NOT_CONVERGED = 1
SEASD_W_PRECOND_FALLBACK = 2

SEASD_FP64, SEASD_FP32, SEASD_MIXED = 0, 1, 2
SEASD_PARTS_REAL, SEASD_PARTS_WAVE, SEASD_PARTS_SELF, SEASD_PARTS_ALL = 1, 2, 4, 7
SEASD_PRECOND_NONE, SEASD_PRECOND_BLOCKDIAG, SEASD_PRECOND_LEARNED_GUESS = 0, 1, 3

PHASES = ("bin", "pair", "window", "spread", "fft_x_fwd", "fft_y_fwd", "fft_z_scale", "fft_y_inv", "fft_x_inv",
          "gather")

# exported symbols of include/seasd.h
SYMBOLS = ("seasd_create", "seasd_destroy", "seasd_default_config", "seasd_set_config",
           "seasd_mobility_apply", "seasd_mobility_apply_static", "seasd_solve_farfield", "seasd_solve_mixed", "seasd_brownian_farfield", "seasd_profile_enable",
           "seasd_profile_read", "seasd_error_string", "seasd_autotune", "seasd_batch_create",
           "seasd_batch_apply", "seasd_batch_configs", "seasd_batch_destroy",
           "seasd_mobility_apply_batched", "seasd_net_create", "seasd_net_destroy", "seasd_net_param_count",
           "seasd_net_get_params", "seasd_net_set_params", "seasd_net_save", "seasd_net_load",
           "seasd_net_loss_grad", "seasd_net_train_step", "seasd_precond_attach", "seasd_precond_load")


SEASD_SIZE_REAL = 0
SEASD_SIZE_HYBRID = 1
SEASD_SIZE_WAVE = 2


class seasd_config(ctypes.Structure):
    _fields_ = [
        ("grid", ctypes.c_int32 * 3),
        ("P", ctypes.c_int32),
        ("size_approach", ctypes.c_int32),
        ("m", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("rc_factor", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("parts", ctypes.c_int32),
        ("compressible", ctypes.c_int32),
        ("checks", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("restart", ctypes.c_int32),
        ("precond", ctypes.c_int32),
    ]

    def as_dict(self):
        out = {k: getattr(self, k) for k, _ in self._fields_}
        out["grid"] = tuple(self.grid)
        return out


def _set_field(c: seasd_config, k: str, v):
    """Set one configuration field; grid takes an int (all directions) or 3 ints."""
    if not hasattr(c, k):
        raise KeyError(k)
    if k == "grid":
        vals = [int(v)] * 3 if isinstance(v, numbers.Integral) else [int(u) for u in v]
        if len(vals) != 3:
            raise ValueError("grid needs one or three values")
        c.grid = (ctypes.c_int32 * 3)(*vals)
    else:
        setattr(c, k, v)


class seasd_solve_stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("matvecs", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("true_residual", ctypes.c_double),
        ("setup_ms", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
        ("precond_used", ctypes.c_int32),
        ("guess_used", ctypes.c_int32),
        ("initial_residual", ctypes.c_double),
        ("guess_scale", ctypes.c_double),
        ("learned_ms", ctypes.c_double),
        ("inner_iterations", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class seasd_bsr6(ctypes.Structure):
    _fields_ = [
        ("nnzb", ctypes.c_int64),
        ("rowptr", ctypes.c_void_p),
        ("col", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
    ]


class seasd_brownian_stats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int32),
        ("solves", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("matvecs", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("max_residual", ctypes.c_double),
        ("scale", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SeasdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"seasd error {code}: {msg}")
        self.code = code


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1506_08481_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.seasd_create.argtypes = [ctypes.POINTER(vp), i32]
    lib.seasd_destroy.argtypes = [vp]
    lib.seasd_default_config.argtypes = [ctypes.POINTER(seasd_config)]
    lib.seasd_set_config.argtypes = [vp, ctypes.POINTER(seasd_config)]
    lib.seasd_mobility_apply.argtypes = [vp, i64, dp, dp, ctypes.POINTER(ctypes.c_double), dp, dp, vp]
    lib.seasd_mobility_apply_static.argtypes = [vp, i64, dp, dp, ctypes.POINTER(ctypes.c_double), dp, dp, vp]
    lib.seasd_solve_mixed.argtypes = [vp, i64, dp, dp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(seasd_bsr6),
                                      ctypes.c_double, dp, dp, dp, dp, dp, ctypes.POINTER(seasd_solve_stats), vp]
    lib.seasd_solve_farfield.argtypes = [vp, i64, dp, dp, ctypes.POINTER(ctypes.c_double), dp, dp,
                                         ctypes.POINTER(seasd_solve_stats), vp]
    lib.seasd_brownian_farfield.argtypes = [vp, i64, dp, dp, ctypes.POINTER(ctypes.c_double), dp, dp,
                                            ctypes.c_double, ctypes.POINTER(seasd_brownian_stats), vp]
    lib.seasd_profile_enable.argtypes = [vp, i32]
    lib.seasd_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32]
    lib.seasd_autotune.argtypes = [i64, ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, i32, ctypes.POINTER(seasd_config)]
    lib.seasd_batch_create.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64), dp, dp, ctypes.POINTER(ctypes.c_double),
                                       ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(vp), vp]
    lib.seasd_batch_apply.argtypes = [vp, dp, dp, vp]
    lib.seasd_batch_configs.argtypes = [vp, ctypes.POINTER(seasd_config)]
    lib.seasd_batch_destroy.argtypes = [vp]
    lib.seasd_mobility_apply_batched.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64), dp, dp,
                                                 ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, dp, dp, vp]
    lib.seasd_net_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.c_uint64]
    lib.seasd_net_destroy.argtypes = [vp]
    lib.seasd_net_param_count.argtypes = []
    fp = ctypes.POINTER(ctypes.c_float)
    lib.seasd_net_get_params.argtypes = [vp, fp, i64]
    lib.seasd_net_set_params.argtypes = [vp, fp, i64]
    lib.seasd_net_save.argtypes = [vp, ctypes.c_char_p]
    lib.seasd_net_load.argtypes = [vp, ctypes.c_char_p]
    lib.seasd_net_loss_grad.argtypes = [vp, vp, i64, dp, dp, ctypes.POINTER(ctypes.c_double), i32, dp, dp,
                                        ctypes.POINTER(ctypes.c_double), fp, vp]
    lib.seasd_net_train_step.argtypes = [vp, vp, i64, dp, dp, ctypes.POINTER(ctypes.c_double), i32, dp,
                                         ctypes.c_float, ctypes.POINTER(ctypes.c_double), vp]
    lib.seasd_precond_attach.argtypes = [vp, vp]
    lib.seasd_precond_load.argtypes = [vp, ctypes.c_char_p]
    lib.seasd_error_string.argtypes = [i32]
    lib.seasd_error_string.restype = ctypes.c_char_p
    for name in SYMBOLS:
        if name != "seasd_error_string":
            getattr(lib, name).restype = ctypes.c_int
    lib.seasd_net_param_count.restype = ctypes.c_int64
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _torch_first():
    """Let torch bring up its HIP runtime before the library touches the
    device: torch may carry its own copy of the runtime, which does not start
    once the system copy has claimed the device in this process."""
    import torch
    torch.cuda.init()


def _check(code: int, allow=(SEASD_OK,)) -> int:
    if code not in allow:
        raise SeasdError(code, lib().seasd_error_string(code).decode())
    return code


def default_config(**overrides) -> seasd_config:
    c = seasd_config()
    _check(lib().seasd_default_config(ctypes.byref(c)))
    for k, v in overrides.items():
        _set_field(c, k, v)
    return c


def _box9(box) -> ctypes.Array:
    vals = [float(v) for v in (box.T.reshape(-1) if hasattr(box, "T") else box)]
    if len(vals) != 9:
        raise ValueError("box needs 9 values")
    return (ctypes.c_double * 9)(*vals)


def _stream_ptr(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _device_of(t):
    return (t.device.type, t.device.index if t.device.index is not None else 0)


def _require(t, shape, name, device=None):
    """t must be a contiguous float64 tensor on the GPU `device` (an ordinal,
    or None for any) with the given shape (None entries: any size). Raises
    before anything reaches the library, so a short or strided buffer never
    becomes an out-of-bounds device access."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 GPU tensor")
    if device is not None and _device_of(t) != ("cuda", int(device)):
        raise ValueError(f"{name} is on {t.device}, the engine on cuda:{device}")
    if len(t.shape) != len(shape) or any(s is not None and int(d) != s for d, s in zip(t.shape, shape)):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple('*' if s is None else s for s in shape)}")


def _require_sphere_arrays(pos, radius, device):
    _require(pos, (None, 3), "pos", device)
    n = int(pos.shape[0])
    if n < 1:
        raise ValueError("need at least one sphere")
    _require(radius, (n,), "radius", device)
    return n


class Seasd:
    """Owns one seasd_handle. box: a 3x3 array whose columns are the lattice
    vectors (or 9 numbers a1, a2, a3)."""

    def __init__(self, device: int = 0, **config):
        _torch_first()
        h = ctypes.c_void_p()
        _check(lib().seasd_create(ctypes.byref(h), int(device)))
        self.h = h
        self.device = device
        self.config = default_config(**config)
        _check(lib().seasd_set_config(self.h, ctypes.byref(self.config)))

    def set_config(self, **overrides):
        for k, v in overrides.items():
            _set_field(self.config, k, v)
        _check(lib().seasd_set_config(self.h, ctypes.byref(self.config)))

    def seasd_mobility_apply(self, pos, radius, box, x, y=None, stream=None):
        import torch
        n = _require_sphere_arrays(pos, radius, self.device)
        _require(x, (n, 12), "x", self.device)
        if y is None:
            y = torch.empty((n, 12), dtype=torch.float64, device=pos.device)
        _require(y, (n, 12), "y", self.device)
        if y.data_ptr() == x.data_ptr():
            raise ValueError("y may not alias x")
        _check(lib().seasd_mobility_apply(self.h, n, pos.data_ptr(), radius.data_ptr(), _box9(box),
                                          x.data_ptr(), y.data_ptr(), ctypes.c_void_p(_stream_ptr(stream))))
        return y

    apply = seasd_mobility_apply

    def seasd_mobility_apply_static(self, pos, radius, box, x, y=None, stream=None):
        """The allocation-free product (workspace in the library's static
        device array; y must be supplied by a caller that cannot allocate)."""
        import torch
        n = _require_sphere_arrays(pos, radius, self.device)
        _require(x, (n, 12), "x", self.device)
        if y is None:
            y = torch.empty((n, 12), dtype=torch.float64, device=pos.device)
        _require(y, (n, 12), "y", self.device)
        if y.data_ptr() == x.data_ptr():
            raise ValueError("y may not alias x")
        _check(lib().seasd_mobility_apply_static(self.h, n, pos.data_ptr(), radius.data_ptr(), _box9(box),
                                                 x.data_ptr(), y.data_ptr(), ctypes.c_void_p(_stream_ptr(stream))))
        return y

    apply_static = seasd_mobility_apply_static

    def seasd_solve_farfield(self, pos, radius, box, b, x0=None, stream=None):
        import torch
        n = _require_sphere_arrays(pos, radius, self.device)
        _require(b, (n, 12), "b", self.device)
        if x0 is not None:
            _require(x0, (n, 12), "x0", self.device)
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        st = seasd_solve_stats()
        code = lib().seasd_solve_farfield(self.h, n, pos.data_ptr(), radius.data_ptr(), _box9(box),
                                          b.data_ptr(), x.data_ptr(), ctypes.byref(st),
                                          ctypes.c_void_p(_stream_ptr(stream)))
        _check(code, allow=(SEASD_OK, SEASD_W_NOT_CONVERGED, SEASD_W_PRECOND_FALLBACK))
        out = st.as_dict()
        out["code"] = code
        return x, out

    solve = seasd_solve_farfield

    def seasd_solve_mixed(self, pos, radius, box, rowptr, col, val, lam, fp, einf, stream=None):
        """Near-field / far-field solve (Sec. 4.1) for the near-field resistance
        given as 6x6 blocks in block-row form (rowptr int32 [n+1], col int32
        [nnzb], val float64 [nnzb, 6, 6], all on the device). Returns the
        far-field force-torque [n, 6], stresslet [n, 5], velocity [n, 6] and
        the solve statistics."""
        import torch
        n = _require_sphere_arrays(pos, radius, self.device)
        for t, name in ((rowptr, "rowptr"), (col, "col")):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
                raise TypeError(f"{name} must be a contiguous int32 GPU tensor")
            if _device_of(t) != ("cuda", int(self.device)):
                raise ValueError(f"{name} is on {t.device}, the engine on cuda:{self.device}")
        if tuple(rowptr.shape) != (n + 1,):
            raise ValueError(f"rowptr has shape {tuple(rowptr.shape)}, expected ({n + 1},)")
        nnzb = int(col.shape[0])
        _require(val, (nnzb, 6, 6), "val", self.device)
        rp = rowptr.cpu().numpy()
        cl = col.cpu().numpy()
        if rp[0] != 0 or rp[-1] != nnzb or (rp[1:] < rp[:-1]).any() or (nnzb and (cl.min() < 0 or cl.max() >= n)):
            raise ValueError("rowptr / col do not describe a block-row matrix of n block rows")
        _require(fp, (n, 6), "fp", self.device)
        _require(einf, (n, 5), "einf", self.device)
        f = torch.empty((n, 6), dtype=torch.float64, device=pos.device)
        s = torch.empty((n, 5), dtype=torch.float64, device=pos.device)
        u = torch.empty((n, 6), dtype=torch.float64, device=pos.device)
        m = seasd_bsr6(nnzb, rowptr.data_ptr(), col.data_ptr(), val.data_ptr())
        st = seasd_solve_stats()
        code = lib().seasd_solve_mixed(self.h, n, pos.data_ptr(), radius.data_ptr(), _box9(box), ctypes.byref(m),
                                       float(lam), fp.data_ptr(), einf.data_ptr(), f.data_ptr(), s.data_ptr(),
                                       u.data_ptr(), ctypes.byref(st), ctypes.c_void_p(_stream_ptr(stream)))
        _check(code, allow=(SEASD_OK, SEASD_W_NOT_CONVERGED))
        out = st.as_dict()
        out["code"] = code
        return f, s, u, out

    solve_mixed = seasd_solve_mixed

    def seasd_brownian_farfield(self, pos, radius, box, psi, dtau: float = 0.1, stream=None):
        """x = M^(-1/2) psi (incompressible block) by the initial value problem."""
        import torch
        n = _require_sphere_arrays(pos, radius, self.device)
        _require(psi, (n, 12), "psi", self.device)
        x = torch.empty_like(psi)
        st = seasd_brownian_stats()
        code = lib().seasd_brownian_farfield(self.h, n, pos.data_ptr(), radius.data_ptr(), _box9(box),
                                             psi.data_ptr(), x.data_ptr(), float(dtau), ctypes.byref(st),
                                             ctypes.c_void_p(_stream_ptr(stream)))
        _check(code, allow=(SEASD_OK, SEASD_W_NOT_CONVERGED))
        out = st.as_dict()
        out["code"] = code
        return x, out

    brownian = seasd_brownian_farfield

    def seasd_precond_attach(self, net):
        """Use `net` for solves with precond=SEASD_PRECOND_LEARNED_GUESS (None detaches)."""
        _check(lib().seasd_precond_attach(self.h, net.h if net is not None else None))
        self._net = net   # keep it alive while attached

    attach = seasd_precond_attach

    def seasd_precond_load(self, path: str):
        _check(lib().seasd_precond_load(self.h, os.fsencode(path)))

    precond_load = seasd_precond_load

    def profile(self, enable: bool = True):
        _check(lib().seasd_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """Average ms per phase over the products since the last read, plus
        the number of products under the key 'products'."""
        buf = (ctypes.c_double * (len(PHASES) + 1))()
        n = lib().seasd_profile_read(self.h, buf, len(PHASES) + 1)
        if n < 0:
            _check(n)
        out = {PHASES[i]: buf[i] for i in range(len(PHASES))}
        out["products"] = int(buf[len(PHASES)])
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().seasd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """The learned preconditioner network (seasd_net)."""

    def __init__(self, device: int = 0, seed: int = 0):
        _torch_first()
        h = ctypes.c_void_p()
        _check(lib().seasd_net_create(ctypes.byref(h), int(device), ctypes.c_uint64(int(seed))))
        self.h = h
        self.count = int(lib().seasd_net_param_count())

    def params(self):
        import numpy as np
        out = np.zeros(self.count, dtype=np.float32)
        _check(lib().seasd_net_get_params(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), self.count))
        return out

    def set_params(self, values):
        import numpy as np
        v = np.ascontiguousarray(values, dtype=np.float32)
        if v.size != self.count:
            raise ValueError(f"need {self.count} parameters, got {v.size}")
        _check(lib().seasd_net_set_params(self.h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), self.count))

    def save(self, path: str):
        _check(lib().seasd_net_save(self.h, os.fsencode(path)))

    def load(self, path: str):
        _check(lib().seasd_net_load(self.h, os.fsencode(path)))

    def seasd_net_loss_grad(self, eng: "Seasd", pos, radius, box, b, want_loss=True, want_grad=False,
                            stream=None):
        """b: [nrhs, n, 12] (or [n, 12]) float64 device tensor. Returns
        (loss, grad, x0): the mean relative residual of the guesses, its
        gradient (numpy float32) and the guesses."""
        import numpy as np
        import torch
        n = _require_sphere_arrays(pos, radius, eng.device)
        if b.dim() == 2:
            b = b.unsqueeze(0)
        _require(b, (None, n, 12), "b", eng.device)
        nrhs = int(b.shape[0])
        x0 = torch.empty_like(b)
        loss = ctypes.c_double(0.0)
        grad = np.zeros(self.count, dtype=np.float32) if want_grad else None
        _check(lib().seasd_net_loss_grad(
            eng.h, self.h, n, pos.data_ptr(), radius.data_ptr(), _box9(box), nrhs, b.data_ptr(), x0.data_ptr(),
            ctypes.byref(loss) if want_loss else None,
            grad.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if grad is not None else None,
            ctypes.c_void_p(_stream_ptr(stream))))
        return (loss.value if want_loss else None), grad, x0

    loss_grad = seasd_net_loss_grad

    def seasd_net_train_step(self, eng: "Seasd", pos, radius, box, b, lr: float, stream=None) -> float:
        n = _require_sphere_arrays(pos, radius, eng.device)
        if b.dim() == 2:
            b = b.unsqueeze(0)
        _require(b, (None, n, 12), "b", eng.device)
        loss = ctypes.c_double(0.0)
        _check(lib().seasd_net_train_step(eng.h, self.h, int(b.shape[1]), pos.data_ptr(), radius.data_ptr(),
                                          _box9(box), int(b.shape[0]), b.data_ptr(), ctypes.c_float(lr),
                                          ctypes.byref(loss), ctypes.c_void_p(_stream_ptr(stream))))
        return loss.value

    train_step = seasd_net_train_step

    def close(self):
        if getattr(self, "h", None):
            lib().seasd_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def seasd_autotune(n: int, box, a_min: float, a_max: float, target: float = 1e-6,
                   precision: int = SEASD_FP32) -> seasd_config:
    """box: a 3x3 array whose columns are the lattice vectors, 9 numbers, or
    a cube edge L."""
    if isinstance(box, (int, float)):
        box = [float(box), 0, 0, 0, float(box), 0, 0, 0, float(box)]
    c = seasd_config()
    _check(lib().seasd_autotune(int(n), _box9(box), float(a_min), float(a_max), float(target), int(precision),
                                ctypes.byref(c)))
    return c


class Batch:
    """A plan for many independent suspensions (concatenated sphere arrays)
    whose products run as one hipGraph launch."""

    def __init__(self, eng: "Seasd", offsets, pos, radius, boxes, per_sys=None, target: float = 1e-6,
                 stream=None):
        nsys = len(offsets) - 1
        if nsys < 1 or int(offsets[0]) != 0 or any(int(offsets[k + 1]) <= int(offsets[k]) for k in range(nsys)):
            raise ValueError("offsets must start at 0 and increase")
        if len(boxes) != nsys or (per_sys is not None and len(per_sys) != nsys):
            raise ValueError("need one box (and configuration) per suspension")
        n = _require_sphere_arrays(pos, radius, eng.device)
        if n != int(offsets[-1]):
            raise ValueError(f"pos has {n} rows, offsets end at {int(offsets[-1])}")
        self.device = eng.device
        off = (ctypes.c_int64 * (nsys + 1))(*[int(v) for v in offsets])
        bx = [float(v) for b in boxes for v in (b.T.reshape(-1) if hasattr(b, "T") else b)]
        boxes9 = (ctypes.c_double * (9 * nsys))(*bx)
        cfgs = None
        if per_sys is not None:
            cfgs = (seasd_config * nsys)(*per_sys)
        h = ctypes.c_void_p()
        _check(lib().seasd_batch_create(eng.h, nsys, off, pos.data_ptr(), radius.data_ptr(), boxes9,
                                        ctypes.cast(cfgs, ctypes.c_void_p) if cfgs is not None else None,
                                        float(target), ctypes.byref(h), ctypes.c_void_p(_stream_ptr(stream))))
        self.h = h
        self.nsys = nsys
        self.n = int(offsets[-1])

    def apply(self, x, y=None, stream=None):
        import torch
        _require(x, (self.n, 12), "x", self.device)
        if y is None:
            y = torch.empty_like(x)
        _require(y, (self.n, 12), "y", self.device)
        if y.data_ptr() == x.data_ptr():
            raise ValueError("y may not alias x")
        _check(lib().seasd_batch_apply(self.h, x.data_ptr(), y.data_ptr(), ctypes.c_void_p(_stream_ptr(stream))))
        return y

    def configs(self):
        out = (seasd_config * self.nsys)()
        _check(lib().seasd_batch_configs(self.h, out))
        return list(out)

    def close(self):
        if getattr(self, "h", None):
            lib().seasd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_m(P: int) -> float:
    return math.sqrt(math.pi * P)
