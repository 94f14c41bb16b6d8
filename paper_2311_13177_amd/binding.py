"""ctypes binding of libvp.so: the C ABI of include/vp.h with the same names.

The functions below only marshal arguments. Every step of the reconstruction runs in
the HIP library; if the library is missing or cannot load, ``lib()`` raises instead
of falling back to anything else. Device arrays are torch tensors (PyTorch is used
for device memory and streams only); host arrays are NumPy arrays.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_float, c_int32, c_int64, c_uint8, c_uint64, c_void_p
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvp.so")

VP_OK = 0
VP_ERR_ARG = -1
VP_ERR_UNSUPPORTED = -2
VP_ERR_DEVICE = -3
VP_ERR_NONFINITE = -4
VP_ERR_BUDGET = -5
VP_ERR_NOMEM = -6
VP_ERR_TIMEOUT = -7
VP_ERR_CANCELLED = -8
VP_ERR_NOT_FOUND = -9
VP_ERR_STATE = -10

VP_OPT_ADAM = 0
VP_OPT_GD = 1
VP_SCHED_ALL_BLADES = 0
VP_SCHED_CYCLIC = 1
VP_SCHED_RANDOM = 2


class VPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class vp_geometry(ctypes.Structure):
    _fields_ = [("n", c_int32), ("n_spec", c_int32), ("n_time", c_int32), ("n_blades", c_int32),
                ("angle_rad", POINTER(c_double)), ("lines", POINTER(c_int32)),
                ("blade_time", POINTER(c_double)), ("spec_shift_px", POINTER(c_double))]


class vp_tiles(ctypes.Structure):
    _fields_ = [("proj_rows", c_int32), ("proj_parts", c_int32), ("gath_rows", c_int32), ("gath_bins", c_int32),
                ("upd_bins", c_int32), ("gath_waves", c_int32), ("proj_waves", c_int32), ("gath_resident", c_int32)]

    def as_tuple(self):
        return (self.proj_rows, self.proj_parts, self.gath_rows, self.gath_bins, self.upd_bins, self.gath_waves,
                self.proj_waves, self.gath_resident)


class vp_options(ctypes.Structure):
    _fields_ = [("tv_weight", c_float), ("l1_weight", c_float), ("tv_eps", c_float), ("n_steps", c_int32),
                ("optimizer", c_int32), ("lr", c_float), ("beta1", c_float), ("beta2", c_float),
                ("adam_eps", c_float), ("schedule", c_int32), ("split_bin", c_int32), ("device", c_int32),
                ("tiles", vp_tiles), ("autotune", c_int32), ("seed", ctypes.c_uint32), ("data_weight", c_float)]


VP_KP_MAX_SCALES = 2


class vp_kplanes(ctypes.Structure):
    """K-Planes model (Section 4.1): features F, time nodes R_t, the x/y nodes of each scale
    and the grid regulariser weights."""
    _fields_ = [("features", c_int32), ("time_res", c_int32), ("n_scales", c_int32),
                ("spatial_res", c_int32 * VP_KP_MAX_SCALES), ("tv_weight", c_float), ("smooth_weight", c_float),
                ("sparse_weight", c_float), ("eps", c_float)]

    @classmethod
    def make(cls, features: int, time_res: int, spatial_res, tv_weight: float = 0.0, smooth_weight: float = 0.0,
             sparse_weight: float = 0.0, eps: float = 1e-3) -> "vp_kplanes":
        res = list(spatial_res)
        m = cls()
        m.features, m.time_res, m.n_scales = int(features), int(time_res), len(res)
        for i, r in enumerate(res[:VP_KP_MAX_SCALES]):
            m.spatial_res[i] = int(r)
        m.tv_weight, m.smooth_weight, m.sparse_weight, m.eps = tv_weight, smooth_weight, sparse_weight, eps
        return m


class vp_result(ctypes.Structure):
    _fields_ = [("volume_out", c_void_p), ("proj_out", c_void_p), ("water_out", c_void_p),
                ("fat_out", c_void_p), ("final_loss", c_double), ("steps_done", c_int64),
                ("status", c_int32)]


_P = c_void_p
_PROTOS = {
    "vp_options_default": (c_int32, [POINTER(vp_options)]),
    "vp_status_string": (ctypes.c_char_p, [c_int32]),
    "vp_last_error": (ctypes.c_char_p, []),
    "vp_plan_create": (c_int32, [POINTER(vp_geometry), POINTER(_P)]),
    "vp_plan_destroy": (c_int32, [_P]),
    "vp_plan_shape": (c_int32, [_P, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]),
    "vp_plan_mask": (c_int32, [_P, c_int32, POINTER(c_uint8)]),
    "vp_plan_shear": (c_int32, [_P, c_int32, c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_float),
                                POINTER(c_float)]),
    "vp_plan_knot": (c_int32, [_P, c_int32, POINTER(c_int32), POINTER(c_float)]),
    "vp_plan_device_bytes": (c_int32, [_P, POINTER(vp_options), POINTER(c_uint64)]),
    "vp_plan_tune": (c_int32, [_P, POINTER(vp_options), POINTER(vp_tiles)]),
    "vp_plan_tiles": (c_int32, [_P, POINTER(vp_options), POINTER(vp_tiles)]),
    "vp_forward": (c_int32, [_P, _P, _P, _P, _P]),
    "vp_forward_noalloc": (c_int32, [_P, _P, _P, _P, _P]),
    "vp_adjoint": (c_int32, [_P, _P, _P, c_int32, _P]),
    "vp_tv_grad": (c_int32, [_P, _P, c_float, c_float, c_float, _P, c_int32, _P]),
    "vp_render": (c_int32, [_P, _P, c_int32, _P, _P, _P, _P]),
    "vp_baseline": (c_int32, [_P, _P, c_int32, c_int32, c_int32, _P, _P]),
    "vp_nu_forward": (c_int32, [_P, _P, _P, _P, _P]),
    "vp_nu_adjoint": (c_int32, [_P, _P, _P, c_int32, _P]),
    "vp_step": (c_int32, [_P, POINTER(vp_options), _P, _P, _P, _P, c_int64, _P, _P]),
    "vp_nu_reconstruct": (c_int32, [_P, POINTER(vp_options), _P, _P, _P, _P, _P, _P, POINTER(c_double)]),
    "vp_nu_session_create": (c_int32, [_P, POINTER(vp_options), _P, _P, POINTER(c_void_p)]),
    "vp_nu_session_step": (c_int32, [_P, c_int32, c_int32]),
    "vp_nu_session_stage_times": (c_int32, [_P, c_int32, POINTER(c_double)]),
    "vp_nu_session_read": (c_int32, [_P, _P, _P, _P, _P, POINTER(c_double)]),
    "vp_nu_session_destroy": (c_int32, [_P]),
    "vp_kplanes_session_get_state": (c_int32, [_P, _P, _P, _P, POINTER(c_int64)]),
    "vp_kplanes_session_set_state": (c_int32, [_P, _P, _P, _P, c_int64]),
    "vp_nu_session_get_state": (c_int32, [_P, _P, _P, _P, POINTER(c_int64)]),
    "vp_nu_session_set_state": (c_int32, [_P, _P, _P, _P, c_int64]),
    "vp_psnr": (c_int32, [_P, _P, c_int64, c_int32, _P, _P]),
    "vp_session_create": (c_int32, [_P, POINTER(vp_options), _P, _P, POINTER(_P)]),
    "vp_session_step": (c_int32, [_P, c_int32, c_int32]),
    "vp_session_steps_done": (c_int32, [_P, POINTER(c_int64)]),
    "vp_session_read": (c_int32, [_P, _P, _P, _P, _P]),
    "vp_session_objective": (c_int32, [_P, POINTER(c_double), POINTER(c_double)]),
    "vp_session_get_state": (c_int32, [_P, _P, _P, _P, POINTER(c_int64)]),
    "vp_session_set_state": (c_int32, [_P, _P, _P, _P, c_int64]),
    "vp_session_stage_times": (c_int32, [_P, c_int32, POINTER(c_double)]),
    "vp_session_destroy": (c_int32, [_P]),
    "vp_reconstruct": (c_int32, [_P, POINTER(vp_options), _P, _P, _P, _P, _P, _P, POINTER(c_double)]),
    "vp_batch_reconstruct": (c_int32, [c_int32, POINTER(_P), POINTER(POINTER(vp_options)), POINTER(_P),
                                       POINTER(POINTER(vp_result))]),
    "vp_batch_create": (c_int32, [c_int32, POINTER(_P), POINTER(POINTER(vp_options)), POINTER(_P), POINTER(_P)]),
    "vp_batch_step": (c_int32, [_P, c_int32, c_int32]),
    "vp_batch_stage_times": (c_int32, [_P, c_int32, POINTER(c_double)]),
    "vp_batch_read": (c_int32, [_P, c_int32, POINTER(vp_result)]),
    "vp_batch_destroy": (c_int32, [_P]),
    "vp_kplanes_param_count": (c_int32, [_P, POINTER(vp_kplanes), POINTER(c_int64)]),
    "vp_kplanes_decode": (c_int32, [_P, POINTER(vp_kplanes), _P, POINTER(c_double), c_int32, _P, _P]),
    "vp_kplanes_gradient": (c_int32, [_P, POINTER(vp_kplanes), _P, _P, _P, POINTER(c_double),
                                      POINTER(c_double), _P]),
    "vp_kplanes_session_create": (c_int32, [_P, POINTER(vp_kplanes), POINTER(vp_options), _P, _P, POINTER(_P)]),
    "vp_kplanes_session_step": (c_int32, [_P, c_int32, c_int32]),
    "vp_kplanes_session_read": (c_int32, [_P, _P, c_int32, POINTER(c_double), _P, _P, _P, POINTER(c_double)]),
    "vp_kplanes_session_stage_times": (c_int32, [_P, c_int32, POINTER(c_double)]),
    "vp_kplanes_session_destroy": (c_int32, [_P]),
    "vp_kplanes_reconstruct": (c_int32, [_P, POINTER(vp_kplanes), POINTER(vp_options), _P, _P, _P, c_int32,
                                         POINTER(c_double), _P, _P, _P, POINTER(c_double)]),
    "vp_server_create": (c_int32, [c_int32, c_uint64, c_int32, POINTER(_P)]),
    "vp_server_submit": (c_int32, [_P, _P, POINTER(vp_options), _P, POINTER(c_uint64)]),
    "vp_server_wait": (c_int32, [_P, c_uint64, c_int64, POINTER(vp_result)]),
    "vp_server_poll": (c_int32, [_P, c_uint64, POINTER(c_int32)]),
    "vp_server_cancel": (c_int32, [_P, c_uint64]),
    "vp_server_stats": (c_int32, [_P, POINTER(c_double), POINTER(c_double), POINTER(c_double),
                                  POINTER(c_int64)]),
    "vp_server_destroy": (c_int32, [_P]),
}

_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """The loaded library. Raises if libvp.so has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_2311_13177_amd.build)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def exported_names() -> list[str]:
    return list(_PROTOS)


def check(status: int) -> None:
    if status != VP_OK:
        msg = lib().vp_last_error().decode() or lib().vp_status_string(status).decode()
        raise VPError(status, msg)


def _dptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(POINTER(ctype))


def _host_c64(a: Optional[np.ndarray], shape=None) -> Optional[np.ndarray]:
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.complex64)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


def _hp(a: Optional[np.ndarray]):
    return None if a is None else c_void_p(a.ctypes.data)


# ------------------------------------------------------------------ options

def vp_options_default(**overrides) -> vp_options:
    """Default options with fields overridden by keyword; `tiles` takes a 4- to 8-tuple
    (proj_rows, proj_parts, gath_rows, gath_bins[, upd_bins[, gath_waves[, proj_waves[, gath_resident]]]])."""
    o = vp_options()
    check(lib().vp_options_default(byref(o)))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        if k == "tiles":
            v = vp_tiles(*[int(x) for x in v])
        setattr(o, k, v)
    return o


# ------------------------------------------------------------------ plans

class Plan:
    """Owns a vp_plan built by vp_plan_create from a geometry."""

    def __init__(self, n: int, n_spec: int, n_time: int, angle_rad, lines, blade_time, spec_shift_px):
        self._angle = np.ascontiguousarray(angle_rad, dtype=np.float64)
        self._lines = np.ascontiguousarray(lines, dtype=np.int32)
        self._time = None if blade_time is None else np.ascontiguousarray(blade_time, dtype=np.float64)
        self._shift = np.ascontiguousarray(spec_shift_px, dtype=np.float64)
        g = vp_geometry(n=n, n_spec=n_spec, n_time=n_time, n_blades=int(self._angle.shape[0]),
                        angle_rad=_dptr(self._angle, c_double), lines=_dptr(self._lines, c_int32),
                        blade_time=None if self._time is None else _dptr(self._time, c_double),
                        spec_shift_px=_dptr(self._shift, c_double))
        h = c_void_p()
        check(lib().vp_plan_create(byref(g), byref(h)))
        self.handle = h
        self.n, self.n_spec, self.n_time, self.n_blades = n, n_spec, n_time, int(self._angle.shape[0])

    @classmethod
    def from_geometry(cls, g: dict) -> "Plan":
        return cls(int(g["n"]), int(g["n_spec"]), int(g["n_time"]), g["angle_rad"], g["lines"],
                   g.get("blade_time"), g["spec_shift_px"])

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.vp_plan_destroy(h)
            self.handle = None

    @property
    def volume_shape(self):
        return (self.n_time, self.n_spec, self.n, self.n)

    @property
    def blade_shape(self):
        return (self.n_blades, self.n, self.n)

    @property
    def render_shape(self):
        return (self.n_time, self.n, self.n)

    def mask(self, b: int) -> np.ndarray:
        out = np.empty((self.n, self.n), dtype=np.uint8)
        check(lib().vp_plan_mask(self.handle, b, _dptr(out, c_uint8)))
        return out.astype(bool)

    def masks(self) -> np.ndarray:
        return np.stack([self.mask(b) for b in range(self.n_blades)])

    def shear(self, b: int, s: int):
        ox, oy, fx, fy = c_int32(), c_int32(), c_float(), c_float()
        check(lib().vp_plan_shear(self.handle, b, s, byref(ox), byref(oy), byref(fx), byref(fy)))
        return ox.value, oy.value, fx.value, fy.value

    def knot(self, b: int):
        k, a = c_int32(), c_float()
        check(lib().vp_plan_knot(self.handle, b, byref(k), byref(a)))
        return k.value, a.value

    def tune(self, opts: Optional[vp_options] = None) -> tuple:
        """Times the tile shapes on the device (vp_plan_tune); returns the fastest."""
        t = vp_tiles()
        check(lib().vp_plan_tune(self.handle, byref(opts if opts is not None else vp_options_default()), byref(t)))
        return t.as_tuple()

    def tiles(self, opts: Optional[vp_options] = None) -> tuple:
        """The tile shape a session with these options would use (vp_plan_tiles)."""
        t = vp_tiles()
        check(lib().vp_plan_tiles(self.handle, byref(opts if opts is not None else vp_options_default()), byref(t)))
        return t.as_tuple()

    def device_bytes(self, opts: Optional[vp_options] = None) -> int:
        out = c_uint64()
        check(lib().vp_plan_device_bytes(self.handle, None if opts is None else byref(opts), byref(out)))
        return int(out.value)


# ------------------------------------------------------------------ operators on torch device tensors

def _dev(t, shape, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.complex64:
        raise TypeError(f"{name} must be a complex64 GPU tensor")
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with shape {tuple(shape)}, got {tuple(t.shape)}")
    return c_void_p(t.data_ptr())


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def vp_forward(plan: Plan, vol, y=None, out=None, stream=None):
    """out = M . DFT2(P vol) - M . y on the GPU (torch tensors); returns out."""
    import torch

    if out is None:
        out = torch.empty(plan.blade_shape, dtype=torch.complex64, device=vol.device)
    check(lib().vp_forward(plan.handle, _dev(vol, plan.volume_shape, "vol"),
                           None if y is None else _dev(y, plan.blade_shape, "y"),
                           _dev(out, plan.blade_shape, "out"), _stream(stream)))
    return out


def vp_forward_noalloc(plan: Plan, vol, out, y=None, stream=None):
    """vp_forward into the caller's `out` with no device allocation (the library's fixed
    scratch array holds the blade images); returns out."""
    check(lib().vp_forward_noalloc(plan.handle, _dev(vol, plan.volume_shape, "vol"),
                                   None if y is None else _dev(y, plan.blade_shape, "y"),
                                   _dev(out, plan.blade_shape, "out"), _stream(stream)))
    return out


def vp_adjoint(plan: Plan, kres, grad=None, accumulate: bool = False, stream=None):
    """grad (+)= A^H kres on the GPU; returns grad."""
    import torch

    if grad is None:
        grad = torch.empty(plan.volume_shape, dtype=torch.complex64, device=kres.device)
        accumulate = False
    check(lib().vp_adjoint(plan.handle, _dev(kres, plan.blade_shape, "kres"),
                           _dev(grad, plan.volume_shape, "grad"), int(bool(accumulate)), _stream(stream)))
    return grad


def vp_tv_grad(plan: Plan, vol, tv_weight: float, l1_weight: float, tv_eps: float, grad=None,
               accumulate: bool = False, stream=None):
    import torch

    if grad is None:
        grad = torch.empty(plan.volume_shape, dtype=torch.complex64, device=vol.device)
        accumulate = False
    check(lib().vp_tv_grad(plan.handle, _dev(vol, plan.volume_shape, "vol"), float(tv_weight), float(l1_weight),
                           float(tv_eps), _dev(grad, plan.volume_shape, "grad"), int(bool(accumulate)),
                           _stream(stream)))
    return grad


def vp_render(plan: Plan, vol, split_bin: int = -1, stream=None):
    import torch

    shp = plan.render_shape
    outs = [torch.empty(shp, dtype=torch.complex64, device=vol.device) for _ in range(3)]
    check(lib().vp_render(plan.handle, _dev(vol, plan.volume_shape, "vol"), int(split_bin),
                          *[_dev(o, shp, "render") for o in outs], _stream(stream)))
    return tuple(outs)


def nu_shape(plan: Plan):
    """Shape [B][Lmax][n] of blade-aligned sample arrays."""
    return (plan.n_blades, int(np.max(plan._lines)), plan.n)


def vp_nu_forward(plan: Plan, vol, y=None, out=None, stream=None):
    """Blade-aligned samples of the projected volume (GPU tensors), minus y if given."""
    import torch

    shp = nu_shape(plan)
    if out is None:
        out = torch.empty(shp, dtype=torch.complex64, device=vol.device)
    check(lib().vp_nu_forward(plan.handle, _dev(vol, plan.volume_shape, "vol"),
                              None if y is None else _dev(y, shp, "y"), _dev(out, shp, "out"), _stream(stream)))
    return out


def vp_nu_adjoint(plan: Plan, samples, grad=None, accumulate: bool = False, stream=None):
    """grad (+)= the transpose of vp_nu_forward applied to samples [B][Lmax][n]."""
    import torch

    if grad is None:
        grad = torch.empty(plan.volume_shape, dtype=torch.complex64, device=samples.device)
        accumulate = False
    check(lib().vp_nu_adjoint(plan.handle, _dev(samples, nu_shape(plan), "samples"),
                              _dev(grad, plan.volume_shape, "grad"), int(bool(accumulate)), _stream(stream)))
    return grad


def vp_nu_reconstruct(plan: Plan, samples: np.ndarray, opts: Optional[vp_options] = None,
                      init: Optional[np.ndarray] = None) -> dict:
    """vp_reconstruct on blade-aligned samples [B][Lmax][n] (host arrays)."""
    opts = opts if opts is not None else vp_options_default()
    y = _host_c64(samples, nu_shape(plan))
    i = _host_c64(init, plan.volume_shape)
    vol = np.empty(plan.volume_shape, np.complex64)
    outs = [np.empty(plan.render_shape, np.complex64) for _ in range(3)]
    loss = c_double()
    check(lib().vp_nu_reconstruct(plan.handle, byref(opts), _hp(y), _hp(i), _hp(vol), *[_hp(o) for o in outs],
                                  byref(loss)))
    return dict(vol=vol, proj=outs[0], water=outs[1], fat=outs[2], final_loss=float(loss.value))


def vp_step(plan: Plan, opts: vp_options, vol, grad, m=None, v=None, t: int = 1, out=None, stream=None):
    """One optimiser step on GPU tensors: returns the new volume (m and v update in place)."""
    import torch

    if out is None:
        out = torch.empty_like(vol)
    check(lib().vp_step(plan.handle, byref(opts), _dev(vol, plan.volume_shape, "vol"),
                        _dev(grad, plan.volume_shape, "grad"),
                        None if m is None else _dev(m, plan.volume_shape, "m"),
                        None if v is None else _dev(v, plan.volume_shape, "v"), int(t),
                        _dev(out, plan.volume_shape, "out"), _stream(stream)))
    return out


NU_STAGES = ("project", "rows_fwd", "cols_fwd", "interp", "spread", "cols_inv", "rows_inv", "gather_update")


class NuSession:
    """Resident fit on blade-aligned samples [B][Lmax][n] (vp_nu_session_*)."""

    def __init__(self, plan: Plan, samples: np.ndarray, opts: Optional[vp_options] = None,
                 init: Optional[np.ndarray] = None):
        self.plan = plan
        self.opts = opts if opts is not None else vp_options_default()
        y = _host_c64(samples, nu_shape(plan))
        i = _host_c64(init, plan.volume_shape)
        h = c_void_p()
        check(lib().vp_nu_session_create(plan.handle, byref(self.opts), _hp(y), _hp(i), byref(h)))
        self.handle = h

    def step(self, n_steps: int, use_graph: bool = True) -> None:
        check(lib().vp_nu_session_step(self.handle, int(n_steps), int(bool(use_graph))))

    def stage_times(self, n_steps: int = 10) -> dict:
        ms = (c_double * len(NU_STAGES))()
        check(lib().vp_nu_session_stage_times(self.handle, int(n_steps), ms))
        return dict(zip(NU_STAGES, list(ms)))

    def read(self, objective: bool = False) -> dict:
        vol = np.empty(self.plan.volume_shape, np.complex64)
        outs = [np.empty(self.plan.render_shape, np.complex64) for _ in range(3)]
        obj = c_double()
        check(lib().vp_nu_session_read(self.handle, _hp(vol), *[_hp(o) for o in outs],
                                       byref(obj) if objective else None))
        res = dict(vol=vol, proj=outs[0], water=outs[1], fat=outs[2])
        if objective:
            res["objective"] = obj.value
        return res

    def get_state(self) -> dict:
        p = self.plan
        vol, m, v = (np.empty(p.volume_shape, np.complex64) for _ in range(3))
        st = c_int64()
        check(lib().vp_nu_session_get_state(self.handle, _hp(vol), _hp(m), _hp(v), byref(st)))
        return dict(vol=vol, m=m, v=v, step=int(st.value))

    def set_state(self, state: dict) -> None:
        p = self.plan
        vol = _host_c64(state["vol"], p.volume_shape)
        m = _host_c64(state.get("m"), p.volume_shape)
        v = _host_c64(state.get("v"), p.volume_shape)
        check(lib().vp_nu_session_set_state(self.handle, _hp(vol), _hp(m), _hp(v), int(state["step"])))

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().vp_nu_session_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def vp_baseline(plan: Plan, kspace, window: int = 0, first_frame: Optional[int] = None,
                n_frames: Optional[int] = None, out=None, stream=None):
    """Coverage-weighted k-space average of blades max(0, f - window + 1) .. f, inverse
    DFT, for frames f = first_frame .. first_frame + n_frames - 1 (GPU tensors).
    Defaults: window 0 (every blade up to the frame), the last frame only."""
    import torch

    B = plan.blade_shape[0]
    if first_frame is None:
        first_frame = B - 1 if n_frames is None else B - n_frames
    if n_frames is None:
        n_frames = B - first_frame
    shp = (n_frames,) + tuple(plan.blade_shape[1:])
    if out is None:
        out = torch.empty(shp, dtype=torch.complex64, device=kspace.device)
    check(lib().vp_baseline(plan.handle, _dev(kspace, plan.blade_shape, "kspace"), int(window),
                            int(first_frame), int(n_frames), _dev(out, shp, "out"), _stream(stream)))
    return out


def vp_psnr(image, truth, stream=None):
    """PSNR on magnitudes of each leading-axis image of `image` against `truth` (GPU
    tensors of equal shape; a 2-D pair is one image). Returns (psnr, mse, peak) as
    float64 tensors on the device, one entry per image."""
    import torch

    if tuple(image.shape) != tuple(truth.shape) or image.dim() < 2:
        raise ValueError("image and truth must share a shape of two or more axes")
    n_images = 1 if image.dim() == 2 else int(np.prod(image.shape[:-2]))
    n_px = int(image.shape[-2] * image.shape[-1])
    terms = torch.empty((n_images, 3), dtype=torch.float64, device=image.device)
    check(lib().vp_psnr(_dev(image, image.shape, "image"), _dev(truth, truth.shape, "truth"), n_px, n_images,
                        c_void_p(terms.data_ptr()), _stream(stream)))
    return terms[:, 2], terms[:, 0], terms[:, 1]


# ------------------------------------------------------------------ sessions and reconstructions

class Session:
    """Resident reconstruction state on one device (vp_session_*)."""

    def __init__(self, plan: Plan, kspace: np.ndarray, opts: Optional[vp_options] = None,
                 init: Optional[np.ndarray] = None):
        self.plan = plan
        self.opts = opts if opts is not None else vp_options_default()
        self._k = _host_c64(kspace, plan.blade_shape)
        i = _host_c64(init, plan.volume_shape)
        h = c_void_p()
        check(lib().vp_session_create(plan.handle, byref(self.opts), _hp(self._k), _hp(i), byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().vp_session_destroy(self.handle)
        self.handle = None

    __del__ = close

    def step(self, n_steps: int, use_graph: bool = True):
        check(lib().vp_session_step(self.handle, int(n_steps), int(bool(use_graph))))

    @property
    def steps_done(self) -> int:
        v = c_int64()
        check(lib().vp_session_steps_done(self.handle, byref(v)))
        return int(v.value)

    def read(self, volume: bool = True):
        p = self.plan
        vol = np.empty(p.volume_shape, np.complex64) if volume else None
        outs = [np.empty(p.render_shape, np.complex64) for _ in range(3)]
        check(lib().vp_session_read(self.handle, _hp(vol), *[_hp(o) for o in outs]))
        return dict(vol=vol, proj=outs[0], water=outs[1], fat=outs[2])

    STAGES = ("project", "rows_fwd", "cols", "rows_inv", "gather_update")

    def stage_times(self, n_steps: int) -> dict:
        """Mean milliseconds per stage over n_steps eager steps (HIP events on the session stream)."""
        out = (c_double * len(self.STAGES))()
        check(lib().vp_session_stage_times(self.handle, int(n_steps), out))
        return dict(zip(self.STAGES, list(out)))

    def objective(self):
        o, d = c_double(), c_double()
        check(lib().vp_session_objective(self.handle, byref(o), byref(d)))
        return float(o.value), float(d.value)

    def get_state(self):
        p = self.plan
        vol = np.empty(p.volume_shape, np.complex64)
        m = np.empty(p.volume_shape, np.complex64)
        v = np.empty(p.volume_shape, np.complex64)
        st = c_int64()
        check(lib().vp_session_get_state(self.handle, _hp(vol), _hp(m), _hp(v), byref(st)))
        return dict(vol=vol, m=m, v=v, step=int(st.value))

    def set_state(self, state: dict):
        p = self.plan
        vol = _host_c64(state["vol"], p.volume_shape)
        m = _host_c64(state.get("m"), p.volume_shape)
        v = _host_c64(state.get("v"), p.volume_shape)
        check(lib().vp_session_set_state(self.handle, _hp(vol), _hp(m), _hp(v), int(state["step"])))


def vp_reconstruct(plan: Plan, kspace: np.ndarray, opts: Optional[vp_options] = None,
                   init: Optional[np.ndarray] = None, volume: bool = True) -> dict:
    """A whole reconstruction; volume=False copies back only the renders and the objective."""
    opts = opts if opts is not None else vp_options_default()
    k = _host_c64(kspace, plan.blade_shape)
    i = _host_c64(init, plan.volume_shape)
    vol = np.empty(plan.volume_shape, np.complex64) if volume else None
    outs = [np.empty(plan.render_shape, np.complex64) for _ in range(3)]
    loss = c_double()
    check(lib().vp_reconstruct(plan.handle, byref(opts), _hp(k), _hp(i), _hp(vol), *[_hp(o) for o in outs],
                               byref(loss)))
    return dict(vol=vol, proj=outs[0], water=outs[1], fat=outs[2], final_loss=float(loss.value))


class Server:
    """Continuous-batching reconstruction server (vp_server_*)."""

    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, max_slots: int = 64):
        h = c_void_p()
        check(lib().vp_server_create(int(device), int(hbm_budget), int(max_slots), byref(h)))
        self.handle = h
        self._plans = {}
        self._opts = {}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().vp_server_destroy(self.handle)
        self.handle = None

    __del__ = close

    def submit(self, plan: Plan, kspace: np.ndarray, opts: Optional[vp_options] = None) -> int:
        opts = opts if opts is not None else vp_options_default()
        k = _host_c64(kspace, plan.blade_shape)
        rid = c_uint64()
        check(lib().vp_server_submit(self.handle, plan.handle, byref(opts), _hp(k), byref(rid)))
        self._plans[rid.value] = plan
        self._opts[rid.value] = opts
        return int(rid.value)

    def poll(self, rid: int) -> bool:
        d = c_int32()
        check(lib().vp_server_poll(self.handle, int(rid), byref(d)))
        return bool(d.value)

    def cancel(self, rid: int) -> None:
        check(lib().vp_server_cancel(self.handle, int(rid)))

    def wait(self, rid: int, timeout_us: int = -1, raise_on_error: bool = True, volume: bool = True) -> dict:
        """The request's result; with volume=False only the renders and the objective are
        copied back (the volume stays on the device until it is released)."""
        plan = self._plans[rid]
        vol = np.empty(plan.volume_shape, np.complex64) if volume else None
        rend = [np.empty(plan.render_shape, np.complex64) for _ in range(3)]
        res = vp_result(volume_out=vol.ctypes.data if volume else None, proj_out=rend[0].ctypes.data,
                        water_out=rend[1].ctypes.data, fat_out=rend[2].ctypes.data)
        st = lib().vp_server_wait(self.handle, int(rid), int(timeout_us), byref(res))
        if st != VP_ERR_TIMEOUT:
            self._plans.pop(rid, None)
            self._opts.pop(rid, None)
        if st != VP_OK and raise_on_error:
            check(st)
        return dict(vol=vol, proj=rend[0], water=rend[1], fat=rend[2], final_loss=float(res.final_loss),
                    steps_done=int(res.steps_done), status=int(st))

    def stats(self) -> dict:
        p50, p99, thr, done = c_double(), c_double(), c_double(), c_int64()
        check(lib().vp_server_stats(self.handle, byref(p50), byref(p99), byref(thr), byref(done)))
        return dict(p50_us=p50.value, p99_us=p99.value, throughput_rps=thr.value, completed=int(done.value))


def vp_batch_reconstruct(plans: Sequence[Plan], kspaces: Sequence[np.ndarray],
                         opts: Sequence[vp_options]) -> list[dict]:
    n = len(plans)
    ks = [_host_c64(k, p.blade_shape) for p, k in zip(plans, kspaces)]
    vols = [np.empty(p.volume_shape, np.complex64) for p in plans]
    rend = [[np.empty(p.render_shape, np.complex64) for _ in range(3)] for p in plans]
    res = [vp_result(volume_out=v.ctypes.data, proj_out=r[0].ctypes.data, water_out=r[1].ctypes.data,
                     fat_out=r[2].ctypes.data) for v, r in zip(vols, rend)]
    plan_arr = (c_void_p * n)(*[p.handle.value for p in plans])
    opt_arr = (POINTER(vp_options) * n)(*[ctypes.pointer(o) for o in opts])
    k_arr = (c_void_p * n)(*[k.ctypes.data for k in ks])
    res_arr = (POINTER(vp_result) * n)(*[ctypes.pointer(r) for r in res])
    status = lib().vp_batch_reconstruct(n, plan_arr, opt_arr, k_arr, res_arr)
    out = []
    for i in range(n):
        out.append(dict(vol=vols[i], proj=rend[i][0], water=rend[i][1], fat=rend[i][2],
                        final_loss=float(res[i].final_loss), steps_done=int(res[i].steps_done),
                        status=int(res[i].status)))
    if status != VP_OK and all(r["status"] == VP_OK for r in out):
        check(status)
    return out


class Batch:
    """A resident batch of slices (vp_batch_*): created once, stepped, timed and read."""

    STAGES = ("project", "rows_fwd", "cols", "rows_inv", "gather_update")

    def __init__(self, plans: Sequence[Plan], kspaces: Sequence[np.ndarray], opts: Sequence[vp_options]):
        n = len(plans)
        self.plans = list(plans)
        ks = [_host_c64(k, p.blade_shape) for p, k in zip(plans, kspaces)]
        self._opts = list(opts)
        plan_arr = (c_void_p * n)(*[p.handle.value for p in plans])
        opt_arr = (POINTER(vp_options) * n)(*[ctypes.pointer(o) for o in self._opts])
        k_arr = (c_void_p * n)(*[k.ctypes.data for k in ks])
        h = c_void_p()
        st = lib().vp_batch_create(n, plan_arr, opt_arr, k_arr, byref(h))
        self.handle = h if h.value else None
        if self.handle is None:
            check(st)

    def step(self, n_steps: int, use_graph: bool = True) -> None:
        check(lib().vp_batch_step(self.handle, int(n_steps), int(bool(use_graph))))

    def stage_times(self, n_steps: int) -> dict:
        out = (c_double * len(self.STAGES))()
        check(lib().vp_batch_stage_times(self.handle, int(n_steps), out))
        return dict(zip(self.STAGES, list(out)))

    def read(self, i: int) -> dict:
        p = self.plans[i]
        vol = np.empty(p.volume_shape, np.complex64)
        rend = [np.empty(p.render_shape, np.complex64) for _ in range(3)]
        res = vp_result(volume_out=vol.ctypes.data, proj_out=rend[0].ctypes.data, water_out=rend[1].ctypes.data,
                        fat_out=rend[2].ctypes.data)
        st = lib().vp_batch_read(self.handle, int(i), byref(res))
        return dict(vol=vol, proj=rend[0], water=rend[1], fat=rend[2], final_loss=float(res.final_loss),
                    steps_done=int(res.steps_done), status=int(st))

    def close(self):
        if getattr(self, "handle", None) is not None:
            lib().vp_batch_destroy(self.handle)
        self.handle = None

    __del__ = close


# ------------------------------------------------------------------ K-Planes dynamic model

def kplanes_param_count(plan: Plan, model: vp_kplanes) -> int:
    out = c_int64()
    check(lib().vp_kplanes_param_count(plan.handle, byref(model), byref(out)))
    return int(out.value)


def _times(times):
    t = np.ascontiguousarray(np.asarray(times, dtype=np.float64).reshape(-1))
    return t, t.ctypes.data_as(POINTER(c_double))


def vp_kplanes_decode(plan: Plan, model: vp_kplanes, params, times, out=None, stream=None):
    """The model at each time: a [len(times)][S][n][n] complex64 GPU tensor."""
    import torch

    t, tp = _times(times)
    np_ = kplanes_param_count(plan, model)
    shp = (len(t), plan.n_spec, plan.n, plan.n)
    if out is None:
        out = torch.empty(shp, dtype=torch.complex64, device=params.device)
    check(lib().vp_kplanes_decode(plan.handle, byref(model), _dev(params, (np_,), "params"), tp, len(t),
                                  _dev(out, shp, "out"), _stream(stream)))
    return out


def vp_kplanes_gradient(plan: Plan, model: vp_kplanes, params, kspace, grad=None, stream=None):
    """Returns (grad, objective, data_term) for GPU tensors params [count] and kspace [B][n][n]."""
    import torch

    np_ = kplanes_param_count(plan, model)
    if grad is None:
        grad = torch.empty((np_,), dtype=torch.complex64, device=params.device)
    obj, data = c_double(), c_double()
    check(lib().vp_kplanes_gradient(plan.handle, byref(model), _dev(params, (np_,), "params"),
                                    _dev(kspace, plan.blade_shape, "kspace"), _dev(grad, (np_,), "grad"),
                                    byref(obj), byref(data), _stream(stream)))
    return grad, obj.value, data.value


class KPlanesSession:
    """Resident K-Planes fit on one device (vp_kplanes_session_*)."""

    def __init__(self, plan: Plan, model: vp_kplanes, kspace: np.ndarray, init: np.ndarray,
                 opts: Optional[vp_options] = None):
        self.plan, self.model = plan, model
        self.opts = opts if opts is not None else vp_options_default()
        self.count = kplanes_param_count(plan, model)
        self._k = _host_c64(kspace, plan.blade_shape)
        self._i = _host_c64(init, (self.count,))
        h = c_void_p()
        check(lib().vp_kplanes_session_create(plan.handle, byref(model), byref(self.opts), _hp(self._k),
                                              _hp(self._i), byref(h)))
        self.handle = h

    def step(self, n_steps: int, use_graph: bool = True) -> None:
        check(lib().vp_kplanes_session_step(self.handle, int(n_steps), int(bool(use_graph))))

    def read(self, frame_times=(), objective: bool = False):
        t, tp = _times(frame_times)
        n = self.plan.blade_shape[1]
        params = np.empty(self.count, dtype=np.complex64)
        outs = [np.empty((len(t), n, n), dtype=np.complex64) for _ in range(3)]
        obj = c_double()
        check(lib().vp_kplanes_session_read(self.handle, _hp(params), len(t), tp if len(t) else None,
                                            *[_hp(o) if len(t) else None for o in outs],
                                            byref(obj) if objective else None))
        res = dict(params=params, proj=outs[0], water=outs[1], fat=outs[2])
        if objective:
            res["objective"] = obj.value
        return res

    def get_state(self) -> dict:
        p, m, v = (np.empty(self.count, np.complex64) for _ in range(3))
        st = c_int64()
        check(lib().vp_kplanes_session_get_state(self.handle, _hp(p), _hp(m), _hp(v), byref(st)))
        return dict(params=p, m=m, v=v, step=int(st.value))

    def set_state(self, state: dict) -> None:
        p = _host_c64(state["params"], (self.count,))
        m = _host_c64(state.get("m"), (self.count,))
        v = _host_c64(state.get("v"), (self.count,))
        check(lib().vp_kplanes_session_set_state(self.handle, _hp(p), _hp(m), _hp(v), int(state["step"])))

    def stage_times(self, n_steps: int = 10):
        ms = (c_double * 6)()
        check(lib().vp_kplanes_session_stage_times(self.handle, int(n_steps), ms))
        return dict(zip(("decode", "blade_fwd_adj", "grad_z", "grad_x", "grad_y", "grids_update"), list(ms)))

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().vp_kplanes_session_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def vp_kplanes_reconstruct(plan: Plan, model: vp_kplanes, kspace: np.ndarray, init: np.ndarray,
                           opts: Optional[vp_options] = None, frame_times=(0.0,)):
    """Whole K-Planes fit: dict(params, proj, water, fat, final_loss)."""
    opts = opts if opts is not None else vp_options_default()
    count = kplanes_param_count(plan, model)
    k = _host_c64(kspace, plan.blade_shape)
    i = _host_c64(init, (count,))
    t, tp = _times(frame_times)
    n = plan.blade_shape[1]
    params = np.empty(count, dtype=np.complex64)
    outs = [np.empty((len(t), n, n), dtype=np.complex64) for _ in range(3)]
    loss = c_double()
    check(lib().vp_kplanes_reconstruct(plan.handle, byref(model), byref(opts), _hp(k), _hp(i), _hp(params),
                                       len(t), tp if len(t) else None, *[_hp(o) if len(t) else None for o in outs],
                                       byref(loss)))
    return dict(params=params, proj=outs[0], water=outs[1], fat=outs[2], final_loss=loss.value)
