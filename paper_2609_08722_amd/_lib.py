"""ctypes view of the C ABI in include/tbr.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtbr.so")

TBR_OK, TBR_PENDING = 0, 1
TBR_E_INVALID, TBR_E_NOMEM, TBR_E_OVERFLOW, TBR_E_CAPACITY = -1, -2, -3, -4
TBR_E_DEVICE, TBR_E_CANCELLED, TBR_E_NOTFOUND = -5, -6, -7
TBR_HARD, TBR_SOFT = 1, 2
TBR_OUT_RGB, TBR_OUT_LABEL, TBR_OUT_OWNER, TBR_OUT_ALL = 1, 2, 4, 7
TBR_STATIC_MAX_STROKES = 8192  # tbr_render_static's stroke limit
TBR_TRANSPORT_CAPSULE, TBR_TRANSPORT_COUPLED, TBR_TRANSPORT_INERT, TBR_TRANSPORT_DROPS16 = 0, 1, 2, 3

STATUS_NAMES = {0: "TBR_OK", 1: "TBR_PENDING", -1: "TBR_E_INVALID", -2: "TBR_E_NOMEM",
                -3: "TBR_E_OVERFLOW", -4: "TBR_E_CAPACITY", -5: "TBR_E_DEVICE",
                -6: "TBR_E_CANCELLED", -7: "TBR_E_NOTFOUND"}


class TbrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Program(C.Structure):
    _fields_ = [("n_strokes", C.c_int32), ("n_palette", C.c_int32),
                ("cx", C.c_void_p), ("cy", C.c_void_p), ("angle", C.c_void_p),
                ("length", C.c_void_p), ("half_width", C.c_void_p),
                ("logits", C.c_void_p), ("palette", C.c_void_p)]


class ProgramGrad(C.Structure):
    _fields_ = [("cx", C.c_void_p), ("cy", C.c_void_p), ("angle", C.c_void_p),
                ("length", C.c_void_p), ("half_width", C.c_void_p),
                ("logits", C.c_void_p), ("palette", C.c_void_p)]


class RenderOpts(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("tau", C.c_float),
                ("tau_min", C.c_float), ("tau_c", C.c_float), ("eps_floor", C.c_float),
                ("ckpt_interval", C.c_int32), ("side_slots", C.c_int32),
                ("transport", C.c_int32), ("coupling", C.c_void_p)]


class AdamOpts(C.Structure):
    _fields_ = [("lr_centre", C.c_float), ("lr_angle", C.c_float), ("lr_length", C.c_float),
                ("lr_width", C.c_float), ("lr_logits", C.c_float), ("lr_palette", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("r_lo", C.c_float), ("r_hi", C.c_float), ("l_max", C.c_float),
                ("step", C.c_int32)]


class WindowOpts(C.Structure):
    _fields_ = [("a_lo", C.c_float), ("a_hi", C.c_float), ("l_max", C.c_float),
                ("r0_first", C.c_float), ("r0_last", C.c_float), ("r_lo_frac", C.c_float),
                ("r_hi_frac", C.c_float), ("lambda_length", C.c_float),
                ("lambda_area", C.c_float)]


class FitJob(C.Structure):
    _fields_ = [("n_strokes", C.c_int32), ("n_palette", C.c_int32), ("params", C.c_void_p),
                ("grads", C.c_void_p), ("adam_m", C.c_void_p), ("adam_v", C.c_void_p),
                ("target_rgb", C.c_void_p), ("loss", C.c_void_p), ("opts", RenderOpts),
                ("adam", AdamOpts)]


class ServeOpts(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("max_queue", C.c_int32), ("max_tick_items", C.c_int32), ("streams", C.c_int32),
                ("fake_device", C.c_int32), ("fake_ns_per_pixel_stroke", C.c_float),
                ("fake_fail_launch", C.c_int32), ("solo_tiles", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("program_id", C.c_uint64), ("mode", C.c_int32), ("width", C.c_int32),
                ("height", C.c_int32), ("tau", C.c_float), ("tau_min", C.c_float),
                ("tau_c", C.c_float), ("eps_floor", C.c_float), ("rgb", C.c_void_p),
                ("label", C.c_void_p), ("owner", C.c_void_p), ("arena_outputs", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double), ("pixel_strokes", C.c_int64),
                ("rgb", C.c_void_p), ("label", C.c_void_p), ("owner", C.c_void_p)]


class ServeStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("cancelled", C.c_int64),
                ("launches", C.c_int64), ("pixel_strokes", C.c_int64), ("queued", C.c_int64),
                ("in_flight", C.c_int64), ("arena_used", C.c_size_t),
                ("arena_bytes", C.c_size_t)]


# Every exported symbol of include/tbr.h, with its ctypes signature.
_vp, _sz, _i32 = C.c_void_p, C.c_size_t, C.c_int32
SIGNATURES = {
    "tbr_render_workspace_bytes": (_sz, [_vp, _i32, _i32, _i32]),
    "tbr_render": (_i32, [_vp, _vp, _i32, _vp, _vp, _vp, _vp, _sz, _i32, _vp]),
    "tbr_render_static": (_i32, [_vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    "tbr_tape_records": (_i32, [_vp, _sz, _vp, _i32, _vp, _vp]),
    "tbr_backward_workspace_bytes": (_sz, [_vp, _i32, _i32]),
    "tbr_render_backward": (_i32, [_vp, _vp, _vp, _sz, _vp, _vp, _vp, _sz, _vp]),
    "tbr_fit_workspace_bytes": (_sz, [_vp, _i32, _i32]),
    "tbr_fit_step": (_i32, [_i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "tbr_set_timing_events": (_i32, [C.c_char_p, _vp, _vp]),
    "tbr_fit_multi_workspace_bytes": (_sz, [_vp, _i32]),
    "tbr_fit_multi_step": (_i32, [_vp, _i32, _vp, _sz, _vp]),
    "tbr_fit_multi_records": (_i32, [_vp, _i32, _vp, _sz, _vp, _vp]),
    "tbr_coupling_check": (_i32, [_vp, _i32, _vp]),
    "tbr_compensate_workspace_bytes": (_sz, [_i32, _i32]),
    "tbr_compensate": (_i32, [_vp, C.c_float, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "tbr_window_map": (_i32, [_i32, _i32, _vp, _vp, _vp, _vp]),
    "tbr_fit_loop_step": (_i32, [_i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                 _vp, _sz, _vp]),
    "tbr_schedule_at": (None, [_i32, _i32, C.c_float, C.c_float, C.c_float, C.c_float, _vp, _vp,
                               _vp]),
    "tbr_serve_program_bytes": (_sz, [_i32, _i32]),
    "tbr_serve_request_bytes": (_sz, [_i32]),
    "tbr_serve_tick_bytes": (_sz, [_vp]),
    "tbr_serve_output_bytes": (_sz, [_i32, _i32, _i32]),
    "tbr_serve_create": (_i32, [_vp, _vp]),
    "tbr_serve_register_program": (_i32, [_vp, _vp, _vp]),
    "tbr_serve_submit": (_i32, [_vp, _vp, _vp]),
    "tbr_serve_poll": (_i32, [_vp, C.c_uint64, _vp]),
    "tbr_serve_cancel": (_i32, [_vp, C.c_uint64]),
    "tbr_serve_release": (_i32, [_vp, C.c_uint64]),
    "tbr_serve_get_stats": (_i32, [_vp, _vp]),
    "tbr_serve_destroy": (None, [_vp]),
    "tbr_serve_now": (C.c_double, []),
    "tbr_last_error": (C.c_char_p, []),
    "tbr_version": (C.c_char_p, []),
}

_lib = None


def load():
    """Load libtbr.so; raise if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2609_08722_amd.build` (hipcc, gfx950)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int) -> int:
    if status < 0:
        raise TbrError(status, load().tbr_last_error().decode())
    return status
