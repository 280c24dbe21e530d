"""ctypes binding of the C ABI in include/gs.h (argument marshalling only).

Every function here has the name and argument order of its C counterpart;
the structs mirror the C structs field by field.  Loading fails loudly
when the HIP library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# GSMI_LIB names another build of the same library (the sanitized host build)
LIB_PATH = os.environ.get("GSMI_LIB") or os.path.join(HERE, "libgsmi.so")

GS_OK = 0
GS_ERR_INVALID = -1
GS_ERR_OOM = -2
GS_ERR_HIP = -3
GS_ERR_CAPACITY = -4
GS_ERR_BUSY = -5
GS_ERR_UNSUPPORTED = -6
GS_ERR_TIMEOUT = -7
GS_ERR_NOT_FOUND = -8

STATUS_NAMES = {0: "GS_OK", -1: "GS_ERR_INVALID", -2: "GS_ERR_OOM", -3: "GS_ERR_HIP", -4: "GS_ERR_CAPACITY",
                -5: "GS_ERR_BUSY", -6: "GS_ERR_UNSUPPORTED", -7: "GS_ERR_TIMEOUT", -8: "GS_ERR_NOT_FOUND"}

P = C.c_void_p
REC_BYTES = 48


class GsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class gs_gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("ld", C.c_int64), ("sh_degree", C.c_int32),
                ("mean", P), ("scale", P), ("quat", P), ("opacity", P), ("sh", P)]


class gs_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("near_z", C.c_float), ("bg", C.c_float * 3)]


class gs_opts(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("reserved", C.c_int32 * 6)]


class gs_proj(C.Structure):
    _fields_ = [("rec", P), ("depth", P), ("rect", P), ("tiles_touched", P)]


class gs_bins(C.Structure):
    _fields_ = [("keys", P), ("vals", P), ("first", P), ("ranges", P), ("pair_count", P), ("status", P),
                ("pair_capacity", C.c_int64), ("cell_masks", P), ("tile_order", P)]


class gs_grads(C.Structure):
    _fields_ = [("ld", C.c_int64), ("mean", P), ("scale", P), ("quat", P), ("opacity", P), ("sh", P),
                ("grad2d", P)]


class gs_params(C.Structure):
    _fields_ = [("n", C.c_int64), ("ld", C.c_int64), ("sh_degree", C.c_int32), ("mean", P), ("log_scale", P),
                ("quat", P), ("logit_opacity", P), ("sh", P)]


class gs_adam_state(C.Structure):
    _fields_ = [("m", P), ("v", P), ("grad_accum", P), ("visible_count", P)]


class gs_adam_config(C.Structure):
    _fields_ = [("lr_mean", C.c_float), ("lr_scale", C.c_float), ("lr_quat", C.c_float), ("lr_opacity", C.c_float),
                ("lr_sh_dc", C.c_float), ("lr_sh_rest", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("step", C.c_int32)]


class gs_partition_config(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("expand", C.c_float), ("visibility_threshold", C.c_float)]


_lib = None

# name -> (argtypes); every function returns gs_status (int) unless listed
_SIGS = {
    "gs_abi_version": [],
    "gs_last_error": [],
    "gs_project": [C.POINTER(gs_gaussians), C.POINTER(gs_camera), C.POINTER(gs_opts), C.POINTER(gs_proj), P],
    "gs_bin_sort_workspace": [C.c_int64, C.c_int64, C.c_int64, C.POINTER(C.c_size_t)],
    "gs_bin_sort": [C.POINTER(gs_proj), C.c_int64, C.POINTER(gs_camera), C.POINTER(gs_opts), C.POINTER(gs_bins),
                    P, C.c_size_t, P],
    "gs_render_fwd": [C.POINTER(gs_proj), C.POINTER(gs_bins), C.POINTER(gs_camera), C.POINTER(gs_opts), P, P, P, P],
    "gs_render_bwd_workspace": [C.POINTER(gs_bins), C.POINTER(C.c_size_t)],
    "gs_render_bwd": [C.POINTER(gs_gaussians), C.POINTER(gs_camera), C.POINTER(gs_opts), C.POINTER(gs_proj),
                      C.POINTER(gs_bins), P, P, P, C.POINTER(gs_grads), P, C.c_size_t, P],
    "gs_sort_workspace": [C.c_int64, C.c_int32, C.POINTER(C.c_size_t)],
    "gs_sort_pairs": [P, P, P, C.c_int64, C.c_int32, P, C.c_size_t, P],
    "gs_render_state_bytes": [C.POINTER(gs_bins), C.POINTER(gs_opts), C.POINTER(C.c_size_t)],
    "gs_render_mask_bytes": [C.POINTER(gs_bins), C.POINTER(gs_opts), C.POINTER(C.c_size_t)],
    "gs_render_fwd_stored": [C.POINTER(gs_proj), C.POINTER(gs_bins), C.POINTER(gs_camera), C.POINTER(gs_opts),
                             P, P, P, P, C.c_size_t, P],
    "gs_render_bwd_stored": [C.POINTER(gs_gaussians), C.POINTER(gs_camera), C.POINTER(gs_opts), C.POINTER(gs_proj),
                             C.POINTER(gs_bins), P, P, P, C.c_size_t, P, C.POINTER(gs_grads), P, C.c_size_t,
                             P],
    "gs_render_stats": [C.POINTER(gs_proj), C.POINTER(gs_bins), C.POINTER(gs_camera), C.POINTER(gs_opts), P, P],
    "gs_loss_workspace": [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)],
    "gs_loss": [P, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, P, P, C.c_size_t, P],
    "gs_loss_noalloc": [P, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, P, P],
    "gs_adam_step": [C.POINTER(gs_params), P, P, C.POINTER(gs_adam_state), C.POINTER(gs_grads), P, P,
                     C.POINTER(gs_adam_config), P],
    "gs_partition_views": [P, C.c_int32, P, C.c_int64, C.POINTER(gs_partition_config), P, P, P, P, P],
    "gs_select_points_workspace": [C.c_int32, C.c_int32, C.c_int64, C.POINTER(C.c_size_t)],
    "gs_select_points": [P, C.c_int64, C.c_int64, P, C.c_int32, P, C.c_int32, P, P, P, P, C.c_size_t, P],
    "gs_merge_keep": [P, C.c_int64, C.c_int64, P, C.c_int32, C.c_int32, P, P],
    "gs_appearance_param_count": [C.c_int32, C.POINTER(C.c_int64)],
    "gs_appearance_workspace": [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)],
    "gs_appearance_fwd": [P, C.c_int32, C.c_int32, P, C.c_int32, P, P, P, P, C.c_size_t, P],
    "gs_appearance_bwd": [P, C.c_int32, C.c_int32, P, C.c_int32, P, P, P, P, P, P, C.c_size_t, P],
    "gs_profile_enable": [C.c_int],
    "gs_profile_select": [C.c_char_p],
    "gs_profile_report": [C.c_char_p, C.c_size_t],
}
_RESTYPES = {"gs_last_error": C.c_char_p, "gs_abi_version": C.c_int}
_OPTIONAL = {}


def register(name, argtypes, restype=C.c_int):
    """Declare a further exported function (used by the batch/serve modules)."""
    _SIGS[name] = argtypes
    _RESTYPES[name] = restype
    if _lib is not None:
        _bind(_lib, name)


def _bind(L, name):
    f = getattr(L, name)
    f.argtypes = _SIGS[name]
    f.restype = _RESTYPES.get(name, C.c_int)


def lib():
    """Load libgsmi.so (raises if it is missing: the HIP path is the only path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2402_17427_amd.build.build() "
                               "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        for name in _SIGS:
            _bind(L, name)
        _lib = L
    return _lib


def check(code: int) -> None:
    if code != GS_OK:
        msg = lib().gs_last_error()
        raise GsError(code, msg.decode() if msg else "")


def call(name: str, *args) -> None:
    check(getattr(lib(), name)(*args))


def make_camera(cam) -> gs_camera:
    """gs_camera from any object with R (9), t (3), fx, fy, cx, cy, width,
    height, near, bg (3)."""
    c = gs_camera()
    R = [float(x) for x in (cam.R.reshape(-1) if hasattr(cam.R, "reshape") else cam.R)]
    t = [float(x) for x in (cam.t.reshape(-1) if hasattr(cam.t, "reshape") else cam.t)]
    c.R[:] = R
    c.t[:] = t
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.near_z = float(getattr(cam, "near", getattr(cam, "near_z", 0.2)))
    c.bg[:] = [float(b) for b in cam.bg]
    return c


def make_opts(tile_w=16, tile_h=16) -> gs_opts:
    o = gs_opts()
    o.tile_w, o.tile_h = int(tile_w), int(tile_h)
    return o


def profile_enable(on: bool) -> None:
    call("gs_profile_enable", 1 if on else 0)


def profile_select(stages=None) -> None:
    """Bracket only the named stages (None: all)."""
    call("gs_profile_select", ",".join(stages).encode() if stages else None)


def profile_report() -> dict:
    """{stage: (total_ms, launches)} of the events recorded since the last
    report (waits for them)."""
    import json
    buf = C.create_string_buffer(1 << 16)
    call("gs_profile_report", buf, len(buf))
    return {k: (float(v[0]), int(v[1])) for k, v in json.loads(buf.value.decode()).items()}
