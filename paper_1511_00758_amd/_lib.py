"""ctypes binding of libstereomesh.so (the C ABI in include/stereomesh.h).

Argument marshalling only. Loading fails loudly when the library has not been
built: there is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstereomesh.so")

c_i16, c_i32, c_i64, c_f32 = ctypes.c_int16, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
c_vp, c_size = ctypes.c_void_p, ctypes.c_size_t

SM_OK, SM_ERR_ARG, SM_ERR_CAPACITY, SM_ERR_HIP, SM_ERR_INTERNAL = 0, -1, -2, -3, -4
STATUS_NAMES = {0: "SM_OK", -1: "SM_ERR_ARG", -2: "SM_ERR_CAPACITY", -3: "SM_ERR_HIP",
                -4: "SM_ERR_INTERNAL"}
# sm_stage indices of sm_stats.stage_us / stage_launches
STAGES = {"census": 0, "match": 1, "compact": 2, "raster": 3, "validate": 4, "rematch": 5,
          "fast": 6, "mesh": 7, "host_triangulate": 12, "host_copies": 13, "total": 14}
N_STAGES = 16
TIME_SELECTED = 0x40000000
NOALLOC_MAX_BYTES = 48 << 20   # SM_NOALLOC_MAX_BYTES


def timing_flag(timing) -> int:
    """sm_stats.timing from True/False or an iterable of stage names to time alone."""
    if timing is True:
        return 1
    if not timing:
        return 0
    flag = TIME_SELECTED
    for name in timing:
        flag |= 1 << STAGES[name]
    return flag


class SmSupport(ctypes.Structure):
    _fields_ = [("u", c_i16), ("v", c_i16), ("d", c_f32)]


class SmTri(ctypes.Structure):
    _fields_ = [("i0", c_i32), ("i1", c_i32), ("i2", c_i32)]


PARAM_FIELDS = ("d_min", "d_max", "census_w", "census_h", "support_step", "n_iters", "t_hi",
                "t_lo", "grad_thr", "lr_tol", "uniqueness", "sz_occ0", "support_mode",
                "fast_threshold", "fast_bins_x", "fast_bins_y", "fast_per_bin", "levels", "host_mesh")
# the paper-variant fields default to the grid candidates and Alg. 2's single level
PARAM_DEFAULTS = {"support_mode": 0, "fast_threshold": 16, "fast_bins_x": 12, "fast_bins_y": 10,
                  "fast_per_bin": 25, "levels": 1, "host_mesh": 0}


class SmParams(ctypes.Structure):
    _fields_ = [(f, c_i32) for f in PARAM_FIELDS]


class SmStats(ctypes.Structure):
    _fields_ = [("timing", c_i32), ("n_support", c_i32 * 8), ("n_tris", c_i32 * 8),
                ("n_valid", c_i64), ("stage_us", c_f32 * N_STAGES),
                ("stage_launches", c_i32 * N_STAGES), ("mesh_device", c_i32),
                ("mesh_fallback", c_i32)]


class SmFrame(ctypes.Structure):
    _fields_ = [("L", c_vp), ("R", c_vp), ("W", c_i32), ("H", c_i32), ("stride", c_i32),
                ("p", SmParams), ("D_f", c_vp), ("C_f", c_vp), ("mask", c_vp),
                ("status", c_i32), ("worker", c_i32), ("latency_us", c_f32)]


EXPORTS = ("sm_census", "sm_match_support", "sm_grid_candidates", "sm_fast_candidates", "sm_triangulate",
           "sm_interpolate", "sm_cells", "sm_validate", "sm_resample",
           "sm_solve_workspace_bytes", "sm_solve", "sm_solve_noalloc", "sm_solve_batch", "sm_solve_many_workspace_bytes",
           "sm_solve_many", "sm_solve_many_capture", "sm_many_graph_run", "sm_many_graph_destroy", "sm_autotune",
           "sm_set_launch_shape", "sm_last_error", "sm_version")


class StereoMeshError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load():
    """Load the library (once) and declare every signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1511_00758_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "sm_census": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp]),
        "sm_match_support": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_i32, c_vp, c_i32, P(SmParams),
                                     c_vp, c_i32, c_vp, c_vp]),
        "sm_grid_candidates": (c_i32, [c_i32, c_i32, c_i32]),
        "sm_fast_candidates": (c_i32, [c_vp, c_i32, c_i32, c_i32, P(SmParams), c_vp, c_vp, c_i32, c_vp,
                                       c_vp]),
        "sm_triangulate": (c_i32, [c_vp, c_i32, c_vp, c_i32, P(c_i32)]),
        "sm_interpolate": (c_i32, [c_vp, c_i32, c_vp, c_i32, c_i32, c_i32, c_vp, c_vp]),
        "sm_cells": (c_i32, [c_i32, c_i32, c_i32]),
        "sm_validate": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i32, c_i32, P(SmParams), c_i32, c_vp,
                                c_vp, c_vp, c_vp, c_vp, c_vp]),
        "sm_resample": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_i32, c_i32, P(SmParams),
                                c_vp, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp]),
        "sm_solve_workspace_bytes": (c_size, [c_i32, c_i32, P(SmParams)]),
        "sm_solve": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, P(SmParams), c_vp, c_size, c_vp,
                             c_vp, c_vp, P(SmStats), c_vp]),
        "sm_solve_noalloc": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, P(SmParams), c_vp, c_vp, c_vp,
                                     P(SmStats), c_vp]),
        "sm_solve_batch": (c_i32, [P(SmFrame), c_i32, P(c_vp), P(c_vp), P(c_size), c_i32,
                                   P(SmStats)]),
        "sm_solve_many_workspace_bytes": (c_size, [P(SmFrame), c_i32]),
        "sm_solve_many": (c_i32, [P(SmFrame), c_i32, c_vp, c_size, c_i32, P(SmStats), c_vp]),
        "sm_solve_many_capture": (c_i32, [P(SmFrame), c_i32, c_vp, c_size, P(SmStats), c_vp, P(c_vp)]),
        "sm_many_graph_run": (c_i32, [c_vp, P(SmStats), c_vp]),
        "sm_many_graph_destroy": (None, [c_vp]),
        "sm_set_launch_shape": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_i32]),
        "sm_autotune": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, P(SmParams), c_vp, c_size, c_vp, c_vp, c_vp,
                                P(c_i32), c_vp]),
        "sm_last_error": (ctypes.c_char_p, []),
        "sm_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status):
    if status != SM_OK:
        msg = load().sm_last_error().decode(errors="replace")
        raise StereoMeshError(status, msg)
    return status


def make_params(d=None, **kw) -> SmParams:
    vals = dict(PARAM_DEFAULTS)
    vals.update(d or {})
    vals.update(kw)
    p = SmParams()
    for f in PARAM_FIELDS:
        if f not in vals:
            raise KeyError(f"missing parameter {f}")
        setattr(p, f, int(vals[f]))
    return p
