"""ctypes binding of the C ABI in include/rt.h (argument marshalling only).

Loads ``librt_mi355x.so`` built by ``paper_2303_11103_amd.build``.  There is
no fallback: if the library is missing or cannot be loaded, importing this
module raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librt_mi355x.so")

RT_OK = 0
RT_ERR_ARG = -1
RT_ERR_CAPACITY = -2
RT_ERR_DEVICE = -3
RT_ERR_OOM = -4

RT_PATTERN_ISO = 0
RT_PATTERN_TR38901 = 1
RT_POL_V = 0


class rt_material(ctypes.Structure):
    _fields_ = [("eps_r", ctypes.c_float), ("sigma", ctypes.c_float)]


class rt_device(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_float * 3), ("yaw", ctypes.c_float), ("pitch", ctypes.c_float),
                ("roll", ctypes.c_float), ("pattern", ctypes.c_int32), ("pol", ctypes.c_int32)]


class rt_trace_params(ctypes.Structure):
    _fields_ = [("freq_hz", ctypes.c_double), ("max_depth", ctypes.c_int32), ("max_paths_per_rx", ctypes.c_int32),
                ("num_rays", ctypes.c_int64), ("t_min", ctypes.c_double), ("ray_begin", ctypes.c_int64),
                ("ray_stride", ctypes.c_int64), ("cand_mode", ctypes.c_int32), ("sphere_kappa", ctypes.c_float)]


class rt_grid(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("cell", ctypes.c_double), ("z", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32)]


class rt_mlp_config(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("ff_scale", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("in_center", ctypes.c_float * 5), ("in_half", ctypes.c_float * 5), ("ff_scale_cell", ctypes.c_float),
                ("prior_rx_z", ctypes.c_float), ("prior_freq_hz", ctypes.c_double), ("ff_rows_tx", ctypes.c_int32),
                ("ff_rows_rel", ctypes.c_int32), ("ff_scale_rel", ctypes.c_float), ("reserved", ctypes.c_int32)]


class rt_scene_info_t(ctypes.Structure):
    _fields_ = [("num_triangles", ctypes.c_int64), ("num_faces", ctypes.c_int32), ("num_materials", ctypes.c_int32),
                ("bvh_nodes", ctypes.c_int64), ("bvh_depth", ctypes.c_int32), ("num_wedges", ctypes.c_int32),
                ("build_ms", ctypes.c_double)]


P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64

# name -> argument types (all return rt_status unless listed in _RESTYPE)
SIGNATURES = {
    "rt_create": [ctypes.POINTER(P), I32],
    "rt_destroy": [P],
    "rt_set_stream": [P, P],
    "rt_synchronize": [P],
    "rt_last_error": [],
    "rt_scene_create": [P, P, I64, P, I64, P, P, I32, ctypes.POINTER(P)],
    "rt_scene_set_scattering": [P, P, I32, ctypes.c_uint64],
    "rt_scene_set_materials": [P, P, I32],
    "rt_scene_info": [P, ctypes.POINTER(rt_scene_info_t)],
    "rt_scene_face_ids": [P, P],
    "rt_scene_destroy": [P],
    "rt_fibonacci_directions": [P, I64, I64, I64, I64, P],
    "rt_trace_record": [P, P, ctypes.POINTER(rt_trace_params), ctypes.POINTER(rt_device), P, P],
    "rt_coverage_maps": [P, P, ctypes.POINTER(rt_trace_params), P, I32, ctypes.POINTER(rt_device),
                         ctypes.POINTER(rt_grid), P, P, P],
    "rt_coverage_map": [P, P, ctypes.POINTER(rt_trace_params), ctypes.POINTER(rt_device), ctypes.POINTER(rt_device),
                        ctypes.POINTER(rt_grid), P, P, P, P],
    "rt_coverage_work": [P, P, ctypes.POINTER(rt_trace_params), ctypes.POINTER(rt_device), ctypes.POINTER(rt_device),
                         ctypes.POINTER(rt_grid), P, P, P],
    "rt_coverage_map_noalloc": [P, P, ctypes.POINTER(rt_trace_params), ctypes.POINTER(rt_device),
                                ctypes.POINTER(rt_device), ctypes.POINTER(rt_grid), P, P, P, P],
    "rt_profile_enable": [P, I32],
    "rt_profile_read": [P, I32, P, P],
    "rt_compute_paths": [P, P, ctypes.POINTER(rt_trace_params), P, I32, P, I32, P, P, P, P, P, P, P, P],
    "rt_last_candidate_count": [P, ctypes.POINTER(I64)],
    "rt_scene_wedges": [P, I32, P, ctypes.POINTER(I32)],
    "rt_coverage_diffraction": [P, P, ctypes.c_double, ctypes.POINTER(rt_device), ctypes.POINTER(rt_device),
                                ctypes.POINTER(rt_grid), P],
    "rt_compute_diffraction": [P, P, ctypes.c_double, P, I32, P, I32, I32, P, P, P, P, P, P, P],
    "rt_compute_scattering": [P, P, ctypes.POINTER(rt_trace_params), P, I32, P, I32, I64, P, P, P, P, P, P, P, P,
                              P],
    "rt_paths_power": [P, P, P, I64, I32, P],
    "rt_paths_power_grad": [P, P, ctypes.POINTER(rt_trace_params), ctypes.POINTER(rt_device), P, I32, I32, P, P,
                            P, P],
    "rt_paths_coef_grad": [P, P, ctypes.POINTER(rt_trace_params), ctypes.POINTER(rt_device), P, I32, I32, P, P,
                           P, P],
    "rt_paths_cfr": [P, I32, I32, I32, P, P, P, P, P, ctypes.c_double, I32, ctypes.c_double, I32, P, I32, P, P, P,
                     I32, ctypes.c_double, P],
    "rt_paths_cfr_adjoint": [P, I32, I32, I32, P, P, P, P, P, ctypes.c_double, I32, ctypes.c_double, I32, P, I32, P,
                             P, P, I32, ctypes.c_double, P, P],
    "rt_coverage_grad": [P, P, ctypes.POINTER(rt_trace_params), ctypes.POINTER(rt_device), ctypes.POINTER(rt_device),
                         ctypes.POINTER(rt_grid), P, P, P, P],
    "rt_mlp_param_count": [ctypes.POINTER(I64)],
    "rt_mlp_create": [P, ctypes.POINTER(rt_mlp_config), ctypes.POINTER(P)],
    "rt_mlp_destroy": [P],
    "rt_mlp_get_params": [P, P, P],
    "rt_mlp_set_params": [P, P, P],
    "rt_mlp_forward": [P, P, I64, P],
    "rt_mlp_grad": [P, P, P, P, I64, P, P],
    "rt_mlp_train_step": [P, P, P, P, I64, ctypes.c_float, P],
    "rt_mlp_valid_index": [P, P, I64, P, I64, ctypes.POINTER(I64)],
    "rt_mlp_sample_batch": [P, P, P, I64, P, I32, ctypes.POINTER(rt_grid), ctypes.c_uint64, ctypes.c_uint64, P, P, P,
                            I64],
    "rt_mlp_predict_maps": [P, P, I32, ctypes.POINTER(rt_grid), P],
    "rt_mlp_predict_maps_fallback": [P, P, ctypes.POINTER(rt_trace_params), P, I32, ctypes.POINTER(rt_device),
                                     ctypes.POINTER(rt_grid), P, P, ctypes.POINTER(I64)],
}
_RESTYPE = {"rt_last_error": ctypes.c_char_p}


class RTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("rt error %d: %s" % (code, msg))
        self.code = code


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("HIP library %s is not built; run `python paper_2303_11103_amd/build.py`" % path)
    lib = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = _RESTYPE.get(name, ctypes.c_int32)
    return lib


lib = load()


def check(code: int):
    if code != RT_OK:
        raise RTError(code, lib.rt_last_error().decode(errors="replace"))
    return code
