"""ctypes view of libtomo.so (the C ABI declared in include/tomo.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any operation.
"""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtomo.so")

TOMO_OK, TOMO_EINVAL, TOMO_ENOMEM, TOMO_EHIP, TOMO_EBUSY, TOMO_ENOENT, TOMO_EAGAIN, TOMO_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "TOMO_OK", -1: "TOMO_EINVAL", -2: "TOMO_ENOMEM", -3: "TOMO_EHIP",
                -4: "TOMO_EBUSY", -5: "TOMO_ENOENT", -6: "TOMO_EAGAIN", -7: "TOMO_ESTATE"}

ROI_TV_NONNEG_CP, ROI_NONNEG_SIRT, ROI_LOCAL_SIRT, ROI_LOCAL_FISTA_TV, ROI_LOCAL_FISTA_HAAR = 0, 1, 2, 3, 4
ROI_FLAG_HALF_DATA, ROI_FLAG_ANISO_TV, ROI_FLAG_BOX, ROI_FLAG_NO_MOMENTUM = 1, 2, 4, 8
ROI_FLAG_PIXEL_UNITS = 16


class tomo_rect(C.Structure):
    _fields_ = [("row0", C.c_int32), ("col0", C.c_int32), ("rows", C.c_int32),
                ("cols", C.c_int32)]


class roi_params(C.Structure):
    _fields_ = [("roi", tomo_rect), ("margin", C.c_int32), ("method", C.c_int32),
                ("lambda_", C.c_float), ("iters", C.c_int32), ("sigma", C.c_float),
                ("tau", C.c_float), ("flags", C.c_uint32), ("box_lo", C.c_float),
                ("box_hi", C.c_float), ("inner_iters", C.c_int32)]


class tomo_launch(C.Structure):
    _fields_ = [("fp_segments", C.c_int32), ("fp_rays_per_lane", C.c_int32),
                ("fp_xcd_order", C.c_int32),
                ("bp_variant", C.c_int32), ("bp_groups", C.c_int32),
                ("bp_pixels_per_thread", C.c_int32), ("bp_xcd_order", C.c_int32)]


# name -> (restype, argtypes), mirroring include/tomo.h
_P = C.c_void_p
_I = C.c_int32
SIGNATURES = {
    "tomo_create": (C.c_int, [C.c_int, _P, C.c_size_t, C.POINTER(_P)]),
    "tomo_destroy": (C.c_int, [_P]),
    "tomo_last_error": (C.c_char_p, [_P]),
    "tomo_set_geometry": (C.c_int, [_P, _I, _I, _I, C.POINTER(C.c_double), C.c_double,
                                    C.c_double, C.POINTER(_I)]),
    "tomo_roi_band": (C.c_int, [_P, _I, tomo_rect, C.POINTER(_I), C.POINTER(_I)]),
    "tomo_roi_ext": (C.c_int, [_P, _I, tomo_rect, _I, C.POINTER(tomo_rect)]),
    "tomo_fp": (C.c_int, [_P, _I, tomo_rect, _P, _P, C.c_int, _P]),
    "tomo_bp": (C.c_int, [_P, _I, tomo_rect, _P, _P, C.c_int, _P]),
    "tomo_fbp_ramlak": (C.c_int, [_P, _I, _P, _P, _P]),
    "tomo_fbp_ramlak_noalloc": (C.c_int, [_P, _I, _P, _P, _P]),
    "tomo_exterior_subtract": (C.c_int, [_P, _I, tomo_rect, _P, _P, _P, _P]),
    "roi_solve": (C.c_int, [_P, _I, _P, _P, C.POINTER(roi_params), _P, _P]),
    "roi_solve_batch": (C.c_int, [_P, _I, _P, _P, _I, C.POINTER(roi_params), C.POINTER(_P), _P]),
    "roi_solve_stitched": (C.c_int, [_P, _I, _P, _P, _I, C.POINTER(roi_params), _P, _I, _P]),
    "roi_step_size": (C.c_int, [_P, _I, tomo_rect, C.POINTER(C.c_float)]),
    "roi_state_bytes": (C.c_int, [_P, _I, C.POINTER(roi_params), C.POINTER(C.c_size_t)]),
    "roi_solve_resume": (C.c_int, [_P, _I, _P, _P, C.POINTER(roi_params), _I, _P, _P, _P]),
    "tomo_sirt_filters": (C.c_int, [_P, _I, _I, _P, _P]),
    "tomo_sirt_filter_sino": (C.c_int, [_P, _I, _P, _I, _P, _P, _P]),
    "roi_solve_local": (C.c_int, [_P, _I, _P, _I, _I, C.POINTER(roi_params), C.POINTER(_P), _P]),
    "tomo_disc_subtract": (C.c_int, [_P, _I, _P, _P, _P, _P]),
    "tomo_disc_add": (C.c_int, [_P, _I, tomo_rect, _P, _P, _P]),
    "tomo_pad_truncated": (C.c_int, [_P, _I, _P, _I, _I, _P, _P]),
    "tomo_register_sinogram": (C.c_int, [_P, _I, _P, C.POINTER(_I)]),
    "tomo_unregister_sinogram": (C.c_int, [_P, _I]),
    "roi_submit": (C.c_int, [_P, _I, C.POINTER(roi_params), _P, C.POINTER(C.c_uint64)]),
    "roi_poll": (C.c_int, [_P, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_float)]),
    "roi_poll_stages": (C.c_int, [_P, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_float)]),
    "tomo_serving_config": (C.c_int, [_P, _I, _I]),
    "tomo_serving_fake": (C.c_int, [_P, C.c_size_t, _I]),
    "tomo_set_launch": (C.c_int, [_P, C.POINTER(tomo_launch)]),
    "tomo_get_launch": (C.c_int, [_P, C.POINTER(tomo_launch)]),
    "tomo_resolve_launch": (C.c_int, [_P, _I, _I, C.POINTER(roi_params), C.POINTER(tomo_launch)]),
    "tomo_autotune": (C.c_int, [_P, _I, _P, _P, _I, C.POINTER(roi_params), C.POINTER(_P), _P,
                                C.POINTER(tomo_launch), C.POINTER(C.c_float)]),
    "tomo_set_graphs": (C.c_int, [_P, C.c_int]),
    "tomo_roi_nnz": (C.c_int, [_P, _I, tomo_rect, C.POINTER(C.c_int64)]),
    "tomo_kernel_timing": (C.c_int, [_P, C.c_int]),
    "tomo_kernel_time": (C.c_int, [_P, _I, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.c_int]),
    "tomo_valu_probe": (C.c_int, [_P, _I, _I, _I, C.c_float, C.c_float, _P, _P]),
    "tomo_workspace_usage": (C.c_int, [_P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "tomo_synchronize": (C.c_int, [_P]),
}

_lib = None


def load():
    """Load libtomo.so and attach the prototypes; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -m paper_1604_02292_amd.build` "
            "(there is no non-HIP fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
