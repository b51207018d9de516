"""ctypes loader of libmnfpty.so: structure layouts and function signatures
of the C ABI declared in include/mnfpty.h.  No computation happens here."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int, c_int32, c_uint16, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmnfpty.so")

MNF_OK = 0
MNF_EINVAL = -1
MNF_EUNSUPPORTED = -2
MNF_EHIP = -3
MNF_ENOMEM = -4
MNF_ENONFINITE = -5
MNF_EDIVERGED = -6

ERROR_NAMES = {MNF_EINVAL: "MNF_EINVAL", MNF_EUNSUPPORTED: "MNF_EUNSUPPORTED",
               MNF_EHIP: "MNF_EHIP", MNF_ENOMEM: "MNF_ENOMEM", MNF_ENONFINITE: "MNF_ENONFINITE",
               MNF_EDIVERGED: "MNF_EDIVERGED"}


class FuseParamsC(ctypes.Structure):
    _fields_ = [("levels", c_int32), ("mu", c_float), ("sigma", c_float), ("sat", c_float),
                ("dark", c_float), ("delta", c_float * 16), ("radiometric", c_int32), ("contrast_exp", c_float)]


class PtychoParamsC(ctypes.Structure):
    _fields_ = [("alg", c_int32), ("alpha", c_float), ("beta", c_float), ("batch", c_int32),
                ("update_probe", c_int32), ("probe_start_iter", c_int32), ("it0", c_int32),
                ("graph", c_int32)]


class UnetShapeC(ctypes.Structure):
    _fields_ = [("H", c_int32), ("widths", c_int32 * 4)]


class PtychoScanC(ctypes.Structure):
    _fields_ = [("O", c_void_p), ("My", c_int32), ("Mx", c_int32), ("P", c_void_p), ("Nw", c_int32),
                ("I", c_void_p), ("Nd", c_int32), ("pos", POINTER(c_int32)), ("J", c_int32),
                ("order", POINTER(c_int32)), ("err_out", c_void_p)]


# name -> (restype, argtypes)
SIGNATURES = {
    "mnf_create": (c_int, [POINTER(c_void_p), c_int]),
    "mnf_destroy": (None, [c_void_p]),
    "mnf_last_error": (ctypes.c_char_p, [c_void_p]),
    "mnf_status": (c_int, [c_void_p, c_void_p]),
    "mnf_supported_sizes": (c_int, [POINTER(c_int32), c_int]),
    "fuse_exposures": (c_int, [c_void_p, c_void_p, POINTER(c_float), c_int, c_int, c_int, c_int,
                               POINTER(FuseParamsC), c_void_p, c_void_p, c_void_p]),
    "fuse_linear": (c_int, [c_void_p, c_void_p, POINTER(c_float), c_int, c_int, c_int, c_int, c_float, c_float,
                            c_int, c_void_p, c_void_p]),
    "ptycho_forward": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_int, c_int,
                               POINTER(c_int32), c_int, c_void_p, c_void_p]),
    "ptycho_iterate": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_int, c_void_p, c_int,
                               POINTER(c_int32), c_int, POINTER(c_int32), c_int,
                               POINTER(PtychoParamsC), c_void_p, c_void_p]),
    "ptycho_forward_subpixel": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_int, c_int,
                                        POINTER(c_float), c_int, c_void_p, c_void_p]),
    "ptycho_iterate_noalloc": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_int, c_void_p, c_int,
                                       POINTER(c_int32), c_int, POINTER(c_int32), c_int,
                                       POINTER(PtychoParamsC), c_void_p, c_void_p]),
    "ptycho_iterate_subpixel": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_int, c_void_p, c_int,
                                        POINTER(c_float), c_int, POINTER(c_int32), c_int,
                                        POINTER(PtychoParamsC), c_void_p, c_void_p]),
    "ptycho_forward_modes": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_int, c_int, c_int,
                                     POINTER(c_int32), c_int, c_void_p, c_void_p]),
    "ptycho_iterate_modes": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_int, c_int, c_void_p, c_int,
                                     POINTER(c_int32), c_int, POINTER(c_int32), c_int,
                                     POINTER(PtychoParamsC), c_void_p, c_void_p]),
    "ptycho_iterate_many": (c_int, [c_void_p, POINTER(PtychoScanC), c_int, c_int, POINTER(PtychoParamsC),
                                    c_void_p]),
    "ptycho_grad": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_int, c_void_p, c_int,
                            POINTER(c_int32), c_int, c_int, c_float, c_int, c_void_p,
                            c_void_p, c_void_p, c_void_p, c_void_p]),
    "ptycho_plan_info": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_int]),
    "ptycho_descend": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_int, c_void_p, c_int,
                               POINTER(c_int32), c_int, c_int, c_float, c_int, c_int, ctypes.c_double,
                               ctypes.c_double, c_int, c_void_p, c_void_p, c_void_p]),
    "detector_expose": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, POINTER(c_float), c_int, c_float,
                                c_float, c_float, ctypes.c_ulonglong, c_void_p, c_void_p]),
    "ptycho_stitch": (c_int, [c_void_p, c_void_p, c_void_p, c_int, POINTER(c_int32), c_int, c_int, c_void_p,
                              c_int, c_int, c_void_p]),
    "detector_resample": (c_int, [c_void_p, c_void_p, c_int, c_int, c_float, c_float, c_int, c_void_p, c_void_p]),
    "mnf_nrmse": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_longlong, c_void_p, c_void_p]),
    "unet_param_count": (ctypes.c_longlong, [POINTER(UnetShapeC)]),
    "unet_forward": (c_int, [c_void_p, POINTER(UnetShapeC), c_void_p, c_void_p, c_float, c_int, c_void_p,
                             c_void_p]),
    "unet_train_step": (c_int, [c_void_p, POINTER(UnetShapeC), c_void_p, c_void_p, c_void_p, c_int, c_float,
                                c_void_p, c_float, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "mnf_conv2d": (c_int, [c_void_p, c_int, c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_int, c_int,
                           c_void_p, c_void_p]),
    "mnf_conv2d_grad": (c_int, [c_void_p, c_int, c_void_p, c_int, c_int, c_int, c_void_p, c_int, c_void_p,
                                c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "mnf_autotune": (c_int, [c_void_p, c_int, c_int, c_int, POINTER(c_double), c_void_p]),
    "mnf_set_variant": (c_int, [c_void_p, c_int, c_int]),
    "mnf_get_variant": (c_int, [c_void_p, c_int]),
    "mnf_profile": (c_int, [c_void_p, ctypes.c_uint32]),
    "mnf_profile_sampled": (c_int, [c_void_p, ctypes.c_uint32, c_int]),
    "mnf_profile_read": (c_int, [c_void_p, c_int, POINTER(ctypes.c_longlong), POINTER(c_double)]),
    "mnf_profile_reset": (c_int, [c_void_p]),
    "mnf_kernel_class_name": (ctypes.c_char_p, [c_int]),
}

KERNEL_CLASSES = ["rows_fwd", "cols_modulus", "rows_inv", "probe_update", "object_update",
                  "small", "fuse", "forward", "grad_cols", "grad_scatter", "shift", "small_run"]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the library once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2608_01746_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
