"""ctypes binding of libfw25.so (declarations in include/fw25.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Importing this module loads the library and fails loudly when it is missing;
there is no fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FW25_LIBRARY", os.path.join(_HERE, "libfw25.so"))

FW_OK, FW_EINVAL, FW_ESTATE, FW_EUNSTABLE, FW_EHIP, FW_ENOMEM, FW_ENONFINITE, FW_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
(FW_OPT_GRAPH_STEPS, FW_OPT_MARCH_CHUNK, FW_OPT_TILE_ROWS, FW_OPT_ROWS_PER_THREAD, FW_OPT_PERSISTENT,
 FW_OPT_TILE_ORDER, FW_OPT_PLANE_KERNELS, FW_OPT_PLANE_ROWS, FW_OPT_VEL_PLANES, FW_OPT_PRS_PLANES,
 FW_OPT_STEP_CHUNK, FW_OPT_RESIDENT_1D) = 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12

FW_FIELD_P, FW_FIELD_VX, FW_FIELD_VY, FW_FIELD_VZ = 0, 1, 2, 3

_NAMES = {0: "FW_OK", -1: "FW_EINVAL", -2: "FW_ESTATE", -3: "FW_EUNSTABLE", -4: "FW_EHIP",
          -5: "FW_ENOMEM", -6: "FW_ENONFINITE", -7: "FW_EUNSUPPORTED"}

# exported symbol -> (restype, argtypes)
_P = ctypes.c_void_p
_I = ctypes.c_int
_L = ctypes.c_int64
_D = ctypes.c_double
SIGNATURES = {
    "fw_last_error": (ctypes.c_char_p, []),
    "fw_abi_version": (_I, []),
    "fw_create_grid": (_I, [ctypes.POINTER(_P), _I, _I, _P, _D, _D, _I, _I, _P]),
    "fw_destroy": (_I, [_P]),
    "fw_workspace_bytes": (_L, [_P]),
    "fw_bind_workspace": (_I, [_P, _P, _L]),
    "fw_set_media": (_I, [_P, _P, _P, _I, _P, _P, _P, _D, ctypes.c_uint64]),
    "fw_set_relaxation_table": (_I, [_P, _I, _P, _P, _P]),
    "fw_set_sources": (_I, [_P, _L, _P, _P, _P, _I, _P, _I]),
    "fw_set_receivers": (_I, [_P, _L, _P, _P, _I]),
    "fw_set_receivers_into": (_I, [_P, _L, _P, _P, _I, _P, _L]),
    "fw_prepare": (_I, [_P]),
    "fw_step": (_I, [_P, _I, _P]),
    "fw_read_receivers": (_I, [_P, _P, _L, _I, _P]),
    "fw_reset_state": (_I, [_P, _P]),
    "fw_get_step": (_I, [_P, ctypes.POINTER(_L)]),
    "fw_state_bytes": (_L, [_P]),
    "fw_save_state": (_I, [_P, _P, _P]),
    "fw_load_state": (_I, [_P, _P, _P]),
    "fw_set_option": (_I, [_P, _I, _L]),
    "fw_time_kernels": (_I, [_P, _I, _P, _P]),
    "fw_adjoint_workspace_bytes": (_L, [_P, _I, _I]),
    "fw_energy_step": (_I, [_P, _P, _P]),
    "fw_energy_step_noalloc": (_I, [_P, _P, _P]),
    "fw_first_nonfinite_step": (_I, [_P, _P, _P]),
    "fw_device_copy": (_I, [_P, _P, _L, _P]),
    "fw_read_field": (_I, [_P, _I, _I, _P, _I, _P]),
    "fw_forward_checkpointed": (_I, [_P, _I, _I, _P, _L, _P]),
    "fw_adjoint": (_I, [_P, _I, _I, _P, _L, _P, _P, _P, _P]),
    "fw_adjoint_modulus": (_I, [_P, _I, _I, _P, _L, _P, _P, _P, _P]),
    "fw_set_class_alpha0": (_I, [_P, _I, _P]),
    "fw_set_strength_map": (_I, [_P, _P, _P]),
    "fw_set_time_space_stencil": (_I, [_P, _D]),
    "fw_set_widened_stencil": (_I, [_P, _D]),
    "fw_get_stencil": (_I, [_P, _P]),
    "fw_stream_probe": (_I, [_P, _I, _I, _I, _P, _P]),
}


class FWError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "?"), code, msg))
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfw25.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    # torch ships its own HIP runtime.  Loaded first, it is the one the
    # library's libamdhip64 dependency binds to, so the library and torch
    # share one runtime (torch's device memory and streams are valid in the
    # library's calls).  Loading the library first would bring in the
    # system's runtime beside torch's, and the library's calls would then
    # fail to find the device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(rc):
    if rc != FW_OK:
        raise FWError(rc, lib.fw_last_error().decode(errors="replace"))
    return rc
