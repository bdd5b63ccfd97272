"""ctypes binding of libehdg.so: the C ABI declared in include/ehdg.h, nothing more.

Fails loudly when the library is missing: there is no fallback implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libehdg.so")

EHDG_OK = 0
EHDG_ERR_INVALID_ARG = 1
EHDG_ERR_UNSUPPORTED = 2
EHDG_ERR_HIP = 3
EHDG_ERR_NOT_CONVERGED = 4
EHDG_ERR_DIVERGED = 5
EHDG_ERR_WORKSPACE_TOO_SMALL = 6

EHDG_TRANSPORT = 0
EHDG_SWE = 1
EHDG_EULER = 2

EHDG_FP64 = 0
EHDG_FP32_REFINE = 1
EHDG_BF16_REFINE = 2
EHDG_FP32 = 3

EXPORTED = [
    "ehdg_reference_points", "ehdg_workspace_bytes", "ehdg_setup", "ehdg_set_forcing", "ehdg_set_initial",
    "ehdg_iterate", "ehdg_solve", "ehdg_step", "ehdg_get_solution", "ehdg_get_residuals", "ehdg_sizes",
    "ehdg_state_bytes", "ehdg_get_state", "ehdg_set_state", "ehdg_destroy", "ehdg_error_string",
    "ehdg_last_error", "ehdg_batch_workspace_bytes", "ehdg_batch_create", "ehdg_batch_solve", "ehdg_batch_step",
    "ehdg_batch_advance", "ehdg_batch_destroy", "ehdg_batch_last_error", "ehdg_variable_workspace_bytes",
    "ehdg_setup_variable", "ehdg_batch_create_static", "ehdg_batch_set_graph", "ehdg_tune_set",
    "ehdg_tune_clear", "ehdg_launch_shape", "ehdg_batch_report_bytes", "ehdg_batch_launch", "ehdg_batch_poll",
    "ehdg_batch_get_solution", "ehdg_batch_set_persistent",
]


class ehdg_desc(ctypes.Structure):
    _fields_ = [
        ("pde", ctypes.c_int32),
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("L", ctypes.c_double * 3),
        ("periodic", ctypes.c_int32 * 3),
        ("degree", ctypes.c_int32),
        ("beta", ctypes.c_double * 3),
        ("sigma", ctypes.c_double),
        ("Phi", ctypes.c_double),
        ("U0", ctypes.c_double * 2),
        ("c0", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("inner_sweeps", ctypes.c_int32),
    ]


_lib = None


def load():
    """Loads libehdg.so once (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1601_06681_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "ehdg_reference_points": (ctypes.c_int, [I32, P, P, P]),
        "ehdg_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(ehdg_desc), ctypes.POINTER(SZ)]),
        "ehdg_setup": (ctypes.c_int, [ctypes.POINTER(ehdg_desc), P, SZ, P, ctypes.POINTER(P)]),
        "ehdg_set_forcing": (ctypes.c_int, [P, P, P]),
        "ehdg_set_initial": (ctypes.c_int, [P, P]),
        "ehdg_iterate": (ctypes.c_int, [P, I32]),
        "ehdg_solve": (ctypes.c_int, [P, D, I32, ctypes.POINTER(I32), ctypes.POINTER(D)]),
        "ehdg_step": (ctypes.c_int, [P, I32, D, I32, P]),
        "ehdg_get_solution": (ctypes.c_int, [P, P]),
        "ehdg_get_residuals": (ctypes.c_int, [P, I32, I32, P]),
        "ehdg_sizes": (ctypes.c_int, [P, ctypes.POINTER(I64), ctypes.POINTER(I32), ctypes.POINTER(I32),
                                      ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "ehdg_state_bytes": (ctypes.c_int, [P, ctypes.POINTER(SZ)]),
        "ehdg_get_state": (ctypes.c_int, [P, P, SZ]),
        "ehdg_set_state": (ctypes.c_int, [P, P, SZ]),
        "ehdg_destroy": (ctypes.c_int, [P]),
        "ehdg_error_string": (ctypes.c_char_p, [ctypes.c_int]),
        "ehdg_last_error": (ctypes.c_char_p, [P]),
        "ehdg_batch_workspace_bytes": (ctypes.c_int, [P, I32, ctypes.POINTER(SZ)]),
        "ehdg_batch_create": (ctypes.c_int, [P, I32, P, SZ, P, ctypes.POINTER(P)]),
        "ehdg_batch_create_static": (ctypes.c_int, [P, I32, P, ctypes.POINTER(P)]),
        "ehdg_batch_set_graph": (ctypes.c_int, [P, I32]),
        "ehdg_batch_set_persistent": (ctypes.c_int, [P, I32]),
        "ehdg_tune_set": (ctypes.c_int, [I32, I32, I32, I32, I32, I32]),
        "ehdg_tune_clear": (ctypes.c_int, []),
        "ehdg_launch_shape": (ctypes.c_int, [P, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "ehdg_batch_solve": (ctypes.c_int, [P, D, I32, P, P]),
        "ehdg_batch_step": (ctypes.c_int, [P, I32, D, I32, P]),
        "ehdg_batch_advance": (ctypes.c_int, [P, I32, D, P, P]),
        "ehdg_batch_report_bytes": (ctypes.c_int, [P, ctypes.POINTER(SZ)]),
        "ehdg_batch_launch": (ctypes.c_int, [P, I32, D, P, P, SZ]),
        "ehdg_batch_poll": (ctypes.c_int, [P, P, ctypes.POINTER(I32)]),
        "ehdg_batch_get_solution": (ctypes.c_int, [P, I32, P]),
        "ehdg_batch_destroy": (ctypes.c_int, [P]),
        "ehdg_batch_last_error": (ctypes.c_char_p, [P]),
        "ehdg_variable_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(ehdg_desc), ctypes.POINTER(SZ)]),
        "ehdg_setup_variable": (ctypes.c_int, [ctypes.POINTER(ehdg_desc), P, P, P, P, SZ, P, ctypes.POINTER(P)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
