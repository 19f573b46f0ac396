"""ctypes binding of ``libhyperpower.so`` (the C ABI in include/hyperpower.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  The library must have been built in-tree
(``python -m paper_2311_06926_amd.build``); loading fails loudly otherwise.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhyperpower.so")

HP_STATUS = {
    0: "HP_OK", -1: "HP_EINVAL", -2: "HP_EHIP", -3: "HP_ENOMEM", -4: "HP_ENOTSPD",
    -5: "HP_EBREAKDOWN", -6: "HP_ENOCONV", -7: "HP_ENAN",
}

PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
KRYLOV = {"minres": 0, "fgmres": 1}
SCHUR = {"Pcq1": 1, "Pcq2": 2, "Pcq_pcg": 3}
SCHEDULE = {"literal": 0, "prev": 1}
SPEC_VELOCITY, SPEC_SCHUR = 0, 1


class HPError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where} failed: {HP_STATUS.get(code, code)}")


class hp_opts(ctypes.Structure):
    _fields_ = [
        ("c_pen", ctypes.c_double),
        ("schur_variant", ctypes.c_int),
        ("l_schedule", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("krylov", ctypes.c_int),
        ("restart", ctypes.c_int),
        ("maxit", ctypes.c_int),
        ("order", ctypes.c_int),
        ("iters", ctypes.c_int),
        ("max_rhs", ctypes.c_int),
        ("poll_lag", ctypes.c_int),
        ("use_graph", ctypes.c_int),
        ("autotune", ctypes.c_int),
        ("op_kchunk", ctypes.c_int),
        ("op_order", ctypes.c_int),
        ("fd_plan", ctypes.c_int),
        ("op_slabs", ctypes.c_int),
        ("schur_level", ctypes.c_int),
        ("schur_pcg_iters", ctypes.c_int),
        ("schur_pcg_tol", ctypes.c_double),
        ("op_fused", ctypes.c_int),
        ("op_staged", ctypes.c_int),
        ("forward", ctypes.c_int),
        ("use_x0", ctypes.c_int),
        ("spectrum_gate", ctypes.c_int),
        ("p0_scale", ctypes.c_double),
        ("breakdown_tol", ctypes.c_double),
        ("op_dma", ctypes.c_int),
        ("op_pres_wide", ctypes.c_int),
    ]


class hp_tuning(ctypes.Structure):
    _fields_ = [
        ("op_kchunk", ctypes.c_int),
        ("op_order", ctypes.c_int),
        ("op_tuned", ctypes.c_int),
        ("op_slabs", ctypes.c_int),
        ("fd_plan", ctypes.c_int * 3),
        ("op_us", ctypes.c_double),
        ("fd_us", ctypes.c_double * 3),
        ("op_staged", ctypes.c_int),
        ("op_pres_wide", ctypes.c_int),
    ]


class hp_solve_info(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("relres", ctypes.c_double),
        ("true_relres", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("iters_per_rhs", ctypes.c_int * 64),
    ]


_lib = None

P = ctypes.c_void_p
I = ctypes.c_int
D = ctypes.c_double

SIGNATURES = {
    "hp_default_opts": (None, [ctypes.POINTER(hp_opts)]),
    "hp_setup": (I, [I, I, D, ctypes.POINTER(hp_opts), P, ctypes.POINTER(P)]),
    "hp_set_nu": (I, [P, D]),
    "hp_sizes": (I, [P, ctypes.POINTER(ctypes.c_int64 * 12), ctypes.POINTER(ctypes.c_int64 * 5)]),
    "hp_apply_K": (I, [P, P, P, I]),
    "hp_apply_K_quad": (I, [P, P, P, I]),
    "hp_apply_A": (I, [P, P, P, I]),
    "hp_apply_B": (I, [P, P, P, I]),
    "hp_apply_Bt": (I, [P, P, P, I]),
    "hp_apply_P0": (I, [P, P, P, I]),
    "hp_apply_hyperpower": (I, [P, I, I, P, P, I]),
    "hp_apply_PV": (I, [P, I, I, P, P, I]),
    "hp_solve": (I, [P, P, P, I, D, ctypes.POINTER(hp_solve_info)]),
    "hp_solve_noalloc": (I, [P, P, P, I, D, ctypes.POINTER(hp_solve_info)]),
    "hp_build_rhs": (I, [P, P, I, P, P, P, P, I]),
    "hp_apply_MV": (I, [P, P, P, I]),
    "hp_grad": (I, [P, P, P, P, P, P, I]),
    "hp_get_tuning": (I, [P, I, ctypes.POINTER(hp_tuning)]),
    "hp_spectrum": (I, [P, I, I, I, I, I, P, P, P, ctypes.POINTER(I), ctypes.POINTER(D),
                        ctypes.POINTER(D)]),
    "hp_destroy": (None, [P]),
    "hp_status_string": (ctypes.c_char_p, [I]),
}


def load():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2311_06926_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code, where):
    if code != 0:
        raise HPError(code, where)
    return code
