"""ctypes view of include/fire2.h and the loader of libfire2.so.

Only argument marshalling lives here.  There is no fallback: if the HIP
library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfire2.so")

FIRE_OK = 0
ERRORS = {-1: "FIRE_E_ARG", -2: "FIRE_E_BOX", -3: "FIRE_E_NONFINITE", -4: "FIRE_E_OVERLAP",
          -5: "FIRE_E_DEVICE", -6: "FIRE_E_OOM"}
STOP = {1: "converged", 2: "max_steps", 3: "maxvdotf", -3: "nonfinite", -4: "overlap"}  # < 0: a batched system's own failure
POT = {"lj": 1, "gupta": 2, "harmonic": 3, "sw": 4}
CONVENTION = {"rgl": 0, "half": 1}
PRECISION = {"fp64": 0, "mixed": 1, "fp32": 2}
INTEGRATOR = {"eulerimplicit": 0, "eulerexplicit": 1, "verlet": 2}
CRITERION = {"fmax": 0, "f2norm": 1}
VARIANT = {"fire2": 0, "fire1": 1}
TRACE_COLS = 9

# Every symbol include/fire2.h declares.
EXPORTS = [
    "fire_params_default", "fire_init", "fire_finalize", "fire_set_params", "fire_get_params",
    "fire_last_error", "fire_stop_name", "fire_energy_forces", "fire_minimize", "fire_minimize_traced",
    "fire_hvp", "fire_lowest_curvature", "fire_minimize_batched", "fire_energy_forces_dev", "fire_hvp_dev",
    "fire_minimize_dev", "fire_minimize_batched_dev", "fire_repeat_forces_dev", "fire_minimize_ex",
    "fire_minimize_ex_dev", "fire_minimize_batched_noalloc", "fire_tuning_info",
]


class fire_box(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("len", ctypes.c_double * 3), ("periodic", ctypes.c_int * 3)]


class fire_potential(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int), ("convention", ctypes.c_int),
        ("eps", ctypes.c_double), ("sigma", ctypes.c_double), ("rc", ctypes.c_double),
        ("A", ctypes.c_double), ("p", ctypes.c_double), ("q", ctypes.c_double), ("xi", ctypes.c_double),
        ("r0", ctypes.c_double), ("r_in", ctypes.c_double), ("r_out", ctypes.c_double),
        ("k", ctypes.c_double * 3),
        ("sw_B", ctypes.c_double), ("sw_a", ctypes.c_double), ("sw_lambda", ctypes.c_double),
        ("sw_gamma", ctypes.c_double),
    ]


class fire_params(ctypes.Structure):
    _fields_ = [
        ("dt_start", ctypes.c_double), ("tmax", ctypes.c_double), ("tmin", ctypes.c_double),
        ("dtgrow", ctypes.c_double), ("dtshrink", ctypes.c_double), ("alpha0", ctypes.c_double),
        ("alphashrink", ctypes.c_double), ("f2a", ctypes.c_double),
        ("delaystep", ctypes.c_int), ("vdfmax", ctypes.c_int), ("halfstepback", ctypes.c_int),
        ("initialdelay", ctypes.c_int), ("integrator", ctypes.c_int), ("criterion", ctypes.c_int),
        ("variant", ctypes.c_int), ("precision", ctypes.c_int),
        ("mixed_switch", ctypes.c_double), ("skin", ctypes.c_double), ("dmax", ctypes.c_double),
    ]


class fire_result(ctypes.Structure):
    _fields_ = [
        ("stop_reason", ctypes.c_int), ("precision_switched", ctypes.c_int),
        ("iterations", ctypes.c_longlong), ("force_evals", ctypes.c_longlong),
        ("iterations_low", ctypes.c_longlong), ("rebuilds", ctypes.c_longlong),
        ("energy", ctypes.c_double), ("energy_per_atom", ctypes.c_double), ("fmax", ctypes.c_double),
        ("f2norm", ctypes.c_double), ("dt", ctypes.c_double), ("alpha", ctypes.c_double),
    ]


class fire_atoms(ctypes.Structure):
    _fields_ = [("frozen", ctypes.c_void_p), ("mass", ctypes.c_void_p)]


class FireError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        self.code = code
        self.name = ERRORS.get(code, str(code))
        super().__init__(f"{self.name}: {msg}")


_lib = None


def load(path: str = LIB_PATH):
    """Load libfire2.so (raises if it is not built).  torch is imported first
    when available so that the library binds to the HIP runtime torch uses."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run python paper_1908_02038_amd/build.py")
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    ctx_p = ctypes.c_void_p
    dp = P(ctypes.c_double)
    ll = ctypes.c_longlong
    lib.fire_params_default.argtypes = [P(fire_params)]
    lib.fire_params_default.restype = None
    lib.fire_init.argtypes = [P(ctx_p), ctypes.c_int, P(fire_params)]
    lib.fire_finalize.argtypes = [ctx_p]
    lib.fire_finalize.restype = None
    lib.fire_set_params.argtypes = [ctx_p, P(fire_params)]
    lib.fire_get_params.argtypes = [ctx_p, P(fire_params)]
    lib.fire_last_error.argtypes = [ctx_p]
    lib.fire_last_error.restype = ctypes.c_char_p
    lib.fire_tuning_info.argtypes = [ctx_p]
    lib.fire_tuning_info.restype = ctypes.c_char_p
    lib.fire_stop_name.argtypes = [ctypes.c_int]
    lib.fire_stop_name.restype = ctypes.c_char_p
    lib.fire_energy_forces.argtypes = [ctx_p, ll, dp, P(fire_box), P(fire_potential), dp, dp]
    lib.fire_minimize.argtypes = [ctx_p, ll, dp, P(fire_box), P(fire_potential), ctypes.c_double, ll,
                                  P(fire_result)]
    lib.fire_minimize_traced.argtypes = [ctx_p, ll, dp, P(fire_box), P(fire_potential), ctypes.c_double, ll,
                                         P(fire_result), dp]
    lib.fire_hvp.argtypes = [ctx_p, ll, dp, dp, P(fire_box), P(fire_potential), dp]
    lib.fire_lowest_curvature.argtypes = [ctx_p, ll, dp, P(fire_box), P(fire_potential), dp, ctypes.c_int, dp, dp]
    lib.fire_minimize_batched.argtypes = [ctx_p, ctypes.c_int, P(ll), dp, P(fire_box), P(fire_potential),
                                          P(fire_params), ctypes.c_double, ll, P(fire_result)]
    lib.fire_energy_forces_dev.argtypes = [ctx_p, ll, ctypes.c_void_p, P(fire_box), P(fire_potential),
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.fire_hvp_dev.argtypes = [ctx_p, ll, ctypes.c_void_p, ctypes.c_void_p, P(fire_box), P(fire_potential),
                                 ctypes.c_void_p, ctypes.c_void_p]
    lib.fire_minimize_dev.argtypes = [ctx_p, ll, ctypes.c_void_p, P(fire_box), P(fire_potential),
                                      ctypes.c_double, ll, P(fire_result), ctypes.c_void_p]
    lib.fire_minimize_batched_dev.argtypes = [ctx_p, ctypes.c_int, P(ll), ctypes.c_void_p, P(fire_box),
                                              P(fire_potential), P(fire_params), ctypes.c_double, ll,
                                              P(fire_result), ctypes.c_void_p]
    lib.fire_minimize_batched_noalloc.argtypes = [ctx_p, ctypes.c_int, P(ll), ctypes.c_void_p, P(fire_box),
                                                  P(fire_potential), P(fire_params), ctypes.c_double, ll,
                                                  P(fire_result), ctypes.c_void_p]
    lib.fire_repeat_forces_dev.argtypes = [ctx_p, ctypes.c_int, ctypes.c_void_p]
    lib.fire_minimize_ex.argtypes = [ctx_p, ll, dp, P(fire_box), P(fire_potential), P(fire_atoms),
                                     ctypes.c_double, ll, P(fire_result), dp]
    lib.fire_minimize_ex_dev.argtypes = [ctx_p, ll, ctypes.c_void_p, P(fire_box), P(fire_potential),
                                         P(fire_atoms), ctypes.c_double, ll, P(fire_result), ctypes.c_void_p]
    _lib = lib
    return lib
