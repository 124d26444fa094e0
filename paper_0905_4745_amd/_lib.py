"""ctypes view of the C ABI in include/minnorm.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libminnorm.so")

MN_C128, MN_C64, MN_F64, MN_F32 = 0, 1, 2, 3


class MnHFactor(C.Structure):
    _fields_ = [("theta", C.c_void_p), ("perm", C.c_void_p), ("zeta", C.c_void_p),
                ("theta_t", C.c_void_p), ("perm_t", C.c_void_p), ("zeta_t", C.c_void_p)]


class MnOpts(C.Structure):
    _fields_ = [("alpha", C.c_double), ("stop_rule", C.c_int32), ("max_iter", C.c_int32),
                ("max_refine", C.c_int32), ("check_every", C.c_int32), ("inner_digits", C.c_int32),
                ("block", C.c_int32), ("streams", C.c_int32), ("precond", C.c_int32),
                ("tune", C.c_int32), ("batch_form", C.c_int32), ("refine", C.c_int32),
                ("max_reseed", C.c_int32), ("seed", C.c_uint64), ("graph", C.c_int32), ("reserved", C.c_int32),
                ("hfactor", C.POINTER(MnHFactor))]


class MnInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("refine_steps", C.c_int32),
                ("nrhs_done", C.c_int32), ("cert_rel", C.c_double), ("rho0", C.c_double),
                ("rho", C.c_double), ("xi", C.c_double), ("stage_ms", C.c_float * 8),
                ("retries", C.c_int32), ("factor", C.c_int32), ("kappa_hat", C.c_double)]

    def as_dict(self):
        return {"status": self.status, "iters": self.iters, "refine_steps": self.refine_steps,
                "nrhs_done": self.nrhs_done, "cert_rel": self.cert_rel, "rho0": self.rho0,
                "rho": self.rho, "xi": self.xi, "retries": self.retries,
                "factor": {1: "gram", 2: "householder"}.get(self.factor, None), "kappa_hat": self.kappa_hat,
                "stage_ms": {k: float(self.stage_ms[i]) for i, k in
                             enumerate(["sketch", "qr", "cg", "final", "refine", "-", "--", "total"])}}


EXPORTS = ["mn_create", "mn_destroy", "mn_set_stream", "mn_status_string", "mn_last_hip_error",
           "mn_workspace_bytes", "mn_profile", "mn_profile_read", "mn_plans_save", "mn_plans_load",
           "mn_plans_count", "srft_draw", "srft_sketch", "srft_sketch_h", "srft_sketch_noalloc", "build_preconditioner",
           "minnorm_solve", "minnorm_solve_batched", "minnorm_steps23"]

_lib = None


def load():
    """The loaded library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_0905_4745_amd.build` "
            "(hipcc, gfx950). There is no CPU fallback.")
    lib = C.CDLL(LIB_PATH)
    P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int, C.c_double
    lib.mn_create.argtypes = [C.POINTER(C.c_void_p), P]
    lib.mn_create.restype = I32
    lib.mn_destroy.argtypes = [P]
    lib.mn_destroy.restype = I32
    lib.mn_set_stream.argtypes = [P, P]
    lib.mn_set_stream.restype = I32
    lib.mn_status_string.argtypes = [I32]
    lib.mn_status_string.restype = C.c_char_p
    lib.mn_last_hip_error.argtypes = []
    lib.mn_last_hip_error.restype = C.c_char_p
    lib.mn_workspace_bytes.argtypes = [P]
    lib.mn_workspace_bytes.restype = I64
    lib.mn_profile.argtypes = [P, I32]
    lib.mn_profile.restype = I32
    lib.mn_profile_read.argtypes = [P, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    lib.mn_profile_read.restype = I32
    lib.mn_plans_save.argtypes = [P, C.c_char_p]
    lib.mn_plans_save.restype = I32
    lib.mn_plans_load.argtypes = [P, C.c_char_p]
    lib.mn_plans_load.restype = I32
    lib.mn_plans_count.argtypes = [P]
    lib.mn_plans_count.restype = I32
    lib.srft_draw.argtypes = [P, I32, C.c_uint64, C.c_int32, C.c_int32, I64, I64, P, P]
    lib.srft_draw.restype = I32
    lib.srft_sketch.argtypes = [P, I32, I64, I64, P, I64, I64, I64, P, P, P, I64]
    lib.srft_sketch.restype = I32
    lib.minnorm_steps23.argtypes = [P, I32, I64, I64, P, I64, P, I64, I64, P, P, P, P, C.POINTER(C.c_double)]
    lib.minnorm_steps23.restype = I32
    lib.srft_sketch_h.argtypes = [P, I32, I64, I64, P, I64, I64, I64, P, P, C.POINTER(MnHFactor), P, I64]
    lib.srft_sketch_h.restype = I32
    lib.srft_sketch_noalloc.argtypes = [P, I32, I64, I64, P, I64, I64, I64, P, P, P, I64]
    lib.srft_sketch_noalloc.restype = I32
    lib.build_preconditioner.argtypes = [P, I32, I64, I64, P, I64, P, I64]
    lib.build_preconditioner.restype = I32
    lib.minnorm_solve.argtypes = [P, I32, I64, I64, P, I64, P, I64, P, I64, I64, D, I64, I64, P, P,
                                  C.POINTER(MnOpts), P, I64, C.POINTER(MnInfo)]
    lib.minnorm_solve.restype = I32
    PP = C.POINTER(C.c_void_p)
    I64P = C.POINTER(C.c_int64)
    lib.minnorm_solve_batched.argtypes = [P, I32, C.c_int32, I64P, I64P, PP, I64P, PP, PP,
                                          C.POINTER(C.c_double), I64P, I64P, PP, PP,
                                          C.POINTER(MnOpts), PP, C.POINTER(MnInfo)]
    lib.minnorm_solve_batched.restype = I32
    _lib = lib
    return lib
