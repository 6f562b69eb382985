"""ctypes binding of libcntr.so (the C ABI declared in include/cntr.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library. Raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcntr.so")

CHECK_ORDER, CHECK_FINITE, CHECK_SYMMETRY = 1, 2, 4

STATUS = {0: "CNTR_OK", -1: "CNTR_EINVAL", -2: "CNTR_ESHAPE", -3: "CNTR_EORDER",
          -4: "CNTR_ESINGULAR", -5: "CNTR_ENONFINITE", -6: "CNTR_EHIP", -7: "CNTR_ENOMEM",
          -8: "CNTR_ENOCONV", -9: "CNTR_ESYMMETRY"}

SYMBOLS = ["cntr_init_matsubara", "cntr_dyson_step", "cntr_convolution", "cntr_sigma_2b",
           "cntr_extrapolate", "cntr_green_from_H", "cntr_matsubara_fourier", "cntr_distance", "cntr_copy_slice", "cntr_solve_2b", "cntr_sync",
           "cntr_last_error", "cntr_finalize", "cntr_version", "cntr_profile_begin", "cntr_profile_begin_every",
           "cntr_profile_end", "cntr_observables", "cntr_sigma_local", "cntr_adjoint_sweep",
           "cntr_solve_2b_batch", "cntr_set_checks", "cntr_mark_slices",
           "cntr_dyson_step_noalloc", "cntr_peierls", "cntr_peierls_grad",
           "cntr_graph_begin", "cntr_graph_end", "cntr_graph_launch", "cntr_graph_destroy",
           "cntr_solve_2b_uneven", "cntr_set_tiles", "cntr_vie2_matsubara", "cntr_vie2_step",
           "cntr_polarization_k", "cntr_sigma_gw_k", "cntr_phonon_free", "cntr_scale_slice",
           "cntr_holstein_mf", "cntr_bubble2_local"]


class CntrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nt", C.c_int32), ("ntau", C.c_int32), ("d", C.c_int32), ("sig", C.c_int32),
                ("k", C.c_int32), ("beta", C.c_double), ("h", C.c_double), ("mu", C.c_double)]


class Profile(C.Structure):
    _fields_ = [("hist_ms", C.c_double), ("hist_launches", C.c_int64), ("hist_bytes", C.c_double),
                ("hist_flops", C.c_double), ("step_ms", C.c_double), ("steps", C.c_int64)]


class GF(C.Structure):
    _fields_ = [("mat", C.c_void_p), ("ret", C.c_void_p), ("les", C.c_void_p), ("tv", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        # torch ships its own HIP runtime under the same soname as the
        # system one; loading torch first makes the library bind to that
        # copy, so both share one runtime (two in one process see no device)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
        P = C.POINTER
        L.cntr_init_matsubara.argtypes = [i32, P(Grid), P(GF), P(GF), P(vp), dbl, i32, vp]
        L.cntr_dyson_step.argtypes = [i32, i32, P(Grid), P(GF), P(GF), P(vp), vp]
        L.cntr_dyson_step_noalloc.argtypes = [i32, i32, P(Grid), P(GF), P(GF), P(vp), vp]
        L.cntr_convolution.argtypes = [i32, i32, P(Grid), P(GF), P(GF), P(GF), P(GF), P(GF), P(vp), vp]
        L.cntr_sigma_2b.argtypes = [i32, i32, P(Grid), P(GF), P(vp), P(GF), P(vp), P(vp), dbl, vp]
        L.cntr_extrapolate.argtypes = [i32, i32, P(Grid), P(GF), vp]
        L.cntr_green_from_H.argtypes = [i32, P(Grid), P(GF), P(vp), vp]
        L.cntr_matsubara_fourier.argtypes = [i32, P(Grid), P(GF), P(GF), P(vp), i32, vp]
        L.cntr_distance.argtypes = [i32, i32, P(Grid), P(GF), P(GF), P(dbl), vp]
        L.cntr_copy_slice.argtypes = [i32, i32, P(Grid), P(GF), P(GF), vp]
        L.cntr_solve_2b.argtypes = [P(Grid), P(GF), P(GF), P(GF), vp, vp, vp, dbl, i32, dbl, dbl,
                                    i32, dbl, i32, i32, P(dbl), vp]
        L.cntr_observables.argtypes = [i32, i32, P(Grid), P(GF), P(GF), P(vp), P(vp), vp, vp, vp]
        L.cntr_sigma_local.argtypes = [i32, i32, P(Grid), P(GF), P(GF), dbl, vp]
        L.cntr_adjoint_sweep.argtypes = [i32, P(Grid), P(GF), P(GF), P(vp), P(vp), dbl, P(GF), P(GF), P(vp),
                                         P(vp), i32, dbl, P(dbl), vp]
        L.cntr_solve_2b_batch.argtypes = [i32, P(Grid), P(GF), P(GF), P(GF), P(vp), P(vp), P(vp), dbl, i32, dbl,
                                          dbl, i32, dbl, i32, P(dbl), vp]
        L.cntr_solve_2b_uneven.argtypes = [i32, P(Grid), P(GF), P(GF), P(GF), P(vp), P(vp), P(vp), dbl, i32, dbl,
                                           dbl, i32, dbl, i32, P(dbl), vp]
        L.cntr_set_tiles.argtypes = [i32, i32, P(C.c_int32), P(C.c_int32)]
        L.cntr_vie2_matsubara.argtypes = [i32, P(Grid), P(GF), P(GF), P(GF), dbl, i32, vp]
        L.cntr_vie2_step.argtypes = [i32, i32, P(Grid), P(GF), P(GF), P(GF), P(GF), vp]
        L.cntr_polarization_k.argtypes = [i32, i32, P(Grid), P(GF), P(GF), dbl, vp]
        L.cntr_sigma_gw_k.argtypes = [i32, i32, P(Grid), P(GF), P(GF), P(GF), dbl, vp]
        L.cntr_bubble2_local.argtypes = [i32, i32, P(Grid), P(GF), P(GF), P(GF), dbl, vp]
        L.cntr_phonon_free.argtypes = [i32, P(Grid), P(GF), P(dbl), vp]
        L.cntr_scale_slice.argtypes = [i32, i32, P(Grid), P(GF), P(GF), P(vp), dbl, vp]
        L.cntr_holstein_mf.argtypes = [i32, i32, P(Grid), P(GF), P(vp), P(dbl), dbl, P(vp), P(vp), vp]
        L.cntr_sync.argtypes = [vp]
        L.cntr_set_checks.argtypes = [i32]
        L.cntr_graph_begin.argtypes = [vp]
        L.cntr_graph_end.argtypes = [vp, P(vp)]
        L.cntr_graph_launch.argtypes = [vp, vp]
        L.cntr_graph_destroy.argtypes = [vp]
        L.cntr_peierls.argtypes = [i32, P(Grid), P(vp), P(vp), P(vp), P(vp), vp]
        L.cntr_peierls_grad.argtypes = [i32, P(Grid), P(vp), P(vp), P(vp), P(vp), P(vp), vp]
        L.cntr_mark_slices.argtypes = [i32, P(GF), i32]
        L.cntr_profile_begin.argtypes = []
        L.cntr_profile_begin_every.argtypes = [C.c_int32]
        L.cntr_profile_end.argtypes = [P(Profile)]
        L.cntr_last_error.restype = C.c_char_p
        L.cntr_version.restype = C.c_char_p
        for name in SYMBOLS:
            if name not in ("cntr_last_error", "cntr_version"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(code):
    if code != 0:
        raise CntrError(code, lib().cntr_last_error().decode())
    return code


def arr(ctype, items):
    a = (ctype * len(items))()
    for i, x in enumerate(items):
        a[i] = x
    return a
