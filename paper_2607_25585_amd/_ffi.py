"""ctypes declarations of the C ABI in ``include/ftlm.h`` (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libftlm.so")

FTLM_C128 = 0
FTLM_C64 = 1

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int32_p = ctypes.POINTER(ctypes.c_int32)


class FtlmSystem(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("two_s", c_int32_p), ("J", c_double_p),
                ("d", c_double_p), ("e", c_double_p), ("g", c_double_p), ("B", c_double_p),
                ("pos", c_double_p)]


class FtlmRunParams(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int32), ("n_lanczos", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("instance", ctypes.c_uint32), ("T", c_double_p), ("n_T", ctypes.c_int32),
                ("fields", c_double_p), ("n_fields", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("columns", ctypes.c_int32),
                ("r_init", ctypes.c_void_p)]


class FtlmResult(ctypes.Structure):
    _fields_ = [("lnZ", c_double_p), ("E", c_double_p), ("C", c_double_p), ("M", c_double_p),
                ("n_lanczos_used", c_int32_p), ("E_min", c_double_p), ("alpha", c_double_p),
                ("beta", c_double_p), ("hv_ms", c_double_p), ("hv_launches", c_int32_p)]


class FtlmMlpWeights(ctypes.Structure):
    _fields_ = [("W", ctypes.c_void_p * 4), ("b", ctypes.c_void_p * 4)]


_lib = None


def lib():
    """Loads the in-tree gfx950 library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libftlm.so is not built; run __graft_entry__.build() or "
                              "python paper_2607_25585_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        I = ctypes.c_int
        L.ftlm_last_error.restype = ctypes.c_char_p
        L.ftlm_version.restype = I
        L.ftlm_hamiltonian_create.argtypes = [ctypes.POINTER(FtlmSystem), ctypes.POINTER(vp)]
        L.ftlm_hamiltonian_destroy.argtypes = [vp]
        L.ftlm_hamiltonian_destroy.restype = None
        L.ftlm_hamiltonian_dim.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
        L.ftlm_hamiltonian_nnz_per_row.argtypes = [vp, c_double_p]
        L.ftlm_hamiltonian_set_field.argtypes = [vp, c_double_p]
        L.ftlm_apply.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
        L.ftlm_gaussian_vectors.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint64, vp,
                                            vp]
        L.ftlm_gaussian_vectors_noalloc.argtypes = L.ftlm_gaussian_vectors.argtypes
        L.ftlm_run_sftlm_workspace_size.argtypes = [vp, ctypes.POINTER(FtlmRunParams),
                                                     ctypes.POINTER(ctypes.c_size_t)]
        L.ftlm_run_workspace_size.argtypes = [vp, ctypes.POINTER(FtlmRunParams),
                                              ctypes.POINTER(ctypes.c_size_t)]
        L.ftlm_run.argtypes = [vp, ctypes.POINTER(FtlmRunParams), vp, ctypes.c_size_t, vp,
                               ctypes.POINTER(FtlmResult)]
        L.ftlm_run_kpm_workspace_size.argtypes = [vp, ctypes.POINTER(FtlmRunParams), ctypes.c_int32,
                                                   ctypes.POINTER(ctypes.c_size_t)]
        L.ftlm_run_kpm.argtypes = [vp, ctypes.POINTER(FtlmRunParams), ctypes.c_int32, vp, ctypes.c_size_t,
                                   vp, ctypes.POINTER(FtlmResult), c_double_p]
        L.ftlm_run_sftlm.argtypes = [vp, ctypes.POINTER(FtlmRunParams), vp, ctypes.c_size_t, vp,
                               ctypes.POINTER(FtlmResult)]
        L.ftlm_run_batched_workspace_size.argtypes = [ctypes.POINTER(vp), ctypes.c_int32,
                                                      ctypes.POINTER(FtlmRunParams),
                                                      ctypes.POINTER(ctypes.c_size_t)]
        L.ftlm_run_batched.argtypes = [ctypes.POINTER(vp), ctypes.c_int32,
                                       ctypes.POINTER(FtlmRunParams), vp, ctypes.c_size_t, vp,
                                       ctypes.POINTER(FtlmResult)]
        L.ftlm_batched_set_tuning.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.ftlm_set_plan_windows.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.ftlm_tridiag_eigen.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp, vp,
                                         vp, vp, vp]
        L.ftlm_boltzmann.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp,
                                     vp, vp, vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp]
        L.ftlm_mlp_workspace_size.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.ftlm_mlp_forward.argtypes = [ctypes.POINTER(FtlmMlpWeights), ctypes.c_int32, vp, vp, vp,
                                       ctypes.c_size_t, vp]
        L.ftlm_mlp_backward.argtypes = [ctypes.POINTER(FtlmMlpWeights), ctypes.c_int32, vp, vp,
                                        vp * 4, vp * 4, vp, ctypes.c_size_t, vp]
        L.ftlm_adam_step.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_int32, vp]
        L.ftlm_describe_passes.argtypes = [ctypes.POINTER(FtlmSystem), ctypes.c_int32,
                                           ctypes.c_int32, c_int32_p,
                                           ctypes.POINTER(ctypes.c_uint32), c_int32_p, c_int32_p,
                                           c_int32_p, c_int32_p, c_double_p]
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.ftlm_describe_windows.argtypes = [ctypes.POINTER(FtlmSystem), ctypes.c_int32,
                                            ctypes.c_int64, ctypes.c_int32, c_int32_p, u32p, u32p,
                                            c_int32_p, u32p, c_int32_p]
        L.ftlm_hamiltonian_autotune.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp,
                                                c_int32_p, c_int32_p, c_int32_p,
                                                ctypes.POINTER(ctypes.c_float)]
        L.ftlm_hamiltonian_set_tuning.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.c_int32, ctypes.c_int32]
        _lib = L
    return _lib


class FtlmError(RuntimeError):
    pass


def check(rc: int, what: str = "") -> None:
    if rc != 0:
        msg = lib().ftlm_last_error().decode(errors="replace")
        raise FtlmError("%s failed (status %d): %s" % (what or "ftlm call", rc, msg))
