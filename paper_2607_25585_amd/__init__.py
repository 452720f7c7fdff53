"""MI355X (gfx950) finite-temperature Lanczos method for anisotropic spin systems.

Thin Python binding over the C ABI of ``include/ftlm.h``: it marshals arguments,
takes device memory and streams from PyTorch, and calls the library; every step
of the computation (H*v, random vectors, Lanczos recursion, Krylov eigenpairs,
Boltzmann sums, surrogate kernels) runs in the library's HIP kernels.

The physics is Sec. 2 of the paper: the Hamiltonian of Eq. (mce-hamop) on the
full product basis, FTLM per Eqs. (E-1-1), (E-1-2), (E-2-C), (E-2-D).
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _ffi
from ._ffi import FTLM_C128, FTLM_C64, FtlmError, check

__all__ = ["Hamiltonian", "gaussian_vectors", "run", "run_batched", "batched_set_tuning", "tridiag_eigen",
           "boltzmann", "FTLM_C128", "FTLM_C64", "FtlmError", "library_path"]


def library_path() -> str:
    return _ffi.LIB_PATH


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64(a, shape=None):
    if a is None:
        return None
    out = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return out.reshape(shape) if shape is not None else out


def _system_struct(system):
    n = len(system.two_s)
    keep = dict(two_s=np.ascontiguousarray(np.asarray(system.two_s, np.int32)),
                J=_f64(system.J, (n, n)) if system.J is not None else None,
                d=_f64(system.d) if system.d is not None else None,
                e=_f64(system.e, (n, 3)) if system.e is not None else None,
                g=_f64(system.g), B=_f64(system.B, (3,)),
                pos=_f64(system.pos, (n, 3)) if system.pos is not None else None)
    s = _ffi.FtlmSystem(n, keep["two_s"].ctypes.data_as(_ffi.c_int32_p), _dptr(keep["J"]),
                        _dptr(keep["d"]), _dptr(keep["e"]), _dptr(keep["g"]), _dptr(keep["B"]),
                        _dptr(keep["pos"]))
    return s, keep


def describe_passes(system, precision: int = FTLM_C128):
    """Host-only: the windowed-pass plan of the one-column H*v (no GPU needed)."""
    s, keep = _system_struct(system)
    npass = ctypes.c_int32()
    check(_ffi.lib().ftlm_describe_passes(ctypes.byref(s), int(precision), 0, ctypes.byref(npass),
                                          None, None, None, None, None, None),
          "ftlm_describe_passes")
    m = npass.value
    wr = np.zeros(m, np.uint32)
    na, npp, ns = (np.zeros(m, np.int32) for _ in range(3))
    n_pairs_total = 4096
    ps = np.zeros(2 * n_pairs_total, np.int32)
    nnz = ctypes.c_double()
    i32 = lambda a: a.ctypes.data_as(_ffi.c_int32_p)  # noqa: E731
    check(_ffi.lib().ftlm_describe_passes(ctypes.byref(s), int(precision), m, ctypes.byref(npass),
                                          wr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                          i32(na), i32(npp), i32(ns), i32(ps), ctypes.byref(nnz)),
          "ftlm_describe_passes")
    tot = int(npp.sum())
    return dict(window_rows=wr, n_active=na, n_pairs=npp, n_singles=ns,
                pair_sites=ps[:2 * tot].reshape(-1, 2), nnz_per_row=nnz.value)


def set_plan_windows(pass_kb: int = 0, l2_kb: int = 0, tile_kb: int = 0) -> None:
    """Window sizes (KiB) of the H*v planners for handles created afterwards
    (``ftlm_set_plan_windows``; zeros restore the defaults)."""
    check(_ffi.lib().ftlm_set_plan_windows(int(pass_kb), int(l2_kb), int(tile_kb)), "ftlm_set_plan_windows")


def describe_windows(system, precision: int = FTLM_C128, window_bytes: int = 0):
    """Host-only: the L2-window plan of the one-column H*v (variant 4)."""
    s, keep = _system_struct(system)
    npass = ctypes.c_int32()
    check(_ffi.lib().ftlm_describe_windows(ctypes.byref(s), int(precision), int(window_bytes), 0,
                                           ctypes.byref(npass), None, None, None, None, None),
          "ftlm_describe_windows")
    m = npass.value
    u32 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))  # noqa: E731
    i32 = lambda a: a.ctypes.data_as(_ffi.c_int32_p)  # noqa: E731
    wr, ws, ss = (np.zeros(m, np.uint32) for _ in range(3))
    npp = np.zeros(m, np.int32)
    ps = np.zeros(2 * 4096, np.int32)
    check(_ffi.lib().ftlm_describe_windows(ctypes.byref(s), int(precision), int(window_bytes), m,
                                           ctypes.byref(npass), u32(wr), u32(ws), i32(npp), u32(ss),
                                           i32(ps)), "ftlm_describe_windows")
    tot = int(npp.sum())
    return dict(window_rows=wr, window_sites=ws, n_pairs=npp, single_sites=ss,
                pair_sites=ps[:2 * tot].reshape(-1, 2))


class Hamiltonian:
    """Compiled Hamiltonian of Eq. (mce-hamop) on the current HIP device.

    ``system`` is any object with fields two_s, J, d, e, g, B, pos (see
    ``ftlm_workloads.System``)."""

    def __init__(self, system):
        n = len(system.two_s)
        self._two_s = np.ascontiguousarray(np.asarray(system.two_s, np.int32))
        self._J = _f64(system.J, (n, n)) if system.J is not None else None
        self._d = _f64(system.d) if system.d is not None else None
        self._e = _f64(system.e, (n, 3)) if system.e is not None else None
        self._g = _f64(system.g)
        self._B = _f64(system.B, (3,))
        self._pos = _f64(system.pos, (n, 3)) if system.pos is not None else None
        s = _ffi.FtlmSystem(n, self._two_s.ctypes.data_as(_ffi.c_int32_p), _dptr(self._J),
                            _dptr(self._d), _dptr(self._e), _dptr(self._g), _dptr(self._B),
                            _dptr(self._pos))
        h = ctypes.c_void_p()
        check(_ffi.lib().ftlm_hamiltonian_create(ctypes.byref(s), ctypes.byref(h)),
              "ftlm_hamiltonian_create")
        self._h = h
        d = ctypes.c_uint64()
        check(_ffi.lib().ftlm_hamiltonian_dim(h, ctypes.byref(d)), "ftlm_hamiltonian_dim")
        self.dim = int(d.value)
        self.n_sites = n

    @property
    def handle(self):
        return self._h

    @property
    def nnz_per_row(self) -> float:
        x = ctypes.c_double()
        check(_ffi.lib().ftlm_hamiltonian_nnz_per_row(self._h, ctypes.byref(x)), "nnz_per_row")
        return float(x.value)

    def set_field(self, B) -> None:
        b = _f64(B, (3,))
        check(_ffi.lib().ftlm_hamiltonian_set_field(self._h, _dptr(b)), "set_field")
        self._B = b

    def set_tuning(self, precision: int, n_cols: int, variant: int, grid_cap: int = 0, kc: int = 0) -> None:
        """Fixes the H*v launch for (precision, n_cols): variant 0 restores the
        built-in choice (see ``ftlm_hamiltonian_set_tuning``)."""
        check(_ffi.lib().ftlm_hamiltonian_set_tuning(self._h, int(precision), int(n_cols), int(variant),
                                                     int(grid_cap), int(kc)), "ftlm_hamiltonian_set_tuning")

    def apply(self, v, out=None):
        """w = H v for a device tensor v of shape [dim] or [dim, K]
        (complex128 or complex64, contiguous)."""
        torch = _torch()
        if v.dtype == torch.complex128:
            prec = FTLM_C128
        elif v.dtype == torch.complex64:
            prec = FTLM_C64
        else:
            raise TypeError("v must be complex128 or complex64")
        if not v.is_cuda or not v.is_contiguous() or v.shape[0] != self.dim or v.dim() > 2:
            raise ValueError("v must be a contiguous device tensor of shape [dim] or [dim, K]")
        K = 1 if v.dim() == 1 else int(v.shape[1])
        w = torch.empty_like(v) if out is None else out
        check(_ffi.lib().ftlm_apply(self._h, prec, K, ctypes.c_void_p(v.data_ptr()),
                                    ctypes.c_void_p(w.data_ptr()), _stream()), "ftlm_apply")
        return w

    def close(self):
        if getattr(self, "_h", None):
            _ffi.lib().ftlm_hamiltonian_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gaussian_vectors(seed, instance, field, r0, n_cols, dim, device="cuda"):
    """Complex Gaussian start vectors [dim, n_cols] (complex128) from the
    library's counter-based generator (Eqs. E-1-1, E-1-2)."""
    torch = _torch()
    out = torch.empty((int(dim), int(n_cols)), dtype=torch.complex128, device=device)
    check(_ffi.lib().ftlm_gaussian_vectors(ctypes.c_uint64(int(seed)), int(instance), int(field),
                                           int(r0), int(n_cols), ctypes.c_uint64(int(dim)),
                                           ctypes.c_void_p(out.data_ptr()), _stream()),
          "ftlm_gaussian_vectors")
    return out


def _params(R, n_lanczos, T, seed, fields, precision, columns, r_init, instance):
    T = _f64(T)
    fl = _f64(fields).reshape(-1, 3) if fields is not None else None
    p = _ffi.FtlmRunParams()
    p.R = int(R)
    p.n_lanczos = int(n_lanczos)
    p.seed = int(seed)
    p.instance = int(instance)
    p.T = _dptr(T)
    p.n_T = len(T)
    p.fields = _dptr(fl) if fl is not None else None
    p.n_fields = len(fl) if fl is not None else 1
    p.precision = int(precision)
    p.columns = int(columns)
    p.r_init = ctypes.c_void_p(r_init.data_ptr()) if r_init is not None else None
    return p, (T, fl, r_init)


def run(ham: Hamiltonian, R: int, n_lanczos: int, T, seed: int = 0, fields=None,
        precision: int = FTLM_C128, columns: int = 0, r_init=None, instance: int = 0,
        return_tridiagonals: bool = False, workspace=None, time_hv: bool = False):
    """FTLM thermodynamics (Sec. 2.2) on the GPU.  Returns a dict of NumPy arrays
    lnZ, E, C, M ([n_fields, n_T]), n_lanczos_used ([n_fields, R]), E_min."""
    torch = _torch()
    p, keep = _params(R, n_lanczos, T, seed, fields, precision, columns, r_init, instance)
    nbytes = ctypes.c_size_t()
    check(_ffi.lib().ftlm_run_workspace_size(ham.handle, ctypes.byref(p), ctypes.byref(nbytes)),
          "ftlm_run_workspace_size")
    ws = workspace
    if ws is None or ws.numel() < nbytes.value:
        ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
    nf, nT = p.n_fields, p.n_T
    out = {k: np.zeros((nf, nT)) for k in ("lnZ", "E", "C", "M")}
    out["n_lanczos_used"] = np.zeros((nf, R), np.int32)
    out["E_min"] = np.zeros(nf)
    res = _ffi.FtlmResult(_dptr(out["lnZ"]), _dptr(out["E"]), _dptr(out["C"]), _dptr(out["M"]),
                          out["n_lanczos_used"].ctypes.data_as(_ffi.c_int32_p),
                          _dptr(out["E_min"]), None, None, None, None)
    if time_hv:
        out["hv_ms"] = np.zeros(1)
        out["hv_launches"] = np.zeros(1, np.int32)
        res.hv_ms = _dptr(out["hv_ms"])
        res.hv_launches = out["hv_launches"].ctypes.data_as(_ffi.c_int32_p)
    if return_tridiagonals:
        out["alpha"] = np.zeros((nf, R, n_lanczos))
        out["beta"] = np.zeros((nf, R, n_lanczos))
        res.alpha = _dptr(out["alpha"])
        res.beta = _dptr(out["beta"])
    check(_ffi.lib().ftlm_run(ham.handle, ctypes.byref(p), ctypes.c_void_p(ws.data_ptr()),
                              ctypes.c_size_t(ws.numel()), _stream(), ctypes.byref(res)),
          "ftlm_run")
    del keep
    return out


def run_sftlm(ham: Hamiltonian, R: int, n_lanczos: int, T, seed: int = 0, fields=None,
              precision: int = FTLM_C128, instance: int = 0, workspace=None):
    """Symmetric FTLM (Eqs. E-2-G, E-2-H) with R/2 time-reversed pairs of random
    vectors.  Returns lnZ, E, C, M ([n_fields, n_T]), n_lanczos_used, E_min."""
    torch = _torch()
    p, keep = _params(R, n_lanczos, T, seed, fields, precision, 1, None, instance)
    nbytes = ctypes.c_size_t()
    check(_ffi.lib().ftlm_run_sftlm_workspace_size(ham.handle, ctypes.byref(p), ctypes.byref(nbytes)),
          "ftlm_run_sftlm_workspace_size")
    ws = workspace
    if ws is None or ws.numel() < nbytes.value:
        ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
    nf, nT = p.n_fields, p.n_T
    out = {k: np.zeros((nf, nT)) for k in ("lnZ", "E", "C", "M")}
    out["n_lanczos_used"] = np.zeros((nf, R), np.int32)
    out["E_min"] = np.zeros(nf)
    res = _ffi.FtlmResult(_dptr(out["lnZ"]), _dptr(out["E"]), _dptr(out["C"]), _dptr(out["M"]),
                          out["n_lanczos_used"].ctypes.data_as(_ffi.c_int32_p),
                          _dptr(out["E_min"]), None, None, None, None)
    check(_ffi.lib().ftlm_run_sftlm(ham.handle, ctypes.byref(p), ctypes.c_void_p(ws.data_ptr()),
                                    ctypes.c_size_t(ws.numel()), _stream(), ctypes.byref(res)),
          "ftlm_run_sftlm")
    return out


def run_kpm(ham: Hamiltonian, R: int, n_moments: int, T, seed: int = 0, fields=None,
            precision: int = FTLM_C128, instance: int = 0, n_bound_steps: int = 40, workspace=None):
    """Chebyshev expansion of the thermal traces (no smoothing kernel) with the
    FTLM random vectors.  Returns lnZ, E, C, M ([n_fields, n_T]), E_lo, E_hi."""
    torch = _torch()
    p, keep = _params(R, n_bound_steps, T, seed, fields, precision, 1, None, instance)
    nbytes = ctypes.c_size_t()
    check(_ffi.lib().ftlm_run_kpm_workspace_size(ham.handle, ctypes.byref(p), int(n_moments),
                                                 ctypes.byref(nbytes)), "ftlm_run_kpm_workspace_size")
    ws = workspace
    if ws is None or ws.numel() < nbytes.value:
        ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
    nf, nT = p.n_fields, p.n_T
    out = {k: np.zeros((nf, nT)) for k in ("lnZ", "E", "C", "M")}
    out["E_min"] = np.zeros(nf)
    bounds = np.zeros((nf, 2))
    res = _ffi.FtlmResult(_dptr(out["lnZ"]), _dptr(out["E"]), _dptr(out["C"]), _dptr(out["M"]),
                          None, _dptr(out["E_min"]), None, None, None, None)
    check(_ffi.lib().ftlm_run_kpm(ham.handle, ctypes.byref(p), int(n_moments), ctypes.c_void_p(ws.data_ptr()),
                                  ctypes.c_size_t(ws.numel()), _stream(), ctypes.byref(res), _dptr(bounds)),
          "ftlm_run_kpm")
    out["E_lo"], out["E_hi"] = bounds[:, 0].copy(), bounds[:, 1].copy()
    return out


def batched_set_tuning(grid_cap: int = 0, unit_bits: int = 0, order: int = 0, block: int = 0) -> None:
    """Launch choices of later run_batched calls on this thread
    (``ftlm_batched_set_tuning``; zeros restore the defaults)."""
    check(_ffi.lib().ftlm_batched_set_tuning(int(grid_cap), int(unit_bits), int(order), int(block)),
          "ftlm_batched_set_tuning")


def run_batched(hams, R: int, n_lanczos: int, T, fields_per_inst, seed: int = 0,
                precision: int = FTLM_C64, workspace=None, columns: int = 0,
                workspace_bytes: Optional[int] = None, time_steps: bool = False, instance0: int = 0):
    """Batched FTLM over many instances and field directions (one persistent
    launch per Lanczos step).  fields_per_inst[k] is an [n_dirs, 3] array;
    instance k draws the random vectors of instance index instance0 + k (so a
    workload can be run in groups of instances with the same vectors as one
    run, or as :func:`run` with instance=instance0 + k).  Returns a list of
    result dicts like :func:`run`; with time_steps the first dict also holds
    "step_ms" (summed duration of the Lanczos step launches) and "steps"."""
    torch = _torch()
    n = len(hams)
    ps = (_ffi.FtlmRunParams * n)()
    keep = []
    for k in range(n):
        p, kp = _params(R, n_lanczos, T, seed, fields_per_inst[k], precision, columns, None, instance0 + k)
        ps[k] = p
        keep.append(kp)
    hs = (ctypes.c_void_p * n)(*[h.handle for h in hams])
    nbytes = ctypes.c_size_t()
    check(_ffi.lib().ftlm_run_batched_workspace_size(hs, n, ps, ctypes.byref(nbytes)),
          "ftlm_run_batched_workspace_size")
    need = int(nbytes.value) if workspace_bytes is None else int(workspace_bytes)
    ws = workspace
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    outs = []
    resarr = (_ffi.FtlmResult * n)()
    for k in range(n):
        nf, nT = ps[k].n_fields, ps[k].n_T
        o = {kk: np.zeros((nf, nT)) for kk in ("lnZ", "E", "C", "M")}
        o["n_lanczos_used"] = np.zeros((nf, R), np.int32)
        o["E_min"] = np.zeros(nf)
        hv = None
        nl = None
        if time_steps and k == 0:
            o["step_ms"] = np.zeros(1)
            o["steps"] = np.zeros(1, np.int32)
            hv = _dptr(o["step_ms"])
            nl = o["steps"].ctypes.data_as(_ffi.c_int32_p)
        resarr[k] = _ffi.FtlmResult(_dptr(o["lnZ"]), _dptr(o["E"]), _dptr(o["C"]), _dptr(o["M"]),
                                    o["n_lanczos_used"].ctypes.data_as(_ffi.c_int32_p),
                                    _dptr(o["E_min"]), None, None, hv, nl)
        outs.append(o)
    check(_ffi.lib().ftlm_run_batched(hs, n, ps, ctypes.c_void_p(ws.data_ptr()),
                                      ctypes.c_size_t(need), _stream(), resarr),
          "ftlm_run_batched")
    del keep
    return outs


def tridiag_eigen(alpha, beta, y=None, n_used=None):
    """Krylov eigenpairs of [n_lanczos, n_cols] FP64 device tridiagonals."""
    torch = _torch()
    nl, nc = alpha.shape
    eps = torch.empty_like(alpha)
    q1 = torch.empty_like(alpha)
    qy = torch.empty_like(alpha)
    scratch = torch.empty(4 * nl * nc, dtype=torch.float64, device=alpha.device)
    vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
    check(_ffi.lib().ftlm_tridiag_eigen(nc, nl, vp(n_used), vp(alpha), vp(beta), vp(y), vp(eps),
                                        vp(q1), vp(qy), vp(scratch), _stream()),
          "ftlm_tridiag_eigen")
    return eps, q1, qy


def boltzmann(R, eps, q1, qy, n_used, dims, T):
    """Boltzmann sums (Eqs. E-2-C, E-2-D) of device Krylov data
    [n_lanczos, n_curves*R]; returns lnZ, E, C, M [n_curves, n_T] and E_min."""
    torch = _torch()
    nl, ncol = eps.shape
    nc = ncol // R
    T = torch.as_tensor(np.asarray(T, np.float64), device=eps.device)
    dims = torch.as_tensor(np.asarray(dims, np.float64).reshape(-1), device=eps.device)
    outs = [torch.empty((nc, len(T)), dtype=torch.float64, device=eps.device) for _ in range(4)]
    emin = torch.empty(nc, dtype=torch.float64, device=eps.device)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    check(_ffi.lib().ftlm_boltzmann(nc, R, nl, vp(n_used), vp(eps), vp(q1), vp(qy), vp(dims),
                                    vp(T), len(T), *[vp(o) for o in outs], vp(emin), _stream()),
          "ftlm_boltzmann")
    return outs + [emin]
