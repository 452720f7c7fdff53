"""Autotuning of the H*v launch with a JSON cache.

The cache key is the spin list, the set of active Hamiltonian terms, the
precision and the column count; its value is the configuration the library's
autotuner measured fastest (variant, grid size, columns per lane).  The cache
file is $FTLM_TUNE_CACHE, else ~/.cache/ftlm_mi355x/hv_tuning.json.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os

import numpy as np

from . import FTLM_C128, _ffi
from ._ffi import check


def cache_path() -> str:
    p = os.environ.get("FTLM_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "ftlm_mi355x", "hv_tuning.json")


def tuning_key(ham, precision: int, n_cols: int) -> str:
    terms = "J%d-d%d-dip%d" % (ham._J is not None and bool(np.any(ham._J)),
                               ham._d is not None and bool(np.any(ham._d)), ham._pos is not None)
    spins = hashlib.sha1(np.asarray(ham._two_s).tobytes()).hexdigest()[:12]
    return "n%d-s%s-%s-p%d-k%d" % (ham.n_sites, spins, terms, precision, n_cols)


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except Exception:
        return {}


def _store(d):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def tune(ham, precision: int = FTLM_C128, n_cols: int = 1, use_cache: bool = True):
    """Returns the chosen configuration dict and applies it to the handle."""
    import torch
    key = tuning_key(ham, precision, n_cols)
    cache = _load() if use_cache else {}
    if key in cache:
        c = cache[key]
        check(_ffi.lib().ftlm_hamiltonian_set_tuning(ham.handle, precision, n_cols, c["variant"],
                                                     c["grid_cap"], c["kc"]), "set_tuning")
        return dict(c, cached=True)
    dt = torch.complex128 if precision == FTLM_C128 else torch.complex64
    shape = (ham.dim,) if n_cols == 1 else (ham.dim, n_cols)
    v = torch.ones(shape, dtype=dt, device="cuda")
    w = torch.empty_like(v)
    var, cap, kc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    ms = ctypes.c_float()
    check(_ffi.lib().ftlm_hamiltonian_autotune(ham.handle, precision, n_cols, ctypes.c_void_p(v.data_ptr()),
                                               ctypes.c_void_p(w.data_ptr()),
                                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                               ctypes.byref(var), ctypes.byref(cap), ctypes.byref(kc),
                                               ctypes.byref(ms)), "ftlm_hamiltonian_autotune")
    c = {"variant": var.value, "grid_cap": cap.value, "kc": kc.value, "ms": ms.value}
    if use_cache:
        cache = _load()
        cache[key] = c
        _store(cache)
    return dict(c, cached=False)
