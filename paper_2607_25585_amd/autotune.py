"""Autotuning of the H*v launch and of the batched run, with a JSON cache.

Plain H*v: the cache key is the spin list, the set of active Hamiltonian
terms, the precision and the column count; its value is the configuration the
library's autotuner measured fastest (variant, grid size, columns per lane).

Batched run: the key is the sorted spin lists of the instances, their term
sets, the precision and R; the value is the fastest (columns per item, grid
cap, rows per work unit, unit order, threads per block) by the duration of the
Lanczos step launches of short batched runs on the caller's instances and
fields.

The cache file is $FTLM_TUNE_CACHE, else ~/.cache/ftlm_mi355x/hv_tuning.json.
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


def batched_key(hams, precision: int, R: int) -> str:
    parts = sorted(tuning_key(h, precision, 0).rsplit("-p", 1)[0] for h in hams)
    digest = hashlib.sha1("|".join(parts).encode()).hexdigest()[:16]
    return "batched-%s-p%d-R%d" % (digest, precision, R)


def tune_batched(hams, R: int, T, fields_per_inst, seed: int = 0, precision: int = FTLM_C128,
                 n_steps: int = 6, use_cache: bool = False):
    """Chooses the batched launch for these instances and fields: columns per
    item K (dividing R), then the threads per block, then the grid cap, then the
    rows per work unit and the unit order, each by the mean duration of a
    Lanczos step (HIP events around the step launches of a run of n_steps steps
    over every curve), coordinate by coordinate.  Applies the choice
    (batched_set_tuning) and returns it; pass its "columns" to run_batched."""
    from . import batched_set_tuning, run_batched
    key = batched_key(hams, precision, R)
    cache = _load() if use_cache else {}
    if key in cache:
        c = cache[key]
        batched_set_tuning(c["grid_cap"], c["unit_bits"], c["order"], c.get("block", 0))
        return dict(c, cached=True)

    def step_ms(K, grid, ubits, order, block):
        batched_set_tuning(grid, ubits, order, block)
        res = run_batched(hams, R, n_steps, T, fields_per_inst, seed=seed, precision=precision,
                          columns=K, time_steps=True)
        return float(res[0]["step_ms"][0]) / n_steps  # summed over the waves of each step

    # best = (ms, K, block, grid, ubits, order)
    best = None
    for K in [k for k in (16, 8, 4, 2, 1) if R % k == 0]:
        ms = step_ms(K, 1024, 11, 0, 512)
        if best is None or ms < best[0]:
            best = (ms, K, 512, 1024, 11, 0)
    for block in (256, 1024):
        ms = step_ms(best[1], 1024, 11, 0, block)
        if ms < best[0]:
            best = (ms, best[1], block, 1024, 11, 0)
    for grid in (256, 512, 2048, 4096):
        ms = step_ms(best[1], grid, 11, 0, best[2])
        if ms < best[0]:
            best = (ms, best[1], best[2], grid, 11, 0)
    for ubits, order in ((12, 0), (11, 1), (12, 1)):
        ms = step_ms(best[1], best[3], ubits, order, best[2])
        if ms < best[0]:
            best = (ms, best[1], best[2], best[3], ubits, order)
    c = {"columns": best[1], "block": best[2], "grid_cap": best[3], "unit_bits": best[4], "order": best[5],
         "step_ms": round(best[0], 4)}
    batched_set_tuning(c["grid_cap"], c["unit_bits"], c["order"], c["block"])
    if use_cache:
        cache = _load()
        cache[key] = c
        _store(cache)
    return dict(c, cached=False)
