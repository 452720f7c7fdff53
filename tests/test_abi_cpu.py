"""CPU checks of the C ABI library: it loads, exports every declared entry point,
and the host-side argument checks reject bad input without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ftlm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ftlm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libftlm():
    from paper_2607_25585_amd import _ffi
    if not os.path.exists(_ffi.LIB_PATH):
        from paper_2607_25585_amd import build
        build.build()
    return _ffi.lib()


def test_header_declares_entry_points():
    names = _declared()
    for must in ("ftlm_hamiltonian_create", "ftlm_apply", "ftlm_run", "ftlm_run_batched",
                 "ftlm_tridiag_eigen", "ftlm_boltzmann", "ftlm_mlp_forward",
                 "ftlm_mlp_backward", "ftlm_adam_step", "ftlm_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(libftlm):
    missing = [n for n in _declared() if not hasattr(libftlm, n)]
    assert not missing, missing


def test_version(libftlm):
    assert libftlm.ftlm_version() >= 10000


def test_library_is_gfx950_code_object():
    from paper_2607_25585_amd import _ffi
    data = open(_ffi.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_create_rejects_bad_arguments_on_host(libftlm):
    """Validation happens before any device call, so it is testable on the CPU."""
    from paper_2607_25585_amd import _ffi
    h = ctypes.c_void_p()
    assert libftlm.ftlm_hamiltonian_create(None, ctypes.byref(h)) == -1
    two_s = (ctypes.c_int32 * 2)(1, 16)
    g = (ctypes.c_double * 2)(2.0, 2.0)
    B = (ctypes.c_double * 3)(0, 0, 1)
    s = _ffi.FtlmSystem(2, two_s, None, None, None, g, B, None)
    assert libftlm.ftlm_hamiltonian_create(ctypes.byref(s), ctypes.byref(h)) == -4  # 2s > 15
    two_s = (ctypes.c_int32 * 2)(1, 1)
    pos = (ctypes.c_double * 6)(0, 0, 0, 0, 0, 0)
    s = _ffi.FtlmSystem(2, two_s, None, None, None, g, B, pos)
    assert libftlm.ftlm_hamiltonian_create(ctypes.byref(s), ctypes.byref(h)) == -1  # coincident
    assert b"coincident" in libftlm.ftlm_last_error()
    big = (ctypes.c_int32 * 17)(*([3] * 17))  # 4^17 > 2^32
    g17 = (ctypes.c_double * 17)(*([2.0] * 17))
    s = _ffi.FtlmSystem(17, big, None, None, None, g17, B, None)
    assert libftlm.ftlm_hamiltonian_create(ctypes.byref(s), ctypes.byref(h)) == -4


def test_apply_and_run_reject_null(libftlm):
    assert libftlm.ftlm_apply(None, 0, 1, None, None, None) == -1
    assert libftlm.ftlm_run(None, None, None, 0, None, None) == -1
    assert libftlm.ftlm_gaussian_vectors(1, 0, 0, 0, 0, 10, None, None) == -1


@pytest.mark.parametrize("wl", ["cfg1", "cfg2", "cfg2_hb", "cfg4", "cfg4_hb"])
@pytest.mark.parametrize("prec", [0, 1])
def test_pass_plan_covers_every_pair_once(libftlm, wl, prec):
    """Host logic of the windowed H*v: every interacting pair is applied by
    exactly one pass, every window fits the LDS budget, and pass counts stay
    bounded."""
    import numpy as np
    import ftlm_workloads as W
    import paper_2607_25585_amd as F
    sysm, _ = W.WORKLOADS[wl]()
    d = F.describe_passes(sysm, prec)
    n = sysm.n_sites
    pairs = set()
    for i in range(n):
        for j in range(i + 1, n):
            if (sysm.J is not None and sysm.J[i, j] != 0) or sysm.pos is not None:
                pairs.add((i, j))
    got = [tuple(sorted(p)) for p in d["pair_sites"].tolist()]
    assert len(got) == len(set(got)) == len(pairs)
    assert set(got) == pairs
    es = 16 if prec == 0 else 8
    assert np.all(d["window_rows"].astype(np.int64) * es <= 64 * 1024)
    assert len(d["window_rows"]) <= 16


def test_plan_windows_setting(libftlm):
    """ftlm_set_plan_windows: smaller LDS windows give more passes (each within
    the new budget), zeros restore the default plan, and out-of-range values are
    refused without changing the setting."""
    import numpy as np
    import ftlm_workloads as W
    import paper_2607_25585_amd as F
    sysm, _ = W.cfg4_hb()
    base = F.describe_passes(sysm, 0)
    try:
        F.set_plan_windows(pass_kb=8)
        small = F.describe_passes(sysm, 0)
        assert len(small["window_rows"]) > len(base["window_rows"])
        assert np.all(small["window_rows"].astype(np.int64) * 16 <= 8 * 1024)
        for bad in ((2, 0, 0), (256, 0, 0), (0, 3, 0), (0, 0, 1 << 17), (-1, 0, 0)):
            assert libftlm.ftlm_set_plan_windows(*bad) == -1  # FTLM_EINVAL
        again = F.describe_passes(sysm, 0)
        assert np.array_equal(again["window_rows"], small["window_rows"])
    finally:
        F.set_plan_windows(0, 0, 0)
    restored = F.describe_passes(sysm, 0)
    assert np.array_equal(restored["window_rows"], base["window_rows"])


def test_batched_tuning_arguments(libftlm):
    """ftlm_batched_set_tuning accepts the documented launch choices and refuses
    the rest (host-only call)."""
    ok = [(0, 0, 0, 0), (64, 11, 1, 256), (65536, 12, 0, 1024), (1024, 11, 0, 512)]
    bad = [(63, 0, 0, 0), (70000, 0, 0, 0), (0, 10, 0, 0), (0, 13, 0, 0), (0, 0, 2, 0), (0, 0, -1, 0),
           (0, 0, 0, 128), (0, 0, 0, 768), (0, 0, 0, 2048)]
    try:
        for a in ok:
            assert libftlm.ftlm_batched_set_tuning(*a) == 0, a
        for a in bad:
            assert libftlm.ftlm_batched_set_tuning(*a) == -1, a  # FTLM_EINVAL
    finally:
        libftlm.ftlm_batched_set_tuning(0, 0, 0, 0)


def _interacting_pairs(sysm):
    n = sysm.n_sites
    return {(i, j) for i in range(n) for j in range(i + 1, n)
            if (sysm.J is not None and sysm.J[i, j] != 0) or sysm.pos is not None}


def _check_window_plan(sysm, prec, wbytes, max_pass=16):
    import numpy as np
    import paper_2607_25585_amd as F
    d = F.describe_windows(sysm, prec, wbytes)
    n = sysm.n_sites
    got = [tuple(sorted(p)) for p in d["pair_sites"].tolist()]
    assert len(got) == len(set(got)) and set(got) == _interacting_pairs(sysm)
    # every pair lies inside the window of the pass that applies it
    k = 0
    for ps, npp in enumerate(d["n_pairs"].tolist()):
        for (i, j) in got[k:k + npp]:
            assert (d["window_sites"][ps] >> i) & 1 and (d["window_sites"][ps] >> j) & 1
        k += npp
    # single flips: disjoint over passes, inside the window, same sites as the LDS plan
    ss = d["single_sites"].astype(np.int64)
    assert all((int(a) & int(b)) == 0 for x, a in enumerate(ss) for b in ss[x + 1:])
    assert all((int(s) & ~int(w)) == 0 for s, w in zip(ss, d["window_sites"]))
    n_single = sum(bin(int(s)).count("1") for s in ss)
    assert n_single == int(F.describe_passes(sysm, prec)["n_singles"].sum())
    es = 16 if prec == 0 else 8
    dim = int(np.prod(np.asarray(sysm.two_s) + 1))
    wr = d["window_rows"].astype(np.int64)
    assert np.all((wr * es <= wbytes) | (wr == dim))
    assert np.all(dim % wr == 0)
    assert len(d["window_rows"]) <= max_pass and n <= 32


@pytest.mark.parametrize("wl", ["cfg1", "cfg2", "cfg2_hb", "cfg4", "cfg4_hb"])
@pytest.mark.parametrize("prec", [0, 1])
def test_window_plan_covers_every_pair_once(libftlm, wl, prec):
    """Host logic of the L2-window H*v: pairs applied once, inside their
    window; single flips placed once; windows within the byte budget."""
    import ftlm_workloads as W
    sysm, _ = W.WORKLOADS[wl]()
    _check_window_plan(sysm, prec, 1 << 20)


@pytest.mark.parametrize("seed,n,max_two_s,half", [(0, 6, 3, False), (1, 5, 4, False),
                                                   (2, 12, 1, True), (3, 16, 1, True),
                                                   (4, 4, 5, False), (5, 9, 2, False),
                                                   (6, 14, 1, True), (7, 7, 3, False)])
def test_window_plan_small_windows(libftlm, seed, n, max_two_s, half):
    import numpy as np
    import ftlm_workloads as W
    rng = np.random.default_rng(1900 + seed)
    sysm = W.random_small_system(rng, n, max_two_s=max_two_s)
    if half:
        sysm.two_s[:] = 1
    for prec in (0, 1):
        _check_window_plan(sysm, prec, 16 * 1024, max_pass=64)
