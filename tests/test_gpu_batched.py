"""GPU parity of the batched persistent FTLM (many instances of uneven dimension,
several field directions each) against the plain GPU run and the CPU oracle,
with the same seeded random vectors."""
import numpy as np
import pytest

import ftlm_workloads as W
from oracle import ftlm as of

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def F():
    import paper_2607_25585_amd as F
    return F


def curve_err(x, ref):
    ref = np.asarray(ref)
    floor = 1e-3 * np.max(np.abs(ref))
    return float(np.max(np.abs(np.asarray(x) - ref) / np.maximum(np.abs(ref), max(floor, 1e-300))))


def _instances():
    rng = np.random.default_rng(321)
    systems = []
    for n, half in ((6, True), (9, True), (4, False), (7, True)):
        s = W.random_small_system(rng, n, max_two_s=1 if half else 3)
        if half:
            s.two_s[:] = 1
        systems.append(s)
    fields = [W.unit_vectors(rng, 2) * 0.8 for _ in systems]
    return systems, fields


@pytest.mark.parametrize("prec,tol,K", [(0, 1e-8, 4), (1, 1e-3, 2)])
def test_batched_matches_oracle(prec, tol, K):
    systems, fields = _instances()
    T = W.t_grid(30)
    R, NL, seed = 4, 40, 17
    hams = [F().Hamiltonian(s) for s in systems]
    got = F().run_batched(hams, R, NL, T, fields, seed=seed, precision=prec, columns=K)
    for k, s in enumerate(systems):
        ref = of.ftlm(s, R, NL, T, seed=seed, fields=fields[k], instance=k)
        for f in range(len(fields[k])):
            for key in ("lnZ", "E", "C", "M"):
                assert curve_err(got[k][key][f], ref[f][key]) < tol, (k, f, key)
            if prec == 0:
                assert np.array_equal(got[k]["n_lanczos_used"][f], ref[f]["n_lanczos_used"])


def test_batched_waves_give_identical_results():
    """A workspace that holds one item at a time splits the run into many waves;
    every reduction is fixed-order, so the curves are bitwise identical."""
    systems, fields = _instances()
    T = W.t_grid(20)
    hams = [F().Hamiltonian(s) for s in systems]
    a = F().run_batched(hams, 4, 30, T, fields, seed=3, precision=0, columns=2)
    import ctypes
    from paper_2607_25585_amd import _ffi
    ps = (_ffi.FtlmRunParams * len(hams))()
    keep = []
    for k in range(len(hams)):
        p, kp = F()._params(4, 30, T, 3, fields[k], 0, 2, None, k)
        ps[k] = p
        keep.append(kp)
    hs = (ctypes.c_void_p * len(hams))(*[h.handle for h in hams])
    nb = ctypes.c_size_t()
    _ffi.check(_ffi.lib().ftlm_run_batched_workspace_size(hs, len(hams), ps, ctypes.byref(nb)))
    # room for about two items of vectors per wave
    items = []
    for k, h in enumerate(hams):
        for _f in range(len(fields[k])):
            for _g in range(4 // 2):
                # four column-interleaved vectors of 2 columns (c128) plus the
                # item's cached diagonal of H (one FP64 value per row)
                items.append(4 * (((h.dim * 2 * 16) + 255) // 256 * 256) + (h.dim * 8 + 255) // 256 * 256)
    small = int(nb.value) - sum(items) + 2 * max(items)
    b = F().run_batched(hams, 4, 30, T, fields, seed=3, precision=0, columns=2, workspace_bytes=small)
    for k in range(len(hams)):
        for key in ("lnZ", "E", "C", "M"):
            assert np.array_equal(a[k][key], b[k][key]), (k, key)


def test_batched_matches_plain_run():
    systems, fields = _instances()
    T = W.t_grid(25)
    hams = [F().Hamiltonian(s) for s in systems]
    bat = F().run_batched(hams, 4, 35, T, fields, seed=9, precision=0, columns=4)
    for k, h in enumerate(hams):
        pl = F().run(h, 4, 35, T, seed=9, fields=fields[k], instance=k)
        for key in ("lnZ", "E", "C", "M"):
            assert np.max(np.abs(bat[k][key] - pl[key])) <= 1e-9 * np.max(np.abs(pl[key])) + 1e-12, (k, key)


def test_batched_large_instances_default_columns():
    """Instances of 2^18 rows (many 2048-row work units per item, so blocks walk
    several units of one item with its tables staged once) next to a small
    one, with the automatic column count (four per item here): FP64 batched
    against the plain GPU run (itself tied to the oracle), FP32 batched within
    the FP32 budget."""
    rng = np.random.default_rng(4242)
    systems = []
    for n in (18, 18, 10):
        s = W.random_small_system(rng, n, max_two_s=1)
        s.two_s[:] = 1
        systems.append(s)
    fields = [W.unit_vectors(rng, 1) * 0.9 for _ in systems]
    T = W.t_grid(20)
    hams = [F().Hamiltonian(s) for s in systems]
    print("case batched large instances dims", [h.dim for h in hams], flush=True)
    b64 = F().run_batched(hams, 4, 25, T, fields, seed=5, precision=0)
    b32 = F().run_batched(hams, 4, 25, T, fields, seed=5, precision=1)
    for k, h in enumerate(hams):
        pl = F().run(h, 4, 25, T, seed=5, fields=fields[k], instance=k)
        for key in ("lnZ", "E", "C", "M"):
            assert np.max(np.abs(b64[k][key] - pl[key])) <= 1e-9 * np.max(np.abs(pl[key])) + 1e-12, (k, key)
        assert curve_err(b32[k]["C"][0], pl["C"][0]) < 1e-3, k
        assert curve_err(b32[k]["M"][0], pl["M"][0]) < 1e-3, k


def test_batched_power_of_two_radices_match_oracle():
    """Instances whose radices are all powers of two (s = 3/2: digits are bit
    fields) next to one with radix 3, FP64 batched against the oracle."""
    rng = np.random.default_rng(777)
    systems = []
    for n, two_s in ((5, 3), (4, 3), (5, 2)):
        s = W.random_small_system(rng, n, max_two_s=3)
        s.two_s[:] = two_s
        systems.append(s)
    fields = [W.unit_vectors(rng, 2) * 0.7 for _ in systems]
    T = W.t_grid(25)
    hams = [F().Hamiltonian(s) for s in systems]
    got = F().run_batched(hams, 4, 30, T, fields, seed=23, precision=0, columns=2)
    for k, s in enumerate(systems):
        ref = of.ftlm(s, 4, 30, T, seed=23, fields=fields[k], instance=k)
        for f in range(len(fields[k])):
            for key in ("lnZ", "E", "C", "M"):
                assert curve_err(got[k][key][f], ref[f][key]) < 1e-8, (k, f, key)


@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-3)])
def test_batched_largest_cfg3_instances_match_oracle(prec, tol):
    """The two largest sizes of the batched workload (spin-1/2 dipolar rings of
    21 and 22 sites, 2^21 and 2^22 rows: many 2048-row units per item, the
    per-unit z-field table of the row bits from 8 up and the cached diagonal of
    H at full width) in one batched run, one field direction each, against the
    oracle with the same seeded vectors."""
    systems, spec, fields = W.cfg3()
    pick = [22, 15]  # N = 21 and N = 22
    sysl = [systems[k] for k in pick]
    assert [s.n_sites for s in sysl] == [21, 22]
    fl = [fields[k][:1] for k in pick]
    T = W.t_grid(24)
    R, NL = 2, 8
    hams = [F().Hamiltonian(s) for s in sysl]
    print("case batched cfg3 N=21,22 prec", prec, flush=True)
    got = F().run_batched(hams, R, NL, T, fl, seed=spec.seed, precision=prec, columns=2)
    for k, s in enumerate(sysl):
        ref = of.ftlm(s, R, NL, T, seed=spec.seed, fields=fl[k], instance=k)
        for key in ("lnZ", "E", "C", "M"):
            assert curve_err(got[k][key][0], ref[0][key]) < tol, (k, key)


@pytest.mark.parametrize("grid,ubits,order,block", [(512, 12, 1, 256), (64, 11, 1, 1024), (4096, 12, 0, 512),
                                                     (256, 11, 0, 1024)])
def test_batched_tuned_launches_match_oracle(grid, ubits, order, block):
    """Every launch choice of the batched autotuner keeps oracle parity: 4096-row
    work units (the spin-1/2 z-field unit table over row bits 8..11), units laid
    out largest instance first, small and large grids, blocks of 256, 512 and
    1024 threads (2048-row units: 8, 4 and 2 rows per thread); a 13-site spin-1/2
    dipolar instance (two 4096-row units) next to smaller ones of general
    radix."""
    rng = np.random.default_rng(515)
    systems = []
    for n, two_s in ((13, 1), (9, 1), (4, 2), (3, 3)):
        s = W.random_small_system(rng, n, max_two_s=3)
        s.two_s[:] = two_s
        systems.append(s)
    fields = [W.unit_vectors(rng, 2) * 0.8 for _ in systems]
    T = W.t_grid(24)
    hams = [F().Hamiltonian(s) for s in systems]
    print("case batched tuning grid", grid, "unit bits", ubits, "order", order, "block", block, flush=True)
    F().batched_set_tuning(grid, ubits, order, block)
    try:
        got = F().run_batched(hams, 4, 30, T, fields, seed=29, precision=0, columns=2, time_steps=True)
    finally:
        F().batched_set_tuning(0, 0, 0)
    assert got[0]["steps"][0] >= 30 and got[0]["step_ms"][0] > 0
    for k, s in enumerate(systems):
        ref = of.ftlm(s, 4, 30, T, seed=29, fields=fields[k], instance=k)
        for f in range(len(fields[k])):
            for key in ("lnZ", "E", "C", "M"):
                assert curve_err(got[k][key][f], ref[f][key]) < 1e-8, (k, f, key)


def test_batched_autotuner_choice_keeps_parity():
    """The batched autotuner on a small uneven set: its choice (columns, grid,
    unit rows, unit order) is applied and the tuned run matches the oracle."""
    from paper_2607_25585_amd import autotune
    rng = np.random.default_rng(616)
    systems = []
    for n in (12, 10, 8):
        s = W.random_small_system(rng, n, max_two_s=1)
        s.two_s[:] = 1
        systems.append(s)
    fields = [W.unit_vectors(rng, 1) * 1.0 for _ in systems]
    T = W.t_grid(24)
    hams = [F().Hamiltonian(s) for s in systems]
    try:
        c = autotune.tune_batched(hams, 4, T, fields, seed=31, precision=0, n_steps=4)
        print("tuned batched launch", c, flush=True)
        assert c["columns"] in (1, 2, 4) and c["unit_bits"] in (11, 12) and c["order"] in (0, 1)
        assert c["block"] in (256, 512, 1024)
        got = F().run_batched(hams, 4, 25, T, fields, seed=31, precision=0, columns=c["columns"])
    finally:
        F().batched_set_tuning(0, 0, 0)
    for k, s in enumerate(systems):
        ref = of.ftlm(s, 4, 25, T, seed=31, fields=fields[k], instance=k)
        for key in ("lnZ", "E", "C", "M"):
            assert curve_err(got[k][key][0], ref[0][key]) < 1e-8, (k, key)
