"""GPU parity of the L2-window H*v passes (XCD-aware window walk) against the CPU
oracle: small systems with tiny windows, so that many passes, both window walks
(per-XCD and flat) and ragged windows are exercised; a Lanczos run through the
multi-pass epilogue; sampled rows at the full cfg2 and cfg4 sizes."""
import numpy as np
import pytest

import ftlm_workloads as W
from oracle import ftlm as of

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _force_l2win(force_variant, plan_windows):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    force_variant(4)
    plan_windows(l2_kb=16, tile_kb=128)


def F():
    import paper_2607_25585_amd as F
    return F


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("seed,n,max_two_s,half", [(0, 6, 3, False), (1, 5, 4, False),
                                                   (2, 12, 1, True), (3, 16, 1, True),
                                                   (4, 4, 5, False), (5, 9, 2, False),
                                                   (6, 14, 1, True), (7, 7, 3, False)])
def test_l2win_hv_matches_oracle(seed, n, max_two_s, half):
    rng = np.random.default_rng(1900 + seed)
    sysm = W.random_small_system(rng, n, max_two_s=max_two_s)
    if half:
        sysm.two_s[:] = 1
    print("case l2win seed", seed, "two_s", sysm.two_s.tolist(), flush=True)
    ham = F().Hamiltonian(sysm)
    v = rng.standard_normal(ham.dim) + 1j * rng.standard_normal(ham.dim)
    oh = of.Ham(sysm)
    ref = oh.apply(v)
    w = ham.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
    assert rel_max(w, ref) < 1e-12
    w32 = ham.apply(torch.as_tensor(v, device="cuda", dtype=torch.complex64)).cpu().numpy()
    ref32 = oh.apply(v.astype(np.complex64).astype(np.complex128))
    assert rel_max(w32, ref32) < 2e-5


@pytest.mark.parametrize("n,half", [(6, False), (14, True)])
def test_l2win_run_matches_oracle(n, half):
    rng = np.random.default_rng(177 + n)
    sysm = W.random_small_system(rng, n, max_two_s=1 if half else 2)
    if half:
        sysm.two_s[:] = 1
    T = W.t_grid(30)
    ham = F().Hamiltonian(sysm)
    got = F().run(ham, 3, 40, T, seed=4, columns=1)
    ref = of.ftlm(sysm, 3, 40, T, seed=4)[0]
    for key in ("lnZ", "E", "C", "M"):
        r = np.asarray(ref[key])
        err = np.max(np.abs(got[key][0] - r) / np.maximum(np.abs(r), 1e-3 * np.abs(r).max()))
        assert err < 1e-8, key


def _sampled(sysm, prec, tol, n_rows=2000):
    ham = F().Hamiltonian(sysm)
    dim = ham.dim
    print("case l2win full-size", sysm.name, "dim", dim, "prec", prec, flush=True)
    v = F().gaussian_vectors(4243, 0, 0, 0, 1, dim).reshape(-1)
    if prec == F().FTLM_C64:
        v = v.to(torch.complex64)
    w = ham.apply(v)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    rows = np.unique(np.concatenate([rng.integers(0, dim, n_rows), [0, dim - 1, dim // 3]]))
    ri = torch.as_tensor(rows, device="cuda")
    w_s = w[ri].cpu().numpy().astype(np.complex128)
    vc = v.cpu().numpy().astype(np.complex128)
    ref = of.Ham(sysm).apply_rows(vc, rows)
    assert rel_max(w_s, ref) < tol
    del v, w
    torch.cuda.empty_cache()


@pytest.mark.parametrize("wl", ["cfg2", "cfg4", "cfg4_hb"])
def test_l2win_full_size_sampled_rows(wl, plan_windows):
    plan_windows(l2_kb=1024, tile_kb=128)
    sysm, _ = W.WORKLOADS[wl]()
    _sampled(sysm, F().FTLM_C128, 1e-12)
    _sampled(sysm, F().FTLM_C64, 2e-5)


@pytest.mark.parametrize("groups", [1, 2, 4])
@pytest.mark.parametrize("seed,n", [(0, 12), (1, 14), (2, 16), (3, 13)])
def test_tile_window_hv_matches_oracle(seed, n, groups, monkeypatch, force_variant):
    """Variant 5 (LDS tile kernel walked over L2 windows), spin 1/2, with one and
    two row groups per tile: tiny windows give many passes (N = 16: ten)."""
    force_variant(5, groups)
    rng = np.random.default_rng(2900 + seed)
    sysm = W.random_small_system(rng, n, max_two_s=1)
    sysm.two_s[:] = 1
    print("case tile-window seed", seed, "n", n, flush=True)
    ham = F().Hamiltonian(sysm)
    v = rng.standard_normal(ham.dim) + 1j * rng.standard_normal(ham.dim)
    oh = of.Ham(sysm)
    assert rel_max(ham.apply(torch.as_tensor(v, device="cuda")).cpu().numpy(), oh.apply(v)) < 1e-12
    w32 = ham.apply(torch.as_tensor(v, device="cuda", dtype=torch.complex64)).cpu().numpy()
    assert rel_max(w32, oh.apply(v.astype(np.complex64).astype(np.complex128))) < 2e-5


@pytest.mark.parametrize("groups", [1, 2, 4])
def test_tile_window_run_matches_oracle(groups, monkeypatch, force_variant):
    force_variant(5, groups)
    rng = np.random.default_rng(2950)
    sysm = W.random_small_system(rng, 15, max_two_s=1)
    sysm.two_s[:] = 1
    T = W.t_grid(30)
    ham = F().Hamiltonian(sysm)
    got = F().run(ham, 2, 30, T, seed=6, columns=1)
    ref = of.ftlm(sysm, 2, 30, T, seed=6)[0]
    for key in ("lnZ", "E", "C", "M"):
        r = np.asarray(ref[key])
        err = np.max(np.abs(got[key][0] - r) / np.maximum(np.abs(r), 1e-3 * np.abs(r).max()))
        assert err < 1e-8, key


@pytest.mark.parametrize("groups", [1, 2, 4])
def test_tile_window_full_size_sampled_rows(groups, plan_windows, force_variant):
    force_variant(5, groups)
    plan_windows(l2_kb=16, tile_kb=2048)
    sysm, _ = W.cfg2()
    _sampled(sysm, F().FTLM_C128, 1e-12)
    _sampled(sysm, F().FTLM_C64, 2e-5)


def test_tile_window_lanczos_full_size_matches_oracle(plan_windows, force_variant):
    """cfg2 at its full size (2^24 rows), in the launch the curve benchmark
    times (tile-window kernel, 512-thread tiles, 2048 blocks, 2 MB windows):
    the Lanczos coefficients of the first two steps, produced by the fused
    epilogue of the last pass and the update kernel, against the oracle's
    recursion from the same seeded start vector (oracle H*v on every row)."""
    force_variant(5, 2)
    plan_windows(l2_kb=16, tile_kb=2048)
    sysm, _ = W.cfg2()
    print("case tile-window Lanczos at full size: cfg2, seed 11, 2 steps", flush=True)
    ham = F().Hamiltonian(sysm)
    got = F().run(ham, 1, 2, np.array([1.0, 10.0]), seed=11, columns=1, return_tridiagonals=True)
    rv = of.gaussian_vector(11, 0, 0, 0, ham.dim)
    a, b, _, k = of.lanczos(of.Ham(sysm), of.Moment(sysm, of.field_direction(sysm.B)), rv, 2)
    assert k == 2 and int(got["n_lanczos_used"][0, 0]) == 2
    # absolute error on the spectral scale (the first alpha is close to zero)
    scale = float(np.max(np.abs(b)))
    assert np.max(np.abs(got["alpha"][0, 0, :2] - a)) < 1e-10 * scale
    assert np.max(np.abs(got["beta"][0, 0, :2] - b)) < 1e-10 * scale


@pytest.mark.parametrize("K", [2, 4, 8])
def test_l2win_columns_general_radix(K):
    """Variant 4 with K interleaved columns (general radix: K/kc column blocks of
    kc columns per lane), tiny windows, every column against the oracle; and a
    Lanczos run whose epilogue reduces kc columns per lane."""
    rng = np.random.default_rng(3100 + K)
    sysm = W.random_small_system(rng, 6, max_two_s=3)
    ham = F().Hamiltonian(sysm)
    v = rng.standard_normal((ham.dim, K)) + 1j * rng.standard_normal((ham.dim, K))
    oh = of.Ham(sysm)
    w = ham.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
    for c in range(K):
        assert rel_max(w[:, c], oh.apply(v[:, c])) < 1e-12, c
    T = W.t_grid(20)
    got = F().run(ham, K, 25, T, seed=8, columns=K)
    ref = of.ftlm(sysm, K, 25, T, seed=8)[0]
    for key in ("lnZ", "E", "C", "M"):
        r = np.asarray(ref[key])
        err = np.max(np.abs(got[key][0] - r) / np.maximum(np.abs(r), 1e-3 * np.abs(r).max()))
        assert err < 1e-8, key
