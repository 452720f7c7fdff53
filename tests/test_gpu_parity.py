"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances: H*v in FP64 within 1e-12 of the oracle relative to max|w|; FTLM
curves in FP64 within 1e-8 with the error measure
|x - x_ref| / max(|x_ref(T)|, 1e-3 max_T |x_ref|) (max over T); FP32 storage
curves within 1e-3 of the FP64 oracle by the same measure.
"""
import numpy as np
import pytest

import ftlm_workloads as W
from oracle import ftlm as of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def F():
    import paper_2607_25585_amd as F
    return F


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def curve_err(x, ref):
    ref = np.asarray(ref)
    floor = 1e-3 * np.max(np.abs(ref))
    return float(np.max(np.abs(np.asarray(x) - ref) / np.maximum(np.abs(ref), max(floor, 1e-300))))


def _rand_v(rng, dim, K=None):
    shape = (dim,) if K is None else (dim, K)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ------------------------------------------------------------------- H*v
@pytest.mark.parametrize("seed", range(8))
def test_hv_general_c128(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 7))
    sysm = W.random_small_system(rng, n, max_two_s=5, dipolar=bool(seed % 2 == 0))
    print("case general seed", seed, "two_s", sysm.two_s.tolist(), flush=True)
    ham = F().Hamiltonian(sysm)
    v = _rand_v(rng, ham.dim)
    w = ham.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
    assert rel_max(w, of.Ham(sysm).apply(v)) < 1e-12


@pytest.mark.parametrize("K", [2, 3, 5, 8, 12])
def test_hv_columns_c128(K):
    rng = np.random.default_rng(40 + K)
    sysm = W.random_small_system(rng, 5, max_two_s=3)
    print("case columns K", K, flush=True)
    ham = F().Hamiltonian(sysm)
    v = _rand_v(rng, ham.dim, K)
    w = ham.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
    oh = of.Ham(sysm)
    for c in range(K):
        assert rel_max(w[:, c], oh.apply(v[:, c])) < 1e-12


@pytest.mark.parametrize("n,K", [(8, 1), (9, 4), (11, 2), (13, 8), (10, 3), (11, 1), (12, 1),
                                 (15, 1)])
def test_hv_spin_half_path(n, K):
    """Spin-1/2 tiles (N >= 8): dipolar pairs with s+- s^z pieces, tilted field."""
    rng = np.random.default_rng(n * 10 + K)
    sysm = W.random_small_system(rng, n, max_two_s=1)
    sysm.two_s[:] = 1
    print("case half n", n, "K", K, flush=True)
    ham = F().Hamiltonian(sysm)
    v = _rand_v(rng, ham.dim, K)
    w = ham.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
    oh = of.Ham(sysm)
    for c in range(K):
        assert rel_max(w[:, c], oh.apply(v[:, c])) < 1e-12


@pytest.mark.parametrize("n,two_s", [(8, 1), (5, 3), (4, 4)])
def test_hv_c64(n, two_s):
    rng = np.random.default_rng(77 + n)
    sysm = W.random_small_system(rng, n, max_two_s=two_s)
    if two_s == 1:
        sysm.two_s[:] = 1
    print("case c64", n, two_s, flush=True)
    ham = F().Hamiltonian(sysm)
    v = _rand_v(rng, ham.dim, 2)
    w = ham.apply(torch.as_tensor(v, device="cuda", dtype=torch.complex64)).cpu().numpy()
    oh = of.Ham(sysm)
    for c in range(2):
        ref = oh.apply(v[:, c].astype(np.complex64).astype(np.complex128))
        assert rel_max(w[:, c], ref) < 2e-5


def test_hv_tiny_and_ragged():
    rng = np.random.default_rng(3)
    for two_s in ([1], [4], [2, 3], [3] * 7):  # dim 2, 5, 12, 4^7 (not a multiple of 256... 16384 is)
        sysm = W.random_small_system(rng, len(two_s), max_two_s=4)
        sysm.two_s[:] = two_s
        print("case tiny", two_s, flush=True)
        ham = F().Hamiltonian(sysm)
        v = _rand_v(rng, ham.dim)
        w = ham.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
        assert rel_max(w, of.Ham(sysm).apply(v)) < 1e-12
    sysm = W.random_small_system(rng, 7, max_two_s=2)
    sysm.two_s[:] = 2  # 3^7 = 2187 rows: ragged last tile
    ham = F().Hamiltonian(sysm)
    v = _rand_v(rng, ham.dim)
    w = ham.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
    assert rel_max(w, of.Ham(sysm).apply(v)) < 1e-12


def test_set_field_matches_new_hamiltonian():
    rng = np.random.default_rng(9)
    sysm = W.random_small_system(rng, 4, max_two_s=3)
    ham = F().Hamiltonian(sysm)
    B2 = np.array([0.3, -1.2, 0.4])
    ham.set_field(B2)
    v = _rand_v(rng, ham.dim)
    w = ham.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
    assert rel_max(w, of.Ham(sysm, B2).apply(v)) < 1e-12


# ------------------------------------------------------------- start vectors
@pytest.mark.parametrize("seed,inst,field,r0", [(0, 0, 0, 0), (12345678901, 3, 7, 5),
                                                 (2 ** 63 + 17, 1, 0, 2)])
def test_gaussian_vectors_match_oracle(seed, inst, field, r0):
    dim, K = 5000, 3
    g = F().gaussian_vectors(seed, inst, field, r0, K, dim).cpu().numpy()
    for c in range(K):
        ref = of.gaussian_vector(seed, r0 + c, field, inst, dim)
        assert np.max(np.abs(g[:, c] - ref)) < 1e-13


# ---------------------------------------------------- Krylov eigen + Boltzmann
def test_tridiag_matches_library_eigensolver():
    import scipy.linalg
    rng = np.random.default_rng(1)
    nl, nc = 120, 37
    a = rng.standard_normal((nl, nc))
    b = np.abs(rng.standard_normal((nl, nc))) + 0.1
    y = rng.standard_normal((nl, nc))
    n_used = rng.integers(1, nl + 1, nc).astype(np.int32)
    n_used[0] = 1
    n_used[1] = nl
    dev = lambda x: torch.as_tensor(x, device="cuda")  # noqa: E731
    eps, q1, qy = [t.cpu().numpy() for t in F().tridiag_eigen(dev(a), dev(b), dev(y), dev(n_used))]
    for c in range(nc):
        k = n_used[c]
        if k == 1:
            ev, Q = np.array([a[0, c]]), np.ones((1, 1))
        else:
            ev, Q = scipy.linalg.eigh_tridiagonal(a[:k, c], b[:k - 1, c])
        order = np.argsort(eps[:k, c])
        scale = max(1.0, np.max(np.abs(ev)))
        assert np.max(np.abs(eps[:k, c][order] - ev)) < 1e-12 * scale
        assert np.max(np.abs(q1[:k, c][order] ** 2 - Q[0] ** 2)) < 1e-11
        assert np.max(np.abs((q1[:k, c] * qy[:k, c])[order] - Q[0] * (Q.T @ y[:k, c]))) < 1e-10
        assert np.all(eps[k:, c] == 0)


def test_boltzmann_matches_oracle():
    rng = np.random.default_rng(2)
    R, nl, nT = 6, 25, 40
    T = W.t_grid(nT)
    eps = np.sort(rng.uniform(-30, 30, (nl, R)), axis=0)
    q = rng.standard_normal((nl, R))
    q1 = q / np.linalg.norm(q, axis=0)
    qy = rng.standard_normal((nl, R))
    n_used = np.full(R, nl, np.int32)
    n_used[2] = 7
    for c in range(R):
        eps[n_used[c]:, c] = 0
        q1[n_used[c]:, c] = 0
    dev = lambda x: torch.as_tensor(x, device="cuda")  # noqa: E731
    lnZ, E, C, M, emin = [t.cpu().numpy() for t in
                          F().boltzmann(R, dev(eps), dev(q1), dev(qy), dev(n_used), [1234.0], T)]
    k = [slice(0, n_used[c]) for c in range(R)]
    ref = of.boltzmann(1234.0, [eps[k[c], c] for c in range(R)], [q1[k[c], c] for c in range(R)],
                       [qy[k[c], c] for c in range(R)], T)
    for key, got in (("lnZ", lnZ), ("E", E), ("C", C), ("M", M)):
        assert curve_err(got[0], ref[key]) < 1e-12, key
    assert emin[0] == ref["E_min"]


# ------------------------------------------------------------------ FTLM
def _run_pair(sysm, R, NL, T, seed, **kw):
    ham = F().Hamiltonian(sysm)
    got = F().run(ham, R, NL, T, seed=seed, **kw)
    return ham, got


def test_run_small_matches_oracle():
    rng = np.random.default_rng(31)
    sysm = W.random_small_system(rng, 4, max_two_s=3)
    T = W.t_grid(50)
    print("case run small dim", W.dimension(sysm.two_s), flush=True)
    ham, got = _run_pair(sysm, 4, 40, T, 99)
    ref = of.ftlm(sysm, 4, 40, T, seed=99)[0]
    for key in ("lnZ", "E", "C", "M"):
        assert curve_err(got[key][0], ref[key]) < 1e-8, key
    assert np.array_equal(got["n_lanczos_used"][0], ref["n_lanczos_used"])


@pytest.mark.parametrize("columns", [1, 3])
def test_run_tridiagonals_match_oracle(columns):
    """alpha_j and beta_j of the first 10 Lanczos steps of every random vector
    against the oracle's recursion on the same seeded vectors (later steps
    drift apart by rounding once the Krylov basis loses orthogonality; the
    curves built from all steps are compared in the other run tests)."""
    rng = np.random.default_rng(41)
    sysm = W.random_small_system(rng, 5, max_two_s=3)
    T = W.t_grid(20)
    dim = W.dimension(sysm.two_s)
    print("case tridiagonals dim", dim, "columns", columns, flush=True)
    assert dim >= 64
    ham, got = _run_pair(sysm, 3, 30, T, 17, columns=columns, return_tridiagonals=True)
    ref = of.ftlm(sysm, 3, 30, T, seed=17, return_columns=True)[0]
    for r in range(3):
        a, b = ref["columns"][r]["alpha"], ref["columns"][r]["beta"]
        assert len(a) >= 10 and int(got["n_lanczos_used"][0, r]) == len(a)
        scale = max(np.max(np.abs(a)), np.max(np.abs(b)))
        assert np.max(np.abs(got["alpha"][0, r, :10] - a[:10])) < 1e-10 * scale, r
        assert np.max(np.abs(got["beta"][0, r, :10] - b[:10])) < 1e-10 * scale, r


def test_run_cfg1_matches_oracle():
    """The exact-check workload (N=8, s=1 ring, dim 6561, R=20, N_L=100)."""
    sysm, spec = W.cfg1()
    ham, got = _run_pair(sysm, spec.R, spec.n_lanczos, spec.T, spec.seed)
    ref = of.ftlm(sysm, spec.R, spec.n_lanczos, spec.T, seed=spec.seed)[0]
    for key in ("lnZ", "E", "C", "M"):
        assert curve_err(got[key][0], ref[key]) < 1e-8, key


@pytest.mark.parametrize("R", [40, 64])
def test_run_one_wave_of_many_columns(R):
    """Below 2^14 rows the default wave holds every random vector (at most 64):
    curves against the oracle on the same seeded vectors."""
    rng = np.random.default_rng(50 + R)
    sysm = W.random_small_system(rng, 6, max_two_s=2)
    dim = W.dimension(sysm.two_s)
    assert 64 <= dim < (1 << 14)
    T = W.t_grid(30)
    print("case one wave R", R, "dim", dim, flush=True)
    ham, got = _run_pair(sysm, R, 30, T, 23)
    ref = of.ftlm(sysm, R, 30, T, seed=23)[0]
    for key in ("lnZ", "E", "C", "M"):
        assert curve_err(got[key][0], ref[key]) < 1e-8, key
    assert np.array_equal(got["n_lanczos_used"][0], ref["n_lanczos_used"])


def test_run_spin_half_tiles_matches_oracle():
    rng = np.random.default_rng(8)
    sysm = W.random_small_system(rng, 10, max_two_s=1)
    sysm.two_s[:] = 1
    T = W.t_grid(30)
    ham, got = _run_pair(sysm, 3, 60, T, 5, columns=3)
    ref = of.ftlm(sysm, 3, 60, T, seed=5)[0]
    for key in ("lnZ", "E", "C", "M"):
        assert curve_err(got[key][0], ref[key]) < 1e-8, key


def test_run_tile_path_matches_oracle():
    """One column per wave on a 13-site spin-1/2 system: the LDS-tile H*v kernel."""
    rng = np.random.default_rng(18)
    sysm = W.random_small_system(rng, 13, max_two_s=1)
    sysm.two_s[:] = 1
    T = W.t_grid(30)
    for prec, tol in ((F().FTLM_C128, 1e-8), (F().FTLM_C64, 1e-3)):
        ham, got = _run_pair(sysm, 2, 50, T, 6, columns=1, precision=prec)
        ref = of.ftlm(sysm, 2, 50, T, seed=6)[0]
        for key in ("lnZ", "E", "C", "M"):
            assert curve_err(got[key][0], ref[key]) < tol, (prec, key)


def test_run_fields_ragged_waves_and_r_init():
    rng = np.random.default_rng(12)
    sysm = W.random_small_system(rng, 4, max_two_s=2)
    T = W.t_grid(25)
    fields = np.array([[0.0, 0.0, 0.5], [1.0, -0.3, 0.2], [0.0, 0.0, 0.0]])
    ham = F().Hamiltonian(sysm)
    got = F().run(ham, 5, 30, T, seed=3, fields=fields, columns=2)
    ref = of.ftlm(sysm, 5, 30, T, seed=3, fields=fields)
    for f in range(3):
        for key in ("lnZ", "E", "C", "M"):
            assert curve_err(got[key][f], ref[f][key]) < 1e-8, (f, key)
    # explicit start vectors, layout (f, nu, r)
    dim = ham.dim
    starts = np.stack([np.stack([of.gaussian_vector(77, r, f, 0, dim) for r in range(5)], axis=1)
                       for f in range(3)])
    rt = torch.as_tensor(starts, device="cuda")
    got2 = F().run(ham, 5, 30, T, fields=fields, columns=5, r_init=rt)
    ref2 = of.ftlm(sysm, 5, 30, T, fields=fields, start_vectors=starts.transpose(0, 2, 1))
    for f in range(3):
        assert curve_err(got2["C"][f], ref2[f]["C"]) < 1e-8


@pytest.mark.parametrize("columns", [1, 2])
def test_run_field_scan_replans_captured_graph(columns):
    """One run over fields that change which sites have single-site flips: an
    isotropic spin-1/2 ring with B along z has none, with B along x every site
    has them, so the H*v plan and its launch arguments change between fields.
    Every field must match the oracle (the Lanczos graph is captured again when
    the launch layout changes)."""
    n = 12
    sysm = W.System(two_s=np.ones(n, np.int32), J=W.ring_couplings(n, 1.0), d=None,
                    e=np.tile([0.0, 0.0, 1.0], (n, 1)), g=np.full(n, 2.0),
                    B=np.array([0.0, 0.0, 0.5]), pos=None, name="ring12")
    T = W.t_grid(30)
    fields = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.5], [0.5, 0.0, 0.0], [0.0, 0.0, 0.5],
                       [0.0, 0.3, 0.4]])
    print("case field scan ring12 columns", columns, flush=True)
    ham = F().Hamiltonian(sysm)
    got = F().run(ham, 2, 40, T, seed=21, fields=fields, columns=columns)
    ref = of.ftlm(sysm, 2, 40, T, seed=21, fields=fields)
    for f in range(len(fields)):
        for key in ("lnZ", "E", "C", "M"):
            assert curve_err(got[key][f], ref[f][key]) < 1e-8, (f, key)


def test_breakdown_reported():
    """dim < N_L: the recursion stops in an invariant subspace."""
    sysm = W.random_small_system(np.random.default_rng(5), 2, max_two_s=1)
    sysm.two_s[:] = 1  # dim 4
    T = W.t_grid(10)
    ham, got = _run_pair(sysm, 2, 10, T, 1)
    assert np.all(got["n_lanczos_used"] <= 4)
    ref = of.ftlm(sysm, 2, 10, T, seed=1)[0]
    assert np.array_equal(got["n_lanczos_used"][0], ref["n_lanczos_used"])
    for key in ("lnZ", "E", "C", "M"):
        assert np.all(np.isfinite(got[key]))
        assert curve_err(got[key][0], ref[key]) < 1e-8, key


def test_fp32_storage_within_budget():
    sysm, spec = W.cfg1()
    ham, got = _run_pair(sysm, 8, spec.n_lanczos, spec.T, spec.seed, precision=F().FTLM_C64)
    ref = of.ftlm(sysm, 8, spec.n_lanczos, spec.T, seed=spec.seed)[0]
    for key in ("C", "E", "M"):
        assert curve_err(got[key][0], ref[key]) < 1e-3, key


def test_run_is_bitwise_deterministic():
    rng = np.random.default_rng(4)
    sysm = W.random_small_system(rng, 9, max_two_s=1)
    sysm.two_s[:] = 1
    T = W.t_grid(20)
    ham = F().Hamiltonian(sysm)
    a = F().run(ham, 4, 40, T, seed=8, columns=4)
    b = F().run(ham, 4, 40, T, seed=8, columns=4)
    for key in ("lnZ", "E", "C", "M"):
        assert np.array_equal(a[key], b[key])


# ------------------------------------------------- full-size sampled rows
def _sampled_rows_check(sysm, K, prec, tol, n_rows=3000):
    ham = F().Hamiltonian(sysm)
    dim = ham.dim
    print("case full-size", sysm.name, "dim", dim, "K", K, "prec", prec, flush=True)
    v = F().gaussian_vectors(4242, 0, 0, 0, K, dim)
    if prec == F().FTLM_C64:
        v = v.to(torch.complex64)
    w = ham.apply(v)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([rng.integers(0, dim, n_rows), [0, dim - 1, dim // 2]]))
    ri = torch.as_tensor(rows, device="cuda")
    w_s = w[ri].cpu().numpy().astype(np.complex128)
    oh = of.Ham(sysm)
    for c in range(min(K, 3)):
        vc = v[:, c].cpu().numpy().astype(np.complex128)
        ref = oh.apply_rows(vc, rows)
        assert rel_max(w_s[:, c], ref) < tol, c
    del v, w
    torch.cuda.empty_cache()


def test_cfg2_full_size_sampled_rows():
    sysm, spec = W.cfg2()
    _sampled_rows_check(sysm, spec.R, F().FTLM_C128, 1e-12)
    _sampled_rows_check(sysm, 1, F().FTLM_C128, 1e-12)
    _sampled_rows_check(sysm, 1, F().FTLM_C64, 2e-5)


def test_cfg4_full_size_sampled_rows():
    sysm, spec = W.cfg4()
    _sampled_rows_check(sysm, 1, F().FTLM_C128, 1e-12)
    _sampled_rows_check(sysm, 2, F().FTLM_C64, 2e-5)


def test_autotune_keeps_parity(tmp_path, monkeypatch):
    monkeypatch.setenv("FTLM_TUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_2607_25585_amd import autotune
    rng = np.random.default_rng(55)
    sysm = W.random_small_system(rng, 12, max_two_s=1)
    sysm.two_s[:] = 1
    ham = F().Hamiltonian(sysm)
    c1 = autotune.tune(ham, F().FTLM_C128, 1)
    c2 = autotune.tune(ham, F().FTLM_C128, 1)
    assert not c1["cached"] and c2["cached"] and c1["variant"] in (1, 2, 3, 4, 5)
    v = _rand_v(rng, ham.dim)
    w = ham.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
    assert rel_max(w, of.Ham(sysm).apply(v)) < 1e-12
