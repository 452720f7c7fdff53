"""GPU parity of the single-pass tile H*v (variant 6) against the CPU oracle:
elementwise on systems of many tiles (terms inside the tile, pairs with one
tile site, pairs and single flips of outer sites, ragged last rows of a thread),
sampled rows at the full sizes of the short-range workloads, and Lanczos runs
through its fused epilogue.  The variant is selected through the tuning call of
the C ABI; a Hamiltonian with row-dependent single-flip coefficients (s+- s^z
pair pieces) must be refused."""
import numpy as np
import pytest

import ftlm_workloads as W
from oracle import ftlm as of

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

STREAM = 6


@pytest.fixture(autouse=True)
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


# launch shapes of the stream kernel (the tuning's kc): block of 1024 or 256
# threads (bits 0..3 = 0 or 1), 2^(bits 4..7) tiles per XCD chunk, and (bit 8)
# the mixed pairs' partner tiles staged in LDS (not for systems of spins 1/2)
SHAPES = [0, 1, 0x40, 0x21, 0x61, 0x60]
STAGED = [0x100, 0x101, 0x140, 0x161]


def _stream_ham(sysm, grid_cap=0, kc=0):
    ham = F().Hamiltonian(sysm)
    for prec in (F().FTLM_C128, F().FTLM_C64):
        ham.set_tuning(prec, 1, STREAM, grid_cap, kc)
    return ham


def _check_full(sysm, seed, grid_cap=0, kc=0):
    rng = np.random.default_rng(seed)
    ham = _stream_ham(sysm, grid_cap, kc)
    print("case stream", sysm.name, "two_s", list(map(int, sysm.two_s)), "dim", ham.dim, "grid", grid_cap,
          "kc", kc, flush=True)
    v = rng.standard_normal(ham.dim) + 1j * rng.standard_normal(ham.dim)
    oh = of.Ham(sysm)
    w = ham.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
    assert rel_max(w, oh.apply(v)) < 1e-12
    v32 = v.astype(np.complex64)
    w32 = ham.apply(torch.as_tensor(v32, device="cuda")).cpu().numpy()
    assert rel_max(w32, oh.apply(v32.astype(np.complex128))) < 2e-5


def _no_dipolar(rng, n, max_two_s, name):
    s = W.random_small_system(rng, n, max_two_s=max_two_s, dipolar=False, name=name)
    return s


@pytest.mark.parametrize("grid_cap", [0, 8, 24])
@pytest.mark.parametrize("kc", SHAPES)
def test_stream_spin_half_all_pairs(grid_cap, kc):
    """16 spins 1/2 (16 tiles of 4096 rows at complex128, 8 of 8192 at
    complex64), exchange between all pairs and a transverse field: pairs of
    every class and single flips of tile and outer sites, every block size,
    chunked and flat tile walks."""
    rng = np.random.default_rng(61)
    s = _no_dipolar(rng, 16, 1, "half16")
    s.two_s[:] = 1
    _check_full(s, 1, grid_cap, kc)


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("kc", [0, 1, 0x41] + STAGED)
def test_stream_spin_two_ring_like(seed, kc):
    """Seven spins 2 (25 tiles of 5^5 rows): general radix, packed digits,
    complex single-ion terms along tilted axes."""
    rng = np.random.default_rng(70 + seed)
    s = _no_dipolar(rng, 7, 4, "s2x7")
    s.two_s[:] = 4
    _check_full(s, 10 + seed, 0, kc)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("kc", [0, 0x100])
def test_stream_mixed_spins(seed, kc):
    rng = np.random.default_rng(80 + seed)
    s = _no_dipolar(rng, 7 if seed < 2 else 9, 5 if seed < 2 else 3, "mixed")
    _check_full(s, 20 + seed, 0, kc)


def test_stream_single_tile_and_real_coefficients():
    """A system smaller than one tile (every term from LDS), and an isotropic
    ring in a field along z (real coefficients, no single flips)."""
    rng = np.random.default_rng(90)
    small = _no_dipolar(rng, 4, 3, "small")
    _check_full(small, 30)
    _check_full(small, 30, 0, 0x100)
    n = 13
    ring = W.System(two_s=np.ones(n, np.int32), J=W.ring_couplings(n, 1.0, 0.3), d=None,
                    e=np.tile([0.0, 0.0, 1.0], (n, 1)), g=np.full(n, 2.0), B=np.array([0.0, 0.0, 0.7]),
                    pos=None, name="ring13")
    _check_full(ring, 31)


def test_stream_staging_refused_for_spin_half():
    """Spin-1/2 systems have one move per mixed pair and row, so the staged
    launch is refused (FTLM_EINVAL) rather than run."""
    rng = np.random.default_rng(92)
    s = _no_dipolar(rng, 14, 1, "half14")
    s.two_s[:] = 1
    ham = _stream_ham(s, 0, 0x100)
    v = torch.ones(ham.dim, dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError, match="status -1"):
        ham.apply(v)


def test_stream_refuses_row_dependent_single_flips():
    rng = np.random.default_rng(91)
    s = W.random_small_system(rng, 5, max_two_s=2, dipolar=True)
    ham = _stream_ham(s)
    v = torch.ones(ham.dim, dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError):
        ham.apply(v)


def _sampled(sysm, prec, tol, n_rows=3000, kc=0, grid_cap=0):
    ham = _stream_ham(sysm, grid_cap, kc)
    dim = ham.dim
    print("case stream full size", sysm.name, "dim", dim, "prec", prec, flush=True)
    v = F().gaussian_vectors(4242, 0, 0, 0, 1, dim)[:, 0].contiguous()
    if prec == F().FTLM_C64:
        v = v.to(torch.complex64)
    w = ham.apply(v)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([rng.integers(0, dim, n_rows), [0, dim - 1, dim // 2]]))
    ri = torch.as_tensor(rows, device="cuda")
    w_s = w[ri].cpu().numpy().astype(np.complex128)
    vc = v.cpu().numpy().astype(np.complex128)
    del v, w
    torch.cuda.empty_cache()
    ref = of.Ham(sysm).apply_rows(vc, rows)
    assert rel_max(w_s, ref) < tol


@pytest.mark.parametrize("which", ["cfg4_hb", "cfg4", "cfg2_hb", "mn9"])
def test_stream_full_size_sampled_rows(which):
    sysm = getattr(W, which)()[0]
    _sampled(sysm, F().FTLM_C128, 1e-12)
    _sampled(sysm, F().FTLM_C64, 2e-5)
    _sampled(sysm, F().FTLM_C128, 1e-12, kc=0x42, grid_cap=1024)
    if which != "cfg2_hb":  # staged launches: not for spins 1/2
        _sampled(sysm, F().FTLM_C128, 1e-12, kc=0x100, grid_cap=1024)
        _sampled(sysm, F().FTLM_C64, 2e-5, kc=0x100)


@pytest.mark.parametrize("which,prec,tol,kc", [("half14", 0, 1e-8, 0), ("s2x6", 0, 1e-8, 0), ("s2x6", 1, 1e-3, 0),
                                                ("s2x6", 0, 1e-8, 0x100), ("s2x6", 1, 1e-3, 0x100)])
def test_stream_lanczos_run_matches_oracle(which, prec, tol, kc):
    """The fused Lanczos epilogue of the stream kernel inside ftlm_run."""
    rng = np.random.default_rng(95)
    if which == "half14":
        s = _no_dipolar(rng, 14, 1, which)
        s.two_s[:] = 1
    else:
        s = _no_dipolar(rng, 6, 4, which)
        s.two_s[:] = 4
    ham = _stream_ham(s, 0, kc)
    T = W.t_grid(30)
    got = F().run(ham, 2, 40, T, seed=12, columns=1, precision=prec)
    ref = of.ftlm(s, 2, 40, T, seed=12)[0]
    for key in ("lnZ", "E", "C", "M"):
        assert curve_err(got[key][0], ref[key]) < tol, key
