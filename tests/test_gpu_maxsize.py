"""Parity at the largest dimensions the library accepts (dim < 2^32): start
vectors and H*v at rows beyond 2^31, where signed or wrapping 32-bit row
arithmetic would go wrong.  The oracle reads only the vector entries that its
sampled rows touch, so its input is a zero vector written at those entries
(pages it never touches are never allocated)."""
import numpy as np
import pytest

import ftlm_workloads as W
from oracle import ftlm as of

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# 2^3 * 3^3 * 7^6 * 13^2: the one product of radices <= 16 within 2048 * 256
# rows of 2^32 (308,200 below it)
NEAR_MAX = [8, 3, 3, 3, 7, 7, 7, 7, 7, 7, 13, 13]


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.empty_cache()


def F():
    import paper_2607_25585_amd as F
    return F


def ring(radix, seed):
    """Exchange ring with single-ion anisotropy along random axes and a tilted
    field: single-site moves of one and two steps and pair moves (no s^+- s^z
    pair pieces, so every H*v variant applies)."""
    n = len(radix)
    rng = np.random.default_rng(seed)
    return W.System(two_s=np.asarray(radix, np.int32) - 1, J=W.ring_couplings(n, 0.7, 0.0),
                    d=np.full(n, -0.8), e=W.unit_vectors(rng, n), g=np.full(n, 2.0),
                    B=np.array([0.3, -0.2, 0.9]), pos=None, name="ring%d" % n)


@pytest.mark.parametrize("variant", [0, 1, 2, 4, 6])
def test_large_spins_elementwise(variant):
    """Spins up to 15/2 (radices 16, 13, 8, 3, 2): every H*v variant for
    general radix against the oracle's full product, both precisions (the
    single-pass tile kernel without the dipolar term, whose s^+- s^z pair
    pieces it does not take)."""
    rng = np.random.default_rng(40 + variant)
    s = W.random_small_system(rng, 5, dipolar=variant != 6, name="large_spins")
    s.two_s[:] = [15, 12, 7, 2, 1]
    ham = F().Hamiltonian(s)
    for prec in (F().FTLM_C128, F().FTLM_C64):
        ham.set_tuning(prec, 1, variant, 0, 0)
    print("case large spins variant", variant, "dim", ham.dim, flush=True)
    v = rng.standard_normal(ham.dim) + 1j * rng.standard_normal(ham.dim)
    ref = of.Ham(s).apply(v)
    w = ham.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
    assert np.max(np.abs(w - ref)) / np.max(np.abs(ref)) < 1e-12
    v32 = v.astype(np.complex64)
    ref32 = of.Ham(s).apply(v32.astype(np.complex128))
    w32 = ham.apply(torch.as_tensor(v32, device="cuda")).cpu().numpy()
    assert np.max(np.abs(w32 - ref32)) / np.max(np.abs(ref32)) < 2e-5
    ham.close()


def sample_rows(dim, rng, n=200):
    edge = [0, 1, dim - 1, dim - 2, (1 << 31) - 1, 1 << 31, (1 << 31) + 1]
    hi = [dim - 1 - k for k in rng.integers(0, 600000, 40)]
    return np.unique(np.clip(np.concatenate([edge, hi, rng.integers(0, dim, n)]), 0, dim - 1)).astype(np.int64)


def partners(sysm, rows):
    """Every row the oracle may read for these rows: any digit of one site, or
    one step of each of two sites."""
    radix = np.asarray(sysm.two_s, np.int64) + 1
    st = np.concatenate([[1], np.cumprod(radix)[:-1]])
    dig = (rows[:, None] // st[None, :]) % radix[None, :]
    out = [rows]
    n = len(radix)
    for k in range(n):
        for b in range(int(radix[k])):
            out.append(rows + (b - dig[:, k]) * st[k])
    for i in range(n):
        for j in range(i + 1, n):
            for a in (-1, 0, 1):
                for b in (-1, 0, 1):
                    ok = ((dig[:, i] + a >= 0) & (dig[:, i] + a < radix[i]) &
                          (dig[:, j] + b >= 0) & (dig[:, j] + b < radix[j]))
                    out.append((rows + a * st[i] + b * st[j])[ok])
    return np.unique(np.concatenate(out))


def check_rows(sysm, v, w, rows, tol):
    """w[rows] against the oracle's rows of H v, from v's entries at the
    partner rows only."""
    dim = int(v.shape[0])
    idx = partners(sysm, rows)
    vh = np.zeros(dim, np.complex128)
    vh[idx] = v[torch.as_tensor(idx, device="cuda")].cpu().numpy().astype(np.complex128)
    ref = of.Ham(sysm).apply_rows(vh, rows)
    got = w[torch.as_tensor(rows, device="cuda")].cpu().numpy().astype(np.complex128)
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    assert err < tol, err


def test_start_vectors_near_two_to_32():
    """Start vectors at dim 4,294,659,096: the grid-stride row counter passes
    2^32 - 2048 * 256 here, so a 32-bit counter would wrap and never finish."""
    dim = W.dimension(np.asarray(NEAR_MAX) - 1)
    assert (1 << 32) - 2048 * 256 < dim < (1 << 32)
    print("case start vectors dim", dim, flush=True)
    v = F().gaussian_vectors(77, 3, 1, 5, 1, dim)[:, 0]
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    idx = sample_rows(dim, rng, 2000)
    got = v[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    ref = of.gaussian_entries(77, 5, 1, 3, idx)
    assert np.max(np.abs(got - ref)) < 1e-13
    del v


@pytest.mark.parametrize("variant", [0, 1])
def test_hv_near_two_to_32_complex64(variant):
    """H*v at complex64 on the 12-site mixed ring of dim 4,294,659,096, the
    built-in launch (single-pass tile kernel) and the direct gather."""
    s = ring(NEAR_MAX, 11)
    ham = F().Hamiltonian(s)
    assert ham.dim == W.dimension(s.two_s)
    if variant:
        ham.set_tuning(F().FTLM_C64, 1, variant, 0, 0)
    print("case hv near 2^32 c64 variant", variant, "dim", ham.dim, flush=True)
    v = F().gaussian_vectors(78, 0, 0, 0, 1, ham.dim)[:, 0].to(torch.complex64)
    torch.cuda.empty_cache()
    w = ham.apply(v)
    torch.cuda.synchronize()
    check_rows(s, v, w, sample_rows(ham.dim, np.random.default_rng(variant)), 2e-5)
    del v, w
    ham.close()


def test_hv_beyond_two_to_31_complex128():
    """H*v at complex128 on 20 spins 1 (dim 3^20 = 3,486,784,401), built-in launch."""
    s = ring([3] * 20, 12)
    ham = F().Hamiltonian(s)
    print("case hv 3^20 c128 dim", ham.dim, flush=True)
    assert ham.dim > (1 << 31)
    v = F().gaussian_vectors(79, 0, 0, 0, 1, ham.dim)[:, 0]
    w = ham.apply(v)
    torch.cuda.synchronize()
    check_rows(s, v, w, sample_rows(ham.dim, np.random.default_rng(2)), 1e-12)
    del v, w
    ham.close()
