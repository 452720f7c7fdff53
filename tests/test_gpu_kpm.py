"""GPU parity of the Chebyshev (KPM) expansion of the thermal traces against the
CPU oracle on the same seeded vectors and spectral bounds, and a cross-check
against the Lanczos driver: both estimate the same per-vector traces, so where
both have converged (T above the expansion's reach) the curves coincide."""
import numpy as np
import pytest

import ftlm_workloads as W
from oracle import kpm as okpm

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


@pytest.mark.parametrize("seed,n,max_two_s,N", [(0, 4, 3, 60), (1, 6, 2, 150), (2, 9, 1, 300)])
def test_kpm_matches_oracle(seed, n, max_two_s, N):
    rng = np.random.default_rng(2600 + seed)
    sysm = W.random_small_system(rng, n, max_two_s=max_two_s)
    T = W.t_grid(40, lo=0.5)
    print("case kpm seed", seed, "two_s", sysm.two_s.tolist(), "N", N, flush=True)
    ham = F().Hamiltonian(sysm)
    got = F().run_kpm(ham, 3, N, T, seed=7, n_bound_steps=30)
    ref = okpm.kpm(sysm, 3, N, T, seed=7, n_bound=30)[0]
    assert abs(got["E_lo"][0] - ref["E_lo"]) < 1e-9 * max(1, abs(ref["E_lo"]))
    assert abs(got["E_hi"][0] - ref["E_hi"]) < 1e-9 * max(1, abs(ref["E_hi"]))
    assert np.max(np.abs(got["lnZ"][0] - ref["lnZ"])) < 1e-8
    for key in ("E", "C", "M"):
        assert curve_err(got[key][0], ref[key]) < 1e-7, key


def test_kpm_agrees_with_lanczos_where_converged():
    """cfg1 (dim 6561): the same 4 random vectors through FTLM (N_L = 100) and the
    Chebyshev expansion (N = 600); above 2 K both have converged to the same
    per-vector traces."""
    sysm, spec = W.cfg1()
    T = W.t_grid(50, lo=2.0)
    ham = F().Hamiltonian(sysm)
    lz = F().run(ham, 4, 100, T, seed=spec.seed)
    kp = F().run_kpm(ham, 4, 600, T, seed=spec.seed, n_bound_steps=60)
    assert np.max(np.abs(lz["lnZ"][0] - kp["lnZ"][0])) < 1e-9
    for key in ("E", "C", "M"):
        assert curve_err(kp[key][0], lz[key][0]) < 1e-8, key
