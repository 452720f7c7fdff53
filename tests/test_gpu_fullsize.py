"""Full-size Lanczos parity: the recursion's first coefficients at the largest
single-system size (cfg4, N=12 spins s=2, 5^12 = 244,140,625 rows), produced in
the launch the library picks by default (the H*v kernel with its fused Lanczos
epilogue and the update kernel), against the oracle's recursion from the same
seeded start vector (oracle H*v on every row).

Alpha and beta agree across implementations only until rounding drives the
loss of orthogonality; the first two steps are compared on the spectral scale
(|alpha_1| can be close to zero)."""
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
    torch.cuda.set_device(0)


def F():
    import paper_2607_25585_amd as F
    return F


def _two_steps(sysm, precision=0, seed=11):
    ham = F().Hamiltonian(sysm)
    print("case full-size Lanczos", sysm.name, "dim", ham.dim, "precision", precision, flush=True)
    got = F().run(ham, 1, 2, np.array([1.0, 10.0]), seed=seed, columns=1, precision=precision,
                  return_tridiagonals=True)
    del ham
    torch.cuda.empty_cache()
    rv = of.gaussian_vector(seed, 0, 0, 0, W.dimension(sysm.two_s))
    a, b, _, k = of.lanczos(of.Ham(sysm), of.Moment(sysm, of.field_direction(sysm.B)), rv, 2)
    del rv
    assert k == 2 and int(got["n_lanczos_used"][0, 0]) == 2
    return got, a, b


@pytest.mark.timeout(900)
@pytest.mark.parametrize("which", ["cfg4", "cfg4_hb"])
def test_cfg4_lanczos_full_size_matches_oracle(which):
    sysm, _ = getattr(W, which)()
    got, a, b = _two_steps(sysm)
    scale = float(np.max(np.abs(b)))
    assert np.max(np.abs(got["alpha"][0, 0, :2] - a)) < 1e-10 * scale
    assert np.max(np.abs(got["beta"][0, 0, :2] - b)) < 1e-10 * scale
