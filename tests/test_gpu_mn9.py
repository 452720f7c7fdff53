"""The Mn9-like centred cube of Sec. 3.3 (s=5/2 centre + 8 s=2 vertices, mixed
radix 6 and 5, dimension 2,343,750): sampled rows of H*v at full size against the
oracle for every H*v variant, and a powder-averaged FTLM over the 10 dodecahedron
directions against the oracle on the same seeded vectors."""
import os

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


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("variant", ["0", "1", "2", "4"])
def test_mn9_sampled_rows(variant, force_variant):
    force_variant(int(variant))
    sysm, spec = W.mn9()
    ham = F().Hamiltonian(sysm)
    assert ham.dim == 2343750
    print("case mn9 rows variant", variant, flush=True)
    v = F().gaussian_vectors(77, 0, 0, 0, 1, ham.dim).reshape(-1)
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([rng.integers(0, ham.dim, 3000), [0, ham.dim - 1]]))
    ri = torch.as_tensor(rows, device="cuda")
    oh = of.Ham(sysm)
    vc = v.cpu().numpy()
    ref = oh.apply_rows(vc, rows)
    w = ham.apply(v)[ri].cpu().numpy()
    assert rel_max(w, ref) < 1e-12
    w32 = ham.apply(v.to(torch.complex64))[ri].cpu().numpy().astype(np.complex128)
    ref32 = oh.apply_rows(vc.astype(np.complex64).astype(np.complex128), rows)
    assert rel_max(w32, ref32) < 2e-5


def test_mn9_powder_average_matches_oracle():
    sysm, spec = W.mn9()
    T = W.t_grid(30)
    ham = F().Hamiltonian(sysm)
    got = F().run(ham, 2, 12, T, seed=spec.seed, fields=spec.fields)
    ref = of.ftlm(sysm, 2, 12, T, seed=spec.seed, fields=spec.fields)
    for f in range(len(spec.fields)):
        assert np.max(np.abs(got["lnZ"][f] - ref[f]["lnZ"])) < 1e-8
        for key in ("E", "C", "M"):
            r = np.asarray(ref[f][key])
            err = np.max(np.abs(got[key][f] - r) / np.maximum(np.abs(r), 1e-3 * np.abs(r).max()))
            assert err < 1e-8, (f, key)
    powder = got["M"].mean(axis=0)
    assert np.all(np.isfinite(powder))
