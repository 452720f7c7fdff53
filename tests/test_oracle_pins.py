"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test names what pins it: a printed value, a closed form, an identity or a
brute-force construction.  None re-types the oracle's own formula.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import ftlm_workloads as W
from oracle import dense
from oracle import ftlm as of

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _sys(two_s, J=None, d=None, e=None, g=None, B=(0, 0, 0), pos=None):
    n = len(two_s)
    return W.System(two_s=np.asarray(two_s, np.int32),
                    J=None if J is None else np.asarray(J, float),
                    d=None if d is None else np.asarray(d, float),
                    e=np.tile([0.0, 0.0, 1.0], (n, 1)) if e is None else np.asarray(e, float),
                    g=np.full(n, 2.0) if g is None else np.asarray(g, float),
                    B=np.asarray(B, float), pos=None if pos is None else np.asarray(pos, float))


def _dense_from_c(system, B=None):
    """Full matrix of the C oracle's H*v, by applying it to every unit vector."""
    ham = of.Ham(system, B)
    H = np.zeros((ham.dim, ham.dim), np.complex128)
    for k in range(ham.dim):
        e = np.zeros(ham.dim, np.complex128)
        e[k] = 1.0
        H[:, k] = ham.apply(e)
    return H


# ---------------------------------------------------------------- C1 dimension
def test_dimension_printed_values():
    g = json.load(open(GOLDEN))
    assert W.dimension(g["mn9_dimension"]["two_s"]) == g["mn9_dimension"]["value"]
    assert W.dimension(g["ring_dimension"]["two_s"]) == g["ring_dimension"]["value"]
    s = _sys([5, 4, 4, 4, 4, 4, 4, 4, 4])
    assert of.Ham(s).dim == 2343750


# ------------------------------------------------------------- spin matrices
@pytest.mark.parametrize("two_s", [1, 2, 3, 4, 5])
def test_spin_algebra(two_s):
    """[s_x, s_y] = i s_z (cyclic) and s^2 = s(s+1): fixes the sign of s_y."""
    s = two_s / 2
    for sx, sy, sz in (dense.spin_matrices(two_s)[:3], of.spin_matrices(two_s)):
        assert np.allclose(sx @ sy - sy @ sx, 1j * sz, atol=1e-14)
        assert np.allclose(sy @ sz - sz @ sy, 1j * sx, atol=1e-14)
        assert np.allclose(sz @ sx - sx @ sz, 1j * sy, atol=1e-14)
        assert np.allclose(sx @ sx + sy @ sy + sz @ sz, s * (s + 1) * np.eye(two_s + 1), atol=1e-13)
        # |m> ascending: s_z diagonal -s..s
        assert np.allclose(np.diag(sz).real, -s + np.arange(two_s + 1))


# ---------------------------------------------------------- C3 closed forms
def _spectra(system):
    return (np.linalg.eigvalsh(dense.hamiltonian_dense(system)),
            np.linalg.eigvalsh(_dense_from_c(system)))


@pytest.mark.parametrize("s1,s2", [(1, 1), (2, 3), (5, 4)])
def test_dimer_heisenberg_zeeman(s1, s2):
    """2J s1.s2 + g mu_B B.S: E = J[S(S+1) - s1(s1+1) - s2(s2+1)] + g mu_B |B| M."""
    J = 0.7
    B = np.array([0.3, -0.8, 0.5])
    sysm = _sys([s1, s2], J=[[0, J], [0, 0]], B=B, g=[2.1, 2.1])
    a, b = s1 / 2, s2 / 2
    ref = []
    for S2 in range(abs(s1 - s2), s1 + s2 + 1, 2):
        S = S2 / 2
        for k in range(S2 + 1):
            M = -S + k
            ref.append(J * (S * (S + 1) - a * (a + 1) - b * (b + 1))
                       + 2.1 * dense.MU_B_K_PER_T * np.linalg.norm(B) * M)
    ref = np.sort(ref)
    for ev in _spectra(sysm):
        assert np.allclose(np.sort(ev), ref, atol=1e-12)


def test_kambe_square():
    """Square ring, 2J sum s_i.s_{i+1} = J[S^2 - S13^2 - S24^2] (Kambe), plus Zeeman."""
    two_s = [2, 2, 2, 2]
    J = W.ring_couplings(4, 0.9)
    B = np.array([0.0, 0.4, -0.2])
    sysm = _sys(two_s, J=J, B=B)
    ref = []
    for S13 in range(0, 3):
        for S24 in range(0, 3):
            for S in range(abs(S13 - S24), S13 + S24 + 1):
                for M in range(-S, S + 1):
                    ref.append(0.9 * (S * (S + 1) - S13 * (S13 + 1) - S24 * (S24 + 1))
                               + 2.0 * dense.MU_B_K_PER_T * np.linalg.norm(B) * M)
    for ev in _spectra(sysm):
        assert np.allclose(np.sort(ev), np.sort(ref), atol=1e-11)


@pytest.mark.parametrize("two_s", [2, 3, 5])
def test_single_ion_field_along_axis(two_s):
    """d (s.e)^2 + g mu_B B.s with B || e: E = d m^2 + g mu_B |B| m."""
    e = np.array([0.3, -0.5, 0.81])
    e = e / np.linalg.norm(e)
    B = 1.7 * e
    d = -2.3
    sysm = _sys([two_s], d=[d], e=[e], B=B, g=[1.95])
    m = -two_s / 2 + np.arange(two_s + 1)
    ref = np.sort(d * m ** 2 + 1.95 * dense.MU_B_K_PER_T * 1.7 * m)
    for ev in _spectra(sysm):
        assert np.allclose(np.sort(ev), ref, atol=1e-12)


def test_dipolar_dimer_closed_form():
    """Two s=1/2: D(s1.s2 - 3 (s1.e)(s2.e)) has levels {-D/2, -D/2, 0, D},
    D = mu0 mu_B^2 g1 g2 / (4 pi r^3)."""
    pos = np.array([[0.1, 0.2, -0.3], [0.35, -0.05, 0.12]])
    g = [2.0, 2.2]
    r = np.linalg.norm(pos[1] - pos[0])
    D = dense.C_DIP_K_NM3 * g[0] * g[1] / r ** 3
    sysm = _sys([1, 1], pos=pos, g=g)
    ref = np.sort([-D / 2, -D / 2, 0.0, D])
    for ev in _spectra(sysm):
        assert np.allclose(np.sort(ev), ref, atol=1e-15)


def test_rotation_and_field_reversal_invariance():
    rng = np.random.default_rng(11)
    sysm = W.random_small_system(rng, 4, max_two_s=3)
    ev0 = np.linalg.eigvalsh(_dense_from_c(sysm))
    Rm = scipy.linalg.expm(np.cross(np.eye(3), rng.standard_normal(3)))  # random rotation
    rot = W.System(two_s=sysm.two_s, J=sysm.J, d=sysm.d, e=sysm.e @ Rm.T, g=sysm.g,
                   B=Rm @ sysm.B, pos=sysm.pos @ Rm.T)
    assert np.allclose(np.linalg.eigvalsh(_dense_from_c(rot)), ev0, atol=1e-11)
    assert np.allclose(np.linalg.eigvalsh(_dense_from_c(sysm, -sysm.B)), ev0, atol=1e-11)


def test_decoupled_ions_additive():
    rng = np.random.default_rng(3)
    two_s = [2, 3, 4]
    e = W.unit_vectors(rng, 3)
    sysm = _sys(two_s, d=[-1.0, 2.0, 0.5], e=e, B=[0.2, 0.7, -1.1], g=[2.0, 1.9, 2.1])
    T = W.t_grid(20)
    full = dense.exact_thermo(sysm, T)
    parts = [dense.exact_thermo(_sys([two_s[i]], d=[sysm.d[i]], e=[e[i]], B=sysm.B, g=[sysm.g[i]]), T)
             for i in range(3)]
    assert np.allclose(full["lnZ"], sum(p["lnZ"] for p in parts), rtol=1e-12, atol=1e-12)
    assert np.allclose(full["M"], sum(p["M"] for p in parts), rtol=1e-10, atol=1e-12)


def _brillouin(s, x):
    a = (2 * s + 1) / (2 * s)
    b = 1 / (2 * s)
    return a / np.tanh(a * x) - b / np.tanh(b * x)


def test_brillouin_magnetisation():
    """Free spins: M = g s B_s(g s mu_B B / T) per spin, positive along B."""
    B = np.array([0.5, -0.5, 1.0])
    sysm = _sys([3, 3], B=B, g=[2.0, 2.0])
    T = W.t_grid(30)
    res = dense.exact_thermo(sysm, T)
    s = 1.5
    x = 2.0 * s * dense.MU_B_K_PER_T * np.linalg.norm(B) / T
    assert np.allclose(res["M"], 2 * 2.0 * s * _brillouin(s, x), rtol=1e-10)


# ------------------------------------------------------------- C4 traces
def test_trace_identities():
    rng = np.random.default_rng(5)
    sysm = W.random_small_system(rng, 4, max_two_s=3)
    for H in (dense.hamiltonian_dense(sysm), _dense_from_c(sysm)):
        dim = H.shape[0]
        s = sysm.two_s / 2
        c = s * (s + 1) / 3
        q = s * (s + 1) * (3 * s ** 2 + 3 * s - 1) / 15
        dc = sysm.d * c
        t1 = dc.sum()
        b = dense.MU_B_K_PER_T * sysm.g * np.linalg.norm(sysm.B)
        t2 = t1 ** 2 - (dc ** 2).sum() + (sysm.d ** 2 * q + b ** 2 * c).sum()
        n = len(s)
        for i in range(n):
            for j in range(i + 1, n):
                r = np.linalg.norm(sysm.pos[j] - sysm.pos[i])
                D = dense.C_DIP_K_NM3 * sysm.g[i] * sysm.g[j] / r ** 3
                t2 += (12 * sysm.J[i, j] ** 2 + 6 * D ** 2) * c[i] * c[j]
        assert abs(np.trace(H).real / dim - t1) < 1e-12
        assert abs(np.trace(H @ H).real / dim - t2) < 1e-11 * max(1, abs(t2))


# --------------------------------------------------- C5 matrix-free H*v
@pytest.mark.parametrize("seed", range(6))
def test_c_hv_matches_dense_kronecker(seed):
    """Brute force: the C oracle's matrix-free H*v equals the Kronecker-built
    matrix times v element by element (separates H from its conjugate)."""
    rng = np.random.default_rng(100 + seed)
    sysm = W.random_small_system(rng, int(rng.integers(2, 6)), max_two_s=4)
    H = dense.hamiltonian_dense(sysm)
    v = rng.standard_normal(H.shape[0]) + 1j * rng.standard_normal(H.shape[0])
    w = of.hv(sysm, v)
    assert np.max(np.abs(w - H @ v)) <= 1e-13 * np.max(np.abs(H @ v))
    assert np.linalg.norm(H - H.conj()) > 1e-3  # the case really is complex


def test_hermitian_and_time_reversal():
    rng = np.random.default_rng(21)
    sysm = W.random_small_system(rng, 5, max_two_s=3)
    ham = of.Ham(sysm)
    dim = ham.dim
    x = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
    y = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
    assert abs(np.vdot(x, ham.apply(y)) - np.vdot(ham.apply(x), y)) < 1e-12 * dim
    # Theta x: index nu -> dim-1-nu, sign (-1)^{sum(2 s_i - d_i)}, complex conjugation
    digits = np.zeros((dim, len(sysm.two_s)), int)
    rest = np.arange(dim)
    for i, t in enumerate(sysm.two_s):
        digits[:, i] = rest % (t + 1)
        rest //= (t + 1)
    sign = (-1.0) ** ((sysm.two_s[None, :] - digits).sum(1))

    def theta(z):
        out = np.empty_like(z)
        out[dim - 1 - np.arange(dim)] = sign * np.conj(z)
        return out
    lhs = theta(ham.apply(x))
    rhs = of.Ham(sysm, -sysm.B).apply(theta(x))
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(lhs))


def test_sz_sectors_preserved():
    """No anisotropy, no dipolar, B || z: total M is conserved."""
    sysm = _sys([1, 2, 3, 1, 2], J=np.triu(np.ones((5, 5)), 1) * 0.4, B=[0, 0, 0.8])
    ham = of.Ham(sysm)
    dims = [t + 1 for t in sysm.two_s]
    Mtot = np.zeros(ham.dim)
    rest = np.arange(ham.dim)
    for t in sysm.two_s:
        Mtot += rest % (t + 1) - t / 2
        rest //= (t + 1)
    rng = np.random.default_rng(0)
    for M in np.unique(Mtot):
        x = np.where(Mtot == M, rng.standard_normal(ham.dim), 0).astype(np.complex128)
        w = ham.apply(x)
        assert np.max(np.abs(w[Mtot != M])) < 1e-14


# ---------------------------------------------------------------- C6 Lanczos
def test_lanczos_moments():
    """sum_n Q_1n^2 eps_n^k = <v1|H^k|v1> for k < 2 N_L."""
    sysm, _ = W.cfg1()
    sysm = _sys([2] * 6, J=W.ring_couplings(6, 1.0), d=[-2.0] * 6, e=sysm.e[:6], B=[0, 0, 1])
    ham = of.Ham(sysm)
    r = of.gaussian_vector(7, 0, 0, 0, ham.dim)
    a, b, y, k = of.lanczos(ham, None, r, 8)
    eps, q1, _ = of.krylov_eigen(a, b)
    v = r / np.linalg.norm(r)
    hk = v.copy()
    for p in range(0, 12):
        mom_exact = np.vdot(v, hk).real
        mom_krylov = np.sum(q1 ** 2 * eps ** p)
        assert abs(mom_exact - mom_krylov) <= 1e-11 * max(1.0, abs(mom_exact)), p
        hk = ham.apply(hk)


def test_invariant_subspace_is_exact():
    """dim <= N_L with re-orthogonalisation: the Krylov estimate of
    <r|exp(-H/T)|r> and <r|O exp(-H/T)|r> equals the dense value."""
    rng = np.random.default_rng(9)
    sysm = W.random_small_system(rng, 3, max_two_s=2)
    H = dense.hamiltonian_dense(sysm)
    O = dense.moment_operator(sysm).toarray()
    ham, mom = of.Ham(sysm), of.Moment(sysm, of.field_direction(sysm.B))
    r = of.gaussian_vector(3, 1, 0, 0, ham.dim)
    a, b, y, k = of.lanczos(ham, mom, r, ham.dim + 4, reorth=True)
    eps, q1, u = of.krylov_eigen(a, b, y)
    v = r / np.linalg.norm(r)
    for t in (0.3, 2.0, 20.0):
        E = scipy.linalg.expm(-H / t)
        z_ref = np.vdot(v, E @ v).real
        assert abs(np.sum(np.exp(-eps / t) * q1 ** 2) - z_ref) < 1e-10 * z_ref
        m_kr = np.sum(np.exp(-eps / t) * q1 * np.real(u))
        assert abs(m_kr - np.vdot(v, O @ E @ v).real) < 1e-10 * z_ref


def test_all_basis_vectors_give_exact_thermo():
    """Start vectors = every basis vector (R = dim): Eq. (E-2-D) becomes the exact trace."""
    rng = np.random.default_rng(4)
    sysm = W.random_small_system(rng, 3, max_two_s=2)
    ham = of.Ham(sysm)
    dim = ham.dim
    starts = np.eye(dim, dtype=np.complex128)[None]
    T = W.t_grid(15)
    res = of.ftlm(sysm, dim, dim + 2, T, start_vectors=starts, reorth=True)[0]
    ex = dense.exact_thermo(sysm, T)
    for key in ("lnZ", "E", "C", "M"):
        assert np.allclose(res[key], ex[key], rtol=1e-9, atol=1e-10), key


# ---------------------------------------------------------- C7 tridiagonal
def test_tridiagonal_toeplitz():
    n, a, b = 37, 0.3, -1.2
    eps, q1, _ = of.krylov_eigen(np.full(n, a), np.full(n, b))
    ref = np.sort(a + 2 * b * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    assert np.allclose(eps, ref, atol=1e-13 * 3)


# ---------------------------------------------------------- C10 Boltzmann
def test_boltzmann_schottky():
    """Two levels -D/2, +D/2 with equal weights: C = (D/T)^2 e^{D/T}/(1+e^{D/T})^2."""
    Dl = 3.0
    T = W.t_grid(50)
    res = of.boltzmann(2, [np.array([-Dl / 2, Dl / 2])], [np.full(2, 1 / np.sqrt(2))],
                       [np.zeros(2)], T)
    x = Dl / T
    ref = x ** 2 * np.exp(-x) / (1 + np.exp(-x)) ** 2
    assert np.allclose(res["C"], ref, rtol=1e-12, atol=1e-300)
    assert np.allclose(res["lnZ"], np.log(2 * np.cosh(Dl / (2 * T))), rtol=1e-13)


def test_high_temperature_limit():
    """C T^2 -> <H^2> - <H>^2 as T -> infinity (exact diagonalisation)."""
    rng = np.random.default_rng(6)
    sysm = W.random_small_system(rng, 3, max_two_s=2)
    H = dense.hamiltonian_dense(sysm)
    dim = H.shape[0]
    var = np.trace(H @ H).real / dim - (np.trace(H).real / dim) ** 2
    T = np.array([1e5])
    res = dense.exact_thermo(sysm, T)
    assert abs(res["C"][0] * T[0] ** 2 - var) < 1e-3 * var


# ---------------------------------------------------------- RNG pins
def test_philox_known_answers():
    """Published known-answer vectors of Philox4x32-10 (Random123 distribution)."""
    assert of.philox4x32_10([0, 0, 0, 0], [0, 0]) == [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]
    assert of.philox4x32_10([0xffffffff] * 4, [0xffffffff] * 2) == \
        [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]
    assert of.philox4x32_10([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344],
                            [0xa4093822, 0x299f31d0]) == [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]


def test_gaussian_vector_statistics():
    """Re and Im i.i.d. N(0,1): mean 0, variance 1 each, uncorrelated."""
    z = of.gaussian_vector(123, 2, 1, 0, 400000)
    n = len(z)
    for x in (z.real, z.imag):
        assert abs(x.mean()) < 5 / math.sqrt(n)
        assert abs(x.var() - 1) < 5 * math.sqrt(2 / n)
        assert abs(np.mean(x ** 4) - 3) < 0.05
    assert abs(np.mean(z.real * z.imag)) < 5 / math.sqrt(n)
    z2 = of.gaussian_vector(123, 3, 1, 0, 1000)
    assert not np.allclose(z[:1000], z2)
    assert np.array_equal(of.gaussian_vector(123, 2, 1, 0, 1000), z[:1000])


def test_gaussian_entries_are_the_vector_components():
    """Listed components equal the whole vector's, in any order and repeated;
    a component depends on its index alone, not on the dimension."""
    z = of.gaussian_vector(321, 4, 2, 7, 5000)
    idx = np.array([4999, 0, 17, 17, 2500, 1])
    assert np.array_equal(of.gaussian_entries(321, 4, 2, 7, idx), z[idx])
    assert np.array_equal(of.gaussian_entries(321, 4, 2, 7, np.array([], np.int64)), np.zeros(0, complex))
    assert of.gaussian_vector(321, 4, 2, 7, 18)[17] == z[17]


# ------------------------------------------------------ C8 FTLM vs exact
def test_ftlm_statistical_vs_exact():
    """FTLM (Eqs. E-2-C, E-2-D) against exact diagonalisation: the exact curve
    lies inside a 4-sigma jackknife band over the random vectors, and the error
    shrinks as R grows."""
    base, _ = W.cfg1()
    sysm = _sys([2] * 6, J=W.ring_couplings(6, 1.0), d=[-2.0] * 6, e=base.e[:6], B=[0, 0, 1])
    T = W.t_grid(40)
    ex = dense.exact_thermo(sysm, T)
    R = 24
    res = of.ftlm(sysm, R, 60, T, seed=77, return_columns=True)[0]
    # jackknife over random vectors for C
    ham_dim = 3 ** 6
    loo = []
    for k in range(R):
        keep = [i for i in range(R) if i != k]
        b = of.boltzmann(ham_dim, [res["eps"][i] for i in keep], [res["q1"][i] for i in keep],
                         [np.zeros_like(res["q1"][i]) for i in keep], T)
        loo.append(b["C"])
    loo = np.array(loo)
    sig = np.sqrt((R - 1) / R * ((loo - loo.mean(0)) ** 2).sum(0))
    assert np.all(np.abs(res["C"] - ex["C"]) <= 4 * sig + 1e-3 * ex["C"].max())
    # error shrinks with R
    big = of.ftlm(sysm, 8 * R, 60, T, seed=78)[0]
    err_small = np.sqrt(np.mean((res["C"] - ex["C"]) ** 2))
    err_big = np.sqrt(np.mean((big["C"] - ex["C"]) ** 2))
    assert err_big < err_small


# ---------------------------------------------------------- C12 MLP oracle
def test_mlp_gradient_finite_differences():
    from oracle import mlp
    rng = np.random.default_rng(0)
    params = mlp.init_params(rng, (7, 16, 12, 9, 3))
    params = [p + 0.05 * rng.standard_normal(p.shape) for p in params]
    x = rng.standard_normal((5, 7))
    t = rng.standard_normal((5, 3))
    loss, grads = mlp.loss_and_grad(params, x, t)
    h = 1e-6
    for k, p in enumerate(params):
        flat = p.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grad(params, x, t)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grad(params, x, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = grads[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (k, idx, fd, an)


def test_adam_first_step_closed_form():
    """With zero moments, the first bias-corrected step is -lr g/(|g| + eps)."""
    from oracle import mlp
    g = [np.array([0.3, -2.0, 1e-3])]
    p, m, v = mlp.adam_step([np.zeros(3)], g, [np.zeros(3)], [np.zeros(3)], 1, lr=0.01)
    assert np.allclose(p[0], -0.01 * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-12)


def test_adam_bias_correction_over_five_steps():
    """Kingma and Ba's bias correction divides the moments by 1 - beta^t.  With
    a constant gradient g, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so every
    bias-corrected step is exactly -lr g/(|g| + eps).  Steps 2..5 separate the
    exponent t from a factor t (1 - b^t and 1 - b t agree only at t = 1), and
    the moments themselves are checked against their closed forms."""
    from oracle import mlp
    g = np.array([0.3, -2.0, 1e-3, 7.5])
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    p, m, v = [np.zeros(4)], [np.zeros(4)], [np.zeros(4)]
    for t in range(1, 6):
        p_old = p[0].copy()
        p, m, v = mlp.adam_step(p, [g], m, v, t, lr=lr, b1=b1, b2=b2, eps=eps)
        assert np.allclose(m[0], (1 - b1 ** t) * g, rtol=1e-13, atol=0)
        assert np.allclose(v[0], (1 - b2 ** t) * g * g, rtol=1e-12, atol=0)
        step = p[0] - p_old
        assert np.allclose(step, -lr * g / (np.abs(g) + eps), rtol=1e-9, atol=0), t
    assert np.allclose(p[0], -5 * lr * g / (np.abs(g) + eps), rtol=1e-9)


@pytest.mark.parametrize("seed,max_two_s", [(71, 1), (72, 3), (73, 5), (74, 5)])
def test_c_hv_rows_equal_full_product_rows(seed, max_two_s):
    """The sampled-row product that the full-size parity tests use as reference
    (``Ham.apply_rows``) equals the pinned full product (``Ham.apply``, itself
    pinned elementwise to the dense Kronecker H) bit for bit, on random
    mixed-spin systems with every term switched on, for the first and last
    rows, duplicates and random rows."""
    rng = np.random.default_rng(seed)
    sysm = W.random_small_system(rng, 5 if max_two_s < 5 else 4, max_two_s=max_two_s)
    ham = of.Ham(sysm)
    v = rng.standard_normal(ham.dim) + 1j * rng.standard_normal(ham.dim)
    full = ham.apply(v)
    rows = np.concatenate([[0, ham.dim - 1, 0, ham.dim - 1, ham.dim // 2, ham.dim // 2],
                           rng.integers(0, ham.dim, 40)]).astype(np.int64)
    got = ham.apply_rows(v, rows)
    assert got.shape == rows.shape
    assert np.array_equal(got.view(np.float64), full[rows].view(np.float64))
    # every row at once, in reverse order
    allr = np.arange(ham.dim - 1, -1, -1, dtype=np.int64)
    assert np.array_equal(ham.apply_rows(v, allr).view(np.float64), full[allr].view(np.float64))


def _radial_ring(n, J, d, tilt, bmag, theta, phi):
    """The surrogate workload's ring construction for n sites: uniform
    nearest-neighbour J, single-ion d along axes tilted by `tilt` towards the
    radial directions phi_i = 2 pi i/n, g = 2, no dipolar term."""
    ang = 2 * np.pi * np.arange(n) / n
    e = np.stack([np.sin(tilt) * np.cos(ang), np.sin(tilt) * np.sin(ang), np.full(n, np.cos(tilt))], axis=1)
    B = bmag * np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])
    return W.System(two_s=np.full(n, 3, np.int32), J=W.ring_couplings(n, J), d=np.full(n, d), e=e,
                    g=np.full(n, 2.0), B=B, pos=None)


def test_radial_ring_depends_on_field_azimuth_through_cos_n_phi():
    """The surrogate's input encoding rests on a symmetry of its ring: with
    radially tilted axes, rotating the field by 2 pi/n about the ring axis, or
    reflecting its azimuth (a mirror of the ring combined with time reversal),
    leaves ln Z, C and M unchanged (exact diagonalisation of a four-site
    s=3/2 ring), while a rotation by pi/n does not."""
    T = W.t_grid(12)
    n = 4
    for phi in (0.3, 1.1):
        ref = dense.exact_thermo(_radial_ring(n, 1.3, -2.2, 0.6, 2.5, 0.9, phi), T)
        for phi2 in (phi + 2 * np.pi / n, -phi, 2 * np.pi / n - phi):
            got = dense.exact_thermo(_radial_ring(n, 1.3, -2.2, 0.6, 2.5, 0.9, phi2), T)
            for k in ("lnZ", "C", "M"):
                assert np.max(np.abs(got[k] - ref[k])) < 1e-10 * max(1.0, np.max(np.abs(ref[k]))), (phi2, k)
        half = dense.exact_thermo(_radial_ring(n, 1.3, -2.2, 0.6, 2.5, 0.9, phi + np.pi / n), T)
        assert np.max(np.abs(half["C"] - ref["C"])) > 1e-5


# ------------------------------------------------ next row: sFTLM, time reversal
def test_oracle_time_reverse_maps_h_b_to_h_minus_b():
    """The oracle's Theta (used for the random-vector pairs) satisfies
    Theta H(B) Theta^-1 = H(-B) on the C oracle's H (brute-force products) and
    Theta^2 = (-1)^{2 S_tot} (Kramers)."""
    rng = np.random.default_rng(31)
    sysm = W.random_small_system(rng, 4, max_two_s=3)
    ham_p, ham_m = of.Ham(sysm), of.Ham(sysm, -np.asarray(sysm.B))
    x = rng.standard_normal(ham_p.dim) + 1j * rng.standard_normal(ham_p.dim)
    lhs = of.time_reverse(sysm.two_s, ham_p.apply(x))
    rhs = ham_m.apply(of.time_reverse(sysm.two_s, x))
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(lhs))
    tt = of.time_reverse(sysm.two_s, of.time_reverse(sysm.two_s, x))
    sign = (-1.0) ** int(np.sum(sysm.two_s))
    assert np.max(np.abs(tt - sign * x)) < 1e-15 * np.max(np.abs(x))


def test_sftlm_invariant_subspace_is_exact():
    """dim <= N_L with re-orthogonalisation: the double sum of Eq. (E-2-H)
    equals <r|exp(-H/2T) O exp(-H/2T)|r> from the dense matrices, so sFTLM over
    the pairs equals the dense ratio of Eq. (E-2-G)."""
    rng = np.random.default_rng(12)
    sysm = W.random_small_system(rng, 3, max_two_s=2)
    H = dense.hamiltonian_dense(sysm)
    O = dense.moment_operator(sysm).toarray()
    dim = H.shape[0]
    T = np.array([0.4, 3.0, 30.0])
    R = 4
    res = of.sftlm(sysm, R, dim + 3, T, seed=5, reorth=True)[0]
    vs = []
    for p in range(R // 2):
        r0 = of.gaussian_vector(5, p, 0, 0, dim)
        for rv in (r0, of.time_reverse(sysm.two_s, r0)):
            vs.append(rv / np.linalg.norm(rv))
    ev, U = np.linalg.eigh(H)
    for k, t in enumerate(T):
        half = (U * np.exp(-(ev - ev[0]) / (2 * t))) @ U.conj().T
        num = sum(np.vdot(half @ v, O @ (half @ v)).real for v in vs)
        den = sum(np.vdot(half @ v, half @ v).real for v in vs)
        assert abs(res["M"][k] - num / den) < 1e-10 * max(1.0, abs(num / den))
        z = den * dim / R * np.exp(-ev[0] / t)
        assert abs(res["lnZ"][k] - np.log(z)) < 1e-10


def test_sftlm_pairs_zero_field_and_field_reversal():
    """With time-reversed pairs, M(B=0) vanishes and the moment along the field
    is the same for B and -B, each to rounding (H(-B) = Theta H(B) Theta^-1, and
    Theta maps the vector set onto itself); a single unpaired vector does not
    share either property."""
    rng = np.random.default_rng(8)
    sysm = W.random_small_system(rng, 4, max_two_s=3)
    T = W.t_grid(12)
    zero = of.sftlm(sysm, 4, 30, T, seed=2, fields=[[0.0, 0.0, 0.0]])[0]
    assert np.max(np.abs(zero["M"])) < 1e-10
    B = np.asarray(sysm.B, float)
    pm = [of.sftlm(sysm, 4, 30, T, seed=2, fields=[b])[0] for b in (B, -B)]  # same vectors
    assert np.max(np.abs(pm[0]["M"] - pm[1]["M"])) < 1e-9 * np.max(np.abs(pm[0]["M"]))
    assert np.max(np.abs(pm[0]["C"] - pm[1]["C"])) < 1e-9 * np.max(np.abs(pm[0]["C"]))
    plain = of.ftlm(sysm, 1, 30, T, seed=2, fields=[[0.0, 0.0, 0.0]])[0]
    assert np.max(np.abs(plain["M"])) > 1e-6


def test_dodecahedron_powder_grid():
    """The 10 directions (one per antipodal vertex pair of a regular
    dodecahedron, Sec. 3.3): the 20 vertices each have exactly 3 nearest
    neighbours at one distance (regular solid), and the directions average any
    quadratic form to its isotropic value tr(A)/3 (powder average exact for
    rank-2 responses)."""
    d = W.dodecahedron_directions()
    assert d.shape == (10, 3)
    v = np.concatenate([d, -d])
    dist = np.linalg.norm(v[:, None] - v[None], axis=2)
    np.fill_diagonal(dist, np.inf)
    dmin = dist.min()
    assert np.all(np.sum(np.abs(dist - dmin) < 1e-12, axis=1) == 3)
    rng = np.random.default_rng(0)
    A = rng.standard_normal((3, 3))
    A = A + A.T
    avg = np.mean([x @ A @ x for x in d])
    assert abs(avg - np.trace(A) / 3) < 1e-14


# ------------------------------------------------------- next row: Chebyshev (KPM)
from oracle import kpm as okpm  # noqa: E402


def test_chebyshev_expansion_coefficients():
    """sum_n c_n(x) T_n(t) = exp(-x (1 + t)) on [-1, 1] (generating function of
    the modified Bessel functions); pins the sign and the factor 2."""
    for x in (0.3, 4.0, 25.0):
        c = okpm.expansion_coefficients(x, 200)
        for t in (-1.0, -0.3, 0.2, 0.9, 1.0):
            tn = np.cos(np.arange(201) * np.arccos(t))
            assert abs(c @ tn - math.exp(-x * (1 + t))) < 1e-13 * max(1.0, math.exp(-x * (1 + t)))


def test_chebyshev_moments_match_spectral_definition():
    """mu_n = sum_k |<k|r>|^2 T_n((E_k - b)/a) from the dense eigenpairs."""
    rng = np.random.default_rng(40)
    sysm = W.random_small_system(rng, 4, max_two_s=2)
    H = dense.hamiltonian_dense(sysm)
    O = dense.moment_operator(sysm).toarray()
    ev, U = np.linalg.eigh(H)
    lo, hi = ev[0] - 0.1, ev[-1] + 0.1
    a, b = 0.5 * (hi - lo), 0.5 * (hi + lo)
    ham, mom = of.Ham(sysm), of.Moment(sysm, of.field_direction(sysm.B))
    r = of.gaussian_vector(9, 0, 0, 0, ham.dim)
    mu, nu = okpm.chebyshev_moments(ham, mom, r, a, b, 30)
    rh = r / np.linalg.norm(r)
    w = np.abs(U.conj().T @ rh) ** 2
    th = np.arccos((ev - b) / a)
    for n in range(33):
        assert abs(mu[n] - w @ np.cos(n * th)) < 1e-12
        Tn = (U * np.cos(n * th)) @ U.conj().T
        assert abs(nu[n] - np.vdot(O @ rh, Tn @ rh).real) < 1e-11


def test_kpm_per_vector_traces_are_exact():
    """With enough moments the expansion reproduces <r|exp(-H/T)|r>,
    <r|H exp(-H/T)|r>, <r|H^2 exp(-H/T)|r> and Re<r|O exp(-H/T)|r> from the
    dense matrices, i.e. ln Z, E, C and M of R = 1 to rounding."""
    rng = np.random.default_rng(41)
    sysm = W.random_small_system(rng, 4, max_two_s=2)
    H = dense.hamiltonian_dense(sysm)
    O = dense.moment_operator(sysm).toarray()
    dim = H.shape[0]
    T = np.array([1.5, 6.0, 40.0])
    res = okpm.kpm(sysm, 1, 400, T, seed=2, n_bound=dim + 5)[0]
    r = of.gaussian_vector(2, 0, 0, 0, dim)
    r = r / np.linalg.norm(r)
    ev, U = np.linalg.eigh(H)
    for k, t in enumerate(T):
        E = (U * np.exp(-(ev - ev[0]) / t)) @ U.conj().T
        z = np.vdot(r, E @ r).real
        e1 = np.vdot(r, H @ E @ r).real / z
        e2 = np.vdot(r, H @ H @ E @ r).real / z
        assert abs(res["lnZ"][k] - (np.log(dim * z) - ev[0] / t)) < 1e-10
        assert abs(res["E"][k] - e1) < 1e-9 * max(1, abs(e1))
        assert abs(res["C"][k] - (e2 - e1 * e1) / t ** 2) < 1e-8 * max(1, abs(e2 / t ** 2))
        assert abs(res["M"][k] - np.vdot(r, O @ E @ r).real / z) < 1e-9
