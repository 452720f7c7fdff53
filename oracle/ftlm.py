"""FTLM oracle driver (CPU, FP64).  TEST INFRASTRUCTURE ONLY.

Follows Sec. 2.2 step by step:

1. random vectors |r> with complex Gaussian components (Eqs. E-1-1, E-1-2),
   keyed by (seed; r, field, instance) through the C library's Philox4x32-10;
2. N_L Lanczos steps from |r>/||r|| (C library, Paige order), recording the
   tridiagonal (alpha, beta) and the overlaps y_a = <O v_1|v_a>;
3. Krylov eigenpairs eps_n^(r), <n(r)|r> from the tridiagonal
   (``scipy.linalg.eigh_tridiagonal``, a library step);
4. Boltzmann sums: Z from Eq. (E-2-D) with one sector (Gamma = 1),
   E and C from the same weights with the centred second moment, and M from the
   ratio estimator Eq. (E-2-C) with O = -sum_i g_i s_i.B_hat:

     Z   = dim/R sum_{r,n} exp(-eps_n/T) Q_1n^2
     <A> = sum_{r,n} exp(-eps_n/T) Q_1n^2 A(eps_n) / sum_{r,n} exp(-eps_n/T) Q_1n^2
     M   = sum_{r,n} exp(-eps_n/T) Q_1n Re(sum_a Q_an y_a)
           / sum_{r,n} exp(-eps_n/T) Q_1n^2

   with E_min = min_r eps_1^(r) factored out of every exponential.

Readings: N_L fixed by the run; a Lanczos breakdown (beta_j <= 1e-12 max(|alpha|,
beta)) truncates the Krylov space; C = (<eps^2> - <eps>^2)/T^2 from Ritz values.

Parity status: pinned statistically against exact diagonalisation, exactly in
the invariant-subspace case (dim <= N_L with re-orthogonalisation), and by the
Schottky and Brillouin closed forms.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import scipy.linalg

from . import build as _build

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build(force=True)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_build.restype = ctypes.c_void_p
        L.oracle_build.argtypes = [ctypes.c_int, ip, dp, dp, dp, dp, dp, dp]
        L.oracle_build_moment.restype = ctypes.c_void_p
        L.oracle_build_moment.argtypes = [ctypes.c_int, ip, dp, dp]
        L.oracle_free.argtypes = [ctypes.c_void_p]
        L.oracle_dim.restype = ctypes.c_int64
        L.oracle_dim.argtypes = [ctypes.c_void_p]
        L.oracle_npairs.restype = ctypes.c_int
        L.oracle_npairs.argtypes = [ctypes.c_void_p]
        L.oracle_hv.argtypes = [ctypes.c_void_p, dp, dp]
        L.oracle_hv_rows.argtypes = [ctypes.c_void_p, dp, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.c_int64, dp]
        L.oracle_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.oracle_gaussian_vector.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_uint32, ctypes.c_int64, dp]
        L.oracle_gaussian_entries.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                              ctypes.c_uint32, ctypes.POINTER(ctypes.c_int64),
                                              ctypes.c_int64, dp]
        L.oracle_lanczos.restype = ctypes.c_int
        L.oracle_lanczos.argtypes = [ctypes.c_void_p, ctypes.c_void_p, dp, ctypes.c_int,
                                     ctypes.c_int, dp, dp, dp, ip]
        L.oracle_spin_matrices.argtypes = [ctypes.c_int, dp, dp, dp]
        _LIB = L
    return _LIB


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64(a, shape=None):
    if a is None:
        return None
    out = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        out = out.reshape(shape)
    return out


class Ham:
    """The C oracle's Hamiltonian (one-site and two-site matrices)."""

    def __init__(self, system, B=None):
        n = system.n_sites
        self._keep = []
        two_s = np.ascontiguousarray(np.asarray(system.two_s, np.int32))
        J = _f64(system.J, (n, n)) if system.J is not None else None
        d = _f64(system.d) if system.d is not None else None
        e = _f64(system.e, (n, 3))
        g = _f64(system.g)
        Bv = _f64(system.B if B is None else B, (3,))
        pos = _f64(system.pos, (n, 3)) if system.pos is not None else None
        self._keep = [two_s, J, d, e, g, Bv, pos]
        self.ptr = lib().oracle_build(n, two_s.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                      _dp(J), _dp(d), _dp(e), _dp(g), _dp(Bv), _dp(pos))
        if not self.ptr:
            raise ValueError("oracle_build failed")
        self.dim = int(lib().oracle_dim(self.ptr))

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().oracle_free(self.ptr)
            self.ptr = None

    def apply(self, v):
        v = np.ascontiguousarray(np.asarray(v, np.complex128))
        assert v.shape == (self.dim,)
        w = np.empty_like(v)
        lib().oracle_hv(self.ptr, _dp(v.view(np.float64)), _dp(w.view(np.float64)))
        return w

    def apply_rows(self, v, rows):
        """(H v)[rows] without forming the whole product."""
        v = np.ascontiguousarray(np.asarray(v, np.complex128))
        assert v.shape == (self.dim,)
        rows = np.ascontiguousarray(np.asarray(rows, np.int64))
        out = np.empty(len(rows), np.complex128)
        lib().oracle_hv_rows(self.ptr, _dp(v.view(np.float64)),
                             rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(rows),
                             _dp(out.view(np.float64)))
        return out


class Moment:
    """O = -sum_i g_i s_i . bhat."""

    def __init__(self, system, bhat):
        two_s = np.ascontiguousarray(np.asarray(system.two_s, np.int32))
        g = _f64(system.g)
        b = _f64(bhat, (3,))
        self._keep = [two_s, g, b]
        self.ptr = lib().oracle_build_moment(system.n_sites,
                                             two_s.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                             _dp(g), _dp(b))
        self.dim = int(lib().oracle_dim(self.ptr))

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().oracle_free(self.ptr)
            self.ptr = None

    def apply(self, v):
        v = np.ascontiguousarray(np.asarray(v, np.complex128))
        w = np.empty_like(v)
        lib().oracle_hv(self.ptr, _dp(v.view(np.float64)), _dp(w.view(np.float64)))
        return w


def spin_matrices(two_s):
    n = two_s + 1
    mats = [np.zeros((n, n), np.complex128) for _ in range(3)]
    lib().oracle_spin_matrices(two_s, *[_dp(m.view(np.float64)) for m in mats])
    return mats


def hv(system, v, B=None):
    return Ham(system, B).apply(v)


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def gaussian_vector(seed, r, field, instance, dim):
    out = np.empty(int(dim), np.complex128)
    lib().oracle_gaussian_vector(ctypes.c_uint64(int(seed)), r, field, instance, int(dim),
                                 _dp(out.view(np.float64)))
    return out


def gaussian_entries(seed, r, field, instance, idx):
    """Components idx of :func:`gaussian_vector` (any dimension above them),
    without forming the vector."""
    idx = np.ascontiguousarray(np.asarray(idx, np.int64))
    assert idx.size == 0 or (idx.min() >= 0 and idx.max() < (1 << 32))
    out = np.empty(len(idx), np.complex128)
    lib().oracle_gaussian_entries(ctypes.c_uint64(int(seed)), r, field, instance,
                                  idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(idx),
                                  _dp(out.view(np.float64)))
    return out


def field_direction(B):
    B = np.asarray(B, np.float64)
    nb = np.linalg.norm(B)
    return B / nb if nb > 0 else np.array([0.0, 0.0, 1.0])


def lanczos(ham, moment, r, n_lanczos, reorth=False):
    """Returns (alpha, beta, y, n_used) for start vector r."""
    r = np.ascontiguousarray(np.asarray(r, np.complex128))
    alpha = np.zeros(n_lanczos)
    beta = np.zeros(n_lanczos)
    y = np.zeros(n_lanczos, np.complex128)
    nu = ctypes.c_int(0)
    rc = lib().oracle_lanczos(ham.ptr, moment.ptr if moment is not None else None,
                              _dp(r.view(np.float64)), n_lanczos, 1 if reorth else 0,
                              _dp(alpha), _dp(beta), _dp(y.view(np.float64)), ctypes.byref(nu))
    if rc != 0:
        raise MemoryError("oracle_lanczos failed (%d)" % rc)
    k = nu.value
    return alpha[:k], beta[:k], y[:k], k


def krylov_eigen(alpha, beta, y=None):
    """Eigenpairs of the Lanczos tridiagonal: eps_n, Q_1n = <n|v_1>, and
    (Q^T y)_n = sum_a Q_an y_a."""
    k = len(alpha)
    if k == 1:
        eps = np.array([alpha[0]])
        Q = np.ones((1, 1))
    else:
        eps, Q = scipy.linalg.eigh_tridiagonal(alpha, beta[:k - 1])
    q1 = Q[0, :]
    u = Q.T @ y if y is not None else None
    return eps, q1, u


def boltzmann(dim, eps_list, q1_list, u_list, T):
    """Boltzmann sums of Eqs. (E-2-C) and (E-2-D) over all random vectors of one
    field.  Returns lnZ, E, C, M on the grid T and E_min."""
    R = len(eps_list)
    T = np.asarray(T, np.float64)
    eps = np.concatenate(eps_list)
    w1 = np.concatenate(q1_list) ** 2
    qu = np.concatenate([q * np.real(u) for q, u in zip(q1_list, u_list)]) if u_list else None
    emin = min(float(e.min()) for e in eps_list)
    lnZ, E, C, M = [], [], [], []
    for t in T:
        boltz = np.exp(-(eps - emin) / t)
        zr = np.sum(boltz * w1)
        lnZ.append(np.log(dim / R) - emin / t + np.log(zr))
        em = np.sum(boltz * w1 * eps) / zr
        E.append(em)
        C.append(np.sum(boltz * w1 * (eps - em) ** 2) / zr / t ** 2)
        M.append(np.sum(boltz * qu) / zr if qu is not None else np.nan)
    return dict(lnZ=np.array(lnZ), E=np.array(E), C=np.array(C), M=np.array(M), E_min=emin)


def ftlm(system, R, n_lanczos, T, seed=0, fields=None, instance=0, start_vectors=None,
         reorth=False, return_columns=False):
    """FTLM curves for each field (rows of `fields`, default the system's B).

    start_vectors: optional [n_fields][R][dim] complex array overriding the
    seeded Gaussian vectors."""
    if fields is None:
        fields = np.asarray(system.B, np.float64)[None, :]
    fields = np.asarray(fields, np.float64).reshape(-1, 3)
    out = []
    for f, B in enumerate(fields):
        ham = Ham(system, B)
        mom = Moment(system, field_direction(B))
        eps_l, q1_l, u_l, nused, cols = [], [], [], [], []
        for r in range(R):
            if start_vectors is not None:
                rv = np.asarray(start_vectors[f][r], np.complex128)
            else:
                rv = gaussian_vector(seed, r, f, instance, ham.dim)
            a, b, y, k = lanczos(ham, mom, rv, n_lanczos, reorth)
            eps, q1, u = krylov_eigen(a, b, y)
            eps_l.append(eps)
            q1_l.append(q1)
            u_l.append(u)
            nused.append(k)
            if return_columns:
                cols.append(dict(alpha=a, beta=b, y=y))
        res = boltzmann(ham.dim, eps_l, q1_l, u_l, T)
        res["n_lanczos_used"] = np.array(nused)
        if return_columns:
            res["columns"] = cols
            res["eps"] = eps_l
            res["q1"] = q1_l
        out.append(res)
    return out


# ---------------------------------------------------------------------------
# Symmetric FTLM with time-reversed pairs of random vectors (Sec. 2.2,
# Eqs. (E-2-G), (E-2-H); pairs of mutually time-reversed vectors as proposed in
# the same section).  TEST INFRASTRUCTURE ONLY.
#
# Readings: R counts vectors, so R/2 Gaussian vectors are drawn (Philox stream
# index = pair index p) and each is used together with its time reverse.  The
# time reversal of the product basis with Condon-Shortley phases is
#     (Theta x)[nu'] = (-1)^{sum_i (2 s_i - d_i(nu))} conj(x[nu]),
# nu' the state with every m_i -> -m_i (digits d_i -> 2 s_i - d_i, i.e.
# nu' = dim - 1 - nu).  The Krylov eigenvectors |n(r)> = sum_a Q_an |v_a> are
# built from the stored Lanczos vectors, and <m|O|n> = (Q^T V^H O V Q)_mn.
# ---------------------------------------------------------------------------


def digit_sums(two_s):
    """sum_i d_i(nu) for every basis index nu (site 0 fastest)."""
    two_s = np.asarray(two_s, np.int64)
    dim = int(np.prod(two_s + 1))
    nu = np.arange(dim, dtype=np.int64)
    tot = np.zeros(dim, np.int64)
    for ts in two_s:
        tot += nu % (ts + 1)
        nu //= ts + 1
    return tot


def time_reverse(two_s, x):
    """Theta x in the product basis (see the module notes above)."""
    x = np.asarray(x, np.complex128)
    two_s = np.asarray(two_s, np.int64)
    phase = np.where((int(two_s.sum()) - digit_sums(two_s)) % 2 == 0, 1.0, -1.0)
    return (phase * np.conj(x))[::-1].copy()


def lanczos_basis(ham, r, n_lanczos, reorth=False):
    """Paige-order Lanczos from r/|r| keeping the basis: returns alpha, beta, V
    ([k][dim], rows v_1..v_k) with the breakdown rule of the FTLM driver."""
    v = np.asarray(r, np.complex128) / np.linalg.norm(r)
    V = [v]
    alpha, beta = [], []
    v_prev = np.zeros_like(v)
    b_prev = 0.0
    scale = 0.0
    for j in range(n_lanczos):
        u = ham.apply(V[-1]) - b_prev * v_prev
        a = float(np.real(np.vdot(V[-1], u)))
        u = u - a * V[-1]
        if reorth:
            for q in V:
                u = u - np.vdot(q, u) * q
        b = float(np.linalg.norm(u))
        alpha.append(a)
        scale = max(scale, abs(a))
        if j + 1 == n_lanczos:
            beta.append(b)
            break
        if not b > 1e-12 * scale:
            beta.append(b)
            break
        scale = max(scale, b)
        beta.append(b)
        v_prev = V[-1]
        b_prev = b
        V.append(u / b)
    k = len(alpha)
    return np.array(alpha), np.array(beta), np.array(V[:k])


def sftlm(system, R, n_lanczos, T, seed=0, fields=None, instance=0, reorth=False):
    """sFTLM curves (Eq. E-2-G for M with O = -sum_i g_i s_i.B_hat; Eq. E-2-D
    for Z; E and C from the Ritz values as in the plain driver) for each field,
    with R/2 time-reversed pairs of random vectors."""
    if R % 2:
        raise ValueError("R must be even (time-reversed pairs)")
    if fields is None:
        fields = np.asarray(system.B, np.float64)[None, :]
    fields = np.asarray(fields, np.float64).reshape(-1, 3)
    T = np.asarray(T, np.float64)
    out = []
    for f, B in enumerate(fields):
        ham = Ham(system, B)
        mom = Moment(system, field_direction(B))
        cols = []
        for p in range(R // 2):
            r0 = gaussian_vector(seed, p, f, instance, ham.dim)
            for rv in (r0, time_reverse(system.two_s, r0)):
                a, b, V = lanczos_basis(ham, rv, n_lanczos, reorth)
                k = len(a)
                if k == 1:
                    eps, Q = np.array([a[0]]), np.ones((1, 1))
                else:
                    eps, Q = scipy.linalg.eigh_tridiagonal(a, b[:k - 1])
                OV = np.array([mom.apply(x) for x in V])
                OK = np.conj(V) @ OV.T          # <v_a|O|v_b>
                cols.append((eps, Q, OK))
        emin = min(float(c[0].min()) for c in cols)
        lnZ, E, C, M = [], [], [], []
        eps_all = np.concatenate([c[0] for c in cols])
        w1_all = np.concatenate([c[1][0, :] ** 2 for c in cols])
        for t in T:
            boltz = np.exp(-(eps_all - emin) / t) * w1_all
            den = boltz.sum()
            em = np.sum(boltz * eps_all) / den
            num = 0.0
            for eps, Q, OK in cols:
                h = np.exp(-(eps - emin) / (2 * t)) * Q[0, :]   # e^{-beta(eps-Emin)/2} <n|r>
                z = Q @ h                                        # sum_n Q_an h_n
                num += float(np.real(z @ OK @ z))
            lnZ.append(np.log(ham.dim / R) - emin / t + np.log(den))
            E.append(em)
            C.append(np.sum(boltz * (eps_all - em) ** 2) / den / t ** 2)
            M.append(num / den)
        out.append(dict(lnZ=np.array(lnZ), E=np.array(E), C=np.array(C), M=np.array(M),
                        E_min=emin, n_lanczos_used=np.array([len(c[0]) for c in cols])))
    return out
