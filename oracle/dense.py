"""Dense reference Hamiltonian and exact thermodynamics (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The Hamiltonian is Sec. 2.1, Eq. (mce-hamop):

    H = 2 sum_{i<j} J_ij s_i.s_j + sum_i d_i (s_i.e_i)^2 + mu_B B.sum_i g_i s_i
        + mu0 mu_B^2/(4 pi) sum_{i<j} g_i g_j / r_ij^3
              (s_i.s_j - 3 (s_i.e_ij)(e_ij.s_j))

built here from Kronecker products of textbook spin matrices, a construction that
involves no basis-index arithmetic.  Basis: product basis of Sec. 2.1 with site 0
the fastest index, local state |m>, m = -s..s stored at digit d = m + s.

Readings (the paper is silent on them):
* energies in kelvin (k_B = 1); mu_B/k_B = 0.67171381563 K/T and
  mu0 mu_B^2/(4 pi k_B) = 6.2294807e-4 K nm^3 (CODATA 2018);
* the dipolar prefactor uses g_i g_j (the printed g^2 for uniform g);
* the observable for M is the moment along the field, O = -sum_i g_i s_i.B_hat
  (units of mu_B), positive for a paramagnet.

Pins: dimer, 4-ring, single-ion and dipolar-dimer closed forms; trace identities;
commutation relations of the spin matrices; Brillouin magnetisation
(``tests/test_oracle_pins.py``).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

MU_B_K_PER_T = 0.67171381563      # mu_B / k_B in K/T (CODATA 2018)
C_DIP_K_NM3 = 6.2294807e-4        # mu0 mu_B^2 / (4 pi k_B) in K nm^3 (CODATA 2018)


def spin_matrices(two_s: int):
    """Textbook spin matrices (sx, sy, sz, s+, s-) for spin s = two_s/2 in the basis
    |m>, m = -s, ..., s (ascending), Condon-Shortley phases."""
    s = two_s / 2.0
    n = two_s + 1
    m = -s + np.arange(n)
    sz = np.diag(m).astype(np.complex128)
    sp_ = np.zeros((n, n), np.complex128)
    for k in range(n - 1):
        # s+ |m> = sqrt(s(s+1) - m(m+1)) |m+1>
        sp_[k + 1, k] = np.sqrt(s * (s + 1) - m[k] * (m[k] + 1))
    sm = sp_.conj().T
    sx = 0.5 * (sp_ + sm)
    sy = (sp_ - sm) / 2j
    return sx, sy, sz, sp_, sm


def embed(op, site: int, dims) -> sp.csr_matrix:
    """Operator `op` acting on `site` of the product space; site 0 is the fastest
    index, so in Kronecker order the last site comes first."""
    out = sp.identity(1, dtype=np.complex128, format="csr")
    for k in reversed(range(len(dims))):
        f = sp.csr_matrix(op) if k == site else sp.identity(int(dims[k]), dtype=np.complex128,
                                                             format="csr")
        out = sp.kron(out, f, format="csr")
    return out


def _site_ops(system):
    dims = [int(t) + 1 for t in system.two_s]
    ops = []
    for i, t in enumerate(system.two_s):
        sx, sy, sz, _, _ = spin_matrices(int(t))
        ops.append([embed(sx, i, dims), embed(sy, i, dims), embed(sz, i, dims)])
    return dims, ops


def hamiltonian_sparse(system) -> sp.csr_matrix:
    """H of Eq. (mce-hamop) as a sparse matrix (built term by term)."""
    dims, ops = _site_ops(system)
    n = len(dims)
    dim = int(np.prod(dims))
    H = sp.csr_matrix((dim, dim), dtype=np.complex128)
    g = np.asarray(system.g, np.float64)
    # exchange 2 J_ij s_i.s_j
    if system.J is not None:
        for i in range(n):
            for j in range(i + 1, n):
                Jij = float(system.J[i][j])
                if Jij != 0.0:
                    H = H + 2.0 * Jij * sum(ops[i][a] @ ops[j][a] for a in range(3))
    # single-ion anisotropy d_i (s_i.e_i)^2
    if system.d is not None:
        for i in range(n):
            e = np.asarray(system.e[i], np.float64)
            e = e / np.linalg.norm(e)
            se = sum(e[a] * ops[i][a] for a in range(3))
            H = H + float(system.d[i]) * (se @ se)
    # Zeeman mu_B B . sum_i g_i s_i
    B = np.asarray(system.B, np.float64)
    for i in range(n):
        H = H + MU_B_K_PER_T * g[i] * sum(B[a] * ops[i][a] for a in range(3))
    # dipolar, all pairs
    if system.pos is not None:
        pos = np.asarray(system.pos, np.float64)
        for i in range(n):
            for j in range(i + 1, n):
                rvec = pos[j] - pos[i]
                r = np.linalg.norm(rvec)
                eij = rvec / r
                pref = C_DIP_K_NM3 * g[i] * g[j] / r ** 3
                sisj = sum(ops[i][a] @ ops[j][a] for a in range(3))
                sie = sum(eij[a] * ops[i][a] for a in range(3))
                sje = sum(eij[a] * ops[j][a] for a in range(3))
                H = H + pref * (sisj - 3.0 * (sie @ sje))
    return H.tocsr()


def hamiltonian_dense(system) -> np.ndarray:
    return hamiltonian_sparse(system).toarray()


def moment_operator(system, bhat=None) -> sp.csr_matrix:
    """O = -sum_i g_i s_i . B_hat (moment along the field, in mu_B)."""
    dims, ops = _site_ops(system)
    if bhat is None:
        B = np.asarray(system.B, np.float64)
        nb = np.linalg.norm(B)
        bhat = B / nb if nb > 0 else np.array([0.0, 0.0, 1.0])
    dim = int(np.prod(dims))
    O = sp.csr_matrix((dim, dim), dtype=np.complex128)
    for i in range(len(dims)):
        O = O - float(system.g[i]) * sum(bhat[a] * ops[i][a] for a in range(3))
    return O.tocsr()


def exact_thermo(system, T, bhat=None):
    """Exact ln Z, E, C, M on the temperature grid T by full diagonalisation.

    Z = sum_k exp(-E_k/T), E and C from centred moments of the Boltzmann weights,
    M = sum_k exp(-E_k/T) <k|O|k> / Z (a sum over degenerate subspaces is basis
    invariant)."""
    H = hamiltonian_dense(system)
    evals, U = np.linalg.eigh(H)
    O = moment_operator(system, bhat)
    diagO = np.real(np.einsum("ik,ik->k", U.conj(), O @ U))
    return thermo_from_spectrum(evals, diagO, T)


def thermo_from_spectrum(evals, diagO, T):
    T = np.asarray(T, np.float64)
    e0 = evals.min()
    lnz, E, C, M = [], [], [], []
    for t in T:
        w = np.exp(-(evals - e0) / t)
        z = w.sum()
        p = w / z
        em = (p * evals).sum()
        lnz.append(np.log(z) - e0 / t)
        E.append(em)
        C.append((p * (evals - em) ** 2).sum() / t ** 2)
        M.append((p * diagO).sum() if diagO is not None else np.nan)
    return dict(lnZ=np.array(lnz), E=np.array(E), C=np.array(C), M=np.array(M),
                E0=float(e0))
