"""Chebyshev (kernel polynomial) trace expansion of the FTLM thermal traces,
without a smoothing kernel (the alternative named in Sec. 4).  TEST
INFRASTRUCTURE ONLY.

Plain CPU FP64 steps:

1. spectral bounds: N_B Lanczos steps (the oracle's Paige-order recursion,
   ``ftlm.lanczos``) from the first random vector; [lo, hi] = [min, max] of the
   Ritz values widened by 2 % of their spread (reading: the margin);
   a = (hi - lo)/2, b = (hi + lo)/2, H~ = (H - b)/a;
2. per random vector r (the Gaussian vectors of the FTLM driver, normalised):
   t_0 = r, t_1 = H~ t_0, t_{n+1} = 2 H~ t_n - t_{n-1}; moments
   mu_n = Re <r|t_n>, nu_n = Re <O r|t_n>, n = 0..N+2;
3. exp(-H/T) = exp(-lo/T) sum_n c_n(a/T) T_n(H~) with
   c_n(x) = (2 - delta_n0) (-1)^n exp(-x) I_n(x)   (Chebyshev expansion of
   exp(-x t), a library Bessel function ``scipy.special.ive``), truncated at n = N;
4. <r|H T_n|r> and <r|H^2 T_n|r> from H = a H~ + b and the product rule
   2 T_1 T_n = T_{n+1} + T_{|n-1|};
5. Z = dim/R exp(-lo/T) sum_r sum_n c_n mu_n^r; E = <H>, C = (<H^2> - <H>^2)/T^2,
   M = sum_r sum_n c_n nu_n^r / sum_r sum_n c_n mu_n^r.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.special

from . import ftlm as of

MARGIN = 0.02


def spectral_bounds(ham, r, n_steps):
    a, b, _, k = of.lanczos(ham, None, r, n_steps)
    eps = np.array([a[0]]) if k == 1 else scipy.linalg.eigh_tridiagonal(a, b[:k - 1], eigvals_only=True)
    lo, hi = float(eps.min()), float(eps.max())
    pad = MARGIN * (hi - lo) + 1e-12 * max(1.0, abs(lo), abs(hi))
    return lo - pad, hi + pad


def chebyshev_moments(ham, mom, r, a, b, n_moments):
    """mu_n, nu_n for n = 0..n_moments+2 (r normalised inside)."""
    t0 = np.asarray(r, np.complex128) / np.linalg.norm(r)
    ov = mom.apply(t0)
    m = n_moments + 3
    mu = np.zeros(m)
    nu = np.zeros(m)
    mu[0], nu[0] = np.vdot(t0, t0).real, np.vdot(ov, t0).real
    t_prev, t = t0, (ham.apply(t0) - b * t0) / a
    mu[1], nu[1] = np.vdot(t0, t).real, np.vdot(ov, t).real
    for n in range(1, m - 1):
        t_next = 2.0 * (ham.apply(t) - b * t) / a - t_prev
        t_prev, t = t, t_next
        mu[n + 1], nu[n + 1] = np.vdot(t0, t).real, np.vdot(ov, t).real
    return mu, nu


def expansion_coefficients(x, n_moments):
    n = np.arange(n_moments + 1)
    c = scipy.special.ive(n, x) * np.where(n % 2 == 0, 1.0, -1.0)
    c[1:] *= 2.0
    return c


def kpm(system, R, n_moments, T, seed=0, fields=None, instance=0, n_bound=40):
    if fields is None:
        fields = np.asarray(system.B, np.float64)[None, :]
    fields = np.asarray(fields, np.float64).reshape(-1, 3)
    T = np.asarray(T, np.float64)
    out = []
    N = n_moments
    for f, B in enumerate(fields):
        ham = of.Ham(system, B)
        mom = of.Moment(system, of.field_direction(B))
        lo, hi = spectral_bounds(ham, of.gaussian_vector(seed, 0, f, instance, ham.dim), n_bound)
        a, b = 0.5 * (hi - lo), 0.5 * (hi + lo)
        mus, nus = [], []
        for r in range(R):
            mu, nu = chebyshev_moments(ham, mom, of.gaussian_vector(seed, r, f, instance, ham.dim), a, b, N)
            mus.append(mu)
            nus.append(nu)
        mu = np.sum(mus, axis=0)
        nu = np.sum(nus, axis=0)
        n = np.arange(N + 1)
        h1 = a * 0.5 * (mu[n + 1] + mu[np.abs(n - 1)]) + b * mu[n]
        h2 = (a * a * 0.25 * (mu[n + 2] + 2 * mu[n] + mu[np.abs(n - 2)])
              + a * b * (mu[n + 1] + mu[np.abs(n - 1)]) + b * b * mu[n])
        lnZ, E, C, M = [], [], [], []
        for t in T:
            c = expansion_coefficients(a / t, N)
            z = c @ mu[:N + 1]
            e1 = (c @ h1) / z
            e2 = (c @ h2) / z
            lnZ.append(np.log(ham.dim / R) - lo / t + np.log(z))
            E.append(e1)
            C.append((e2 - e1 * e1) / t ** 2)
            M.append((c @ nu[:N + 1]) / z)
        out.append(dict(lnZ=np.array(lnZ), E=np.array(E), C=np.array(C), M=np.array(M),
                        E_lo=lo, E_hi=hi, mu=mu, nu=nu))
    return out
