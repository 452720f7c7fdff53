"""Seeded synthetic workloads for the finite-temperature Lanczos method (FTLM).

This module only draws model parameters (couplings, anisotropy axes, g-factors,
fields, positions, temperature grids, run sizes) from seeded generators.  It holds
none of the method's arithmetic: no spin operators, no Hamiltonian, no Lanczos.
Both the CPU oracle (``oracle/``) and the HIP path (``paper_2607_25585_amd``)
consume the same :class:`System` / :class:`RunSpec` objects, so the two sides
see identical inputs while sharing no code of the method.

Model: the spin Hamiltonian of Sec. 2.1 (Heisenberg exchange, single-ion
anisotropy, Zeeman term, all-to-all dipolar coupling).  Units: J, d in kelvin,
B in tesla, positions in nm, g dimensionless; energies in kelvin (k_B = 1).

Workload recipes (all seeded with ``numpy.random.default_rng(1000*K)`` for
workload K):

* ``cfg1``  N=8, s=1 ring, J=1 K nearest neighbour, d=-2 K along seeded random
  unit axes, g=2, B=1 T along z, no dipolar; R=20, N_L=100.  Exact-diagonalisation
  size (dim 6561).
* ``cfg2``  N=24, s=1/2 ring, J=1 K, positions 1 nm x seeded unit vectors, all
  276 dipolar pairs, g=2, B=0.5 T along a seeded unit vector; R=10, N_L=150.
* ``cfg2_hb`` cfg2 without dipolar, B along z (Heisenberg ring in a field).
* ``cfg3``  64 instances, N ~ U{14..22} s=1/2, J ~ U(-2,2) K per instance on the
  nn ring, positions on a 1 nm sphere, all-pairs dipolar, g=2, 50 seeded field
  directions x 1 T, R=16, N_L=120.
* ``cfg4``  N=12, s=2 on a 0.8 nm ring in the xy-plane, J_nn=0.5 K, J_nnn=0.1 K,
  d=-1 K with axes tilted 30 deg from z at seeded azimuths, 66 dipolar pairs,
  g=2, B=2 T along z; R=8, N_L=200 (dim 244,140,625).
* ``cfg4_hb`` cfg4 with nn+nnn Heisenberg only, B along z.
* ``cfg5``  surrogate data: N=8, s=3/2 ring, J ~ U(-3,3) K, d ~ U(-5,5) K,
  tilt ~ U(0,90 deg) with radial azimuths phi_i = 2 pi i/8, |B| ~ U(0,7) T,
  field direction uniform on the sphere; R=20, N_L=100.

Temperature grid: 200 points, T_k = 10**(-1 + 3k/199) K, k = 0..199.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "System", "RunSpec", "t_grid", "ring_couplings", "unit_vectors",
    "cfg1", "cfg2", "cfg2_hb", "cfg3", "cfg4", "cfg4_hb", "cfg5_params",
    "cfg5_system", "random_small_system", "dimension", "ring6", "mn9",
    "dodecahedron_directions", "WORKLOADS",
]


@dataclasses.dataclass
class System:
    """Parameters of one spin system (inputs to the Hamiltonian of Sec. 2.1).

    two_s : [N] int, 2*s_i >= 1
    J     : [N,N] float, J[i,j] read for i<j (exchange, kelvin); may be None
    d     : [N] single-ion anisotropy strengths (kelvin); may be None
    e     : [N,3] anisotropy axes (normalised by the consumers)
    g     : [N] g-factors
    B     : [3] field (tesla)
    pos   : [N,3] positions (nm) or None (no dipolar term)
    """
    two_s: np.ndarray
    J: Optional[np.ndarray]
    d: Optional[np.ndarray]
    e: np.ndarray
    g: np.ndarray
    B: np.ndarray
    pos: Optional[np.ndarray]
    name: str = ""

    @property
    def n_sites(self) -> int:
        return int(len(self.two_s))

    def with_field(self, B) -> "System":
        return dataclasses.replace(self, B=np.asarray(B, dtype=np.float64).copy())


@dataclasses.dataclass
class RunSpec:
    """Sizes of an FTLM run: R random vectors per field, N_L Lanczos steps."""
    R: int
    n_lanczos: int
    seed: int
    T: np.ndarray
    fields: Optional[np.ndarray] = None  # [n_fields,3]; None -> the system's B


def dimension(two_s) -> int:
    """Product of the local dimensions 2 s_i + 1 (Sec. 2.1)."""
    dim = 1
    for t in two_s:
        dim *= int(t) + 1
    return dim


def t_grid(n: int = 200, lo: float = 0.1, hi: float = 100.0) -> np.ndarray:
    """Log-spaced temperature grid with inclusive ends (kelvin)."""
    k = np.arange(n, dtype=np.float64)
    return lo * (hi / lo) ** (k / (n - 1))


def unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    """n seeded unit vectors, uniform on the sphere (normalised Gaussians)."""
    x = rng.standard_normal((n, 3))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def ring_couplings(n: int, j1: float, j2: float = 0.0) -> np.ndarray:
    """Exchange matrix of a ring: j1 between i,i+1 and j2 between i,i+2 (mod n)."""
    J = np.zeros((n, n))
    for i in range(n):
        for off, val in ((1, j1), (2, j2)):
            if val == 0.0:
                continue
            j = (i + off) % n
            a, b = min(i, j), max(i, j)
            J[a, b] += val
    return J


def cfg1() -> tuple[System, RunSpec]:
    rng = np.random.default_rng(1000)
    n = 8
    sysm = System(two_s=np.full(n, 2, np.int32), J=ring_couplings(n, 1.0),
                  d=np.full(n, -2.0), e=unit_vectors(rng, n), g=np.full(n, 2.0),
                  B=np.array([0.0, 0.0, 1.0]), pos=None, name="cfg1")
    return sysm, RunSpec(R=20, n_lanczos=100, seed=1000, T=t_grid())


def _cfg2_base(rng):
    n = 24
    pos = 1.0 * unit_vectors(rng, n)
    bdir = unit_vectors(rng, 1)[0]
    return n, pos, bdir


def cfg2() -> tuple[System, RunSpec]:
    rng = np.random.default_rng(2000)
    n, pos, bdir = _cfg2_base(rng)
    sysm = System(two_s=np.ones(n, np.int32), J=ring_couplings(n, 1.0),
                  d=None, e=np.tile([0.0, 0.0, 1.0], (n, 1)), g=np.full(n, 2.0),
                  B=0.5 * bdir, pos=pos, name="cfg2")
    return sysm, RunSpec(R=10, n_lanczos=150, seed=2000, T=t_grid())


def cfg2_hb() -> tuple[System, RunSpec]:
    s, r = cfg2()
    s = dataclasses.replace(s, pos=None, B=np.array([0.0, 0.0, 0.5]), name="cfg2_hb")
    return s, r


def cfg3(n_instances: int = 64, n_dirs: int = 50) -> tuple[List[System], RunSpec, np.ndarray]:
    """Batched workload: returns (instances, run spec, field directions [n_inst,n_dirs,3])."""
    rng = np.random.default_rng(3000)
    systems = []
    fields = np.zeros((n_instances, n_dirs, 3))
    for k in range(n_instances):
        n = int(rng.integers(14, 23))
        jv = float(rng.uniform(-2.0, 2.0))
        pos = 1.0 * unit_vectors(rng, n)
        dirs = unit_vectors(rng, n_dirs)
        fields[k] = 1.0 * dirs
        systems.append(System(two_s=np.ones(n, np.int32), J=ring_couplings(n, jv), d=None,
                              e=np.tile([0.0, 0.0, 1.0], (n, 1)), g=np.full(n, 2.0),
                              B=fields[k, 0].copy(), pos=pos, name=f"cfg3[{k}]"))
    return systems, RunSpec(R=16, n_lanczos=120, seed=3000, T=t_grid()), fields


def _tilted_axes(phi, tilt_rad):
    st, ct = math.sin(tilt_rad), math.cos(tilt_rad)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.full_like(phi, ct)], axis=1)


def cfg4() -> tuple[System, RunSpec]:
    rng = np.random.default_rng(4000)
    n = 12
    ang = 2 * np.pi * np.arange(n) / n
    pos = 0.8 * np.stack([np.cos(ang), np.sin(ang), np.zeros(n)], axis=1)
    phi = rng.uniform(0, 2 * np.pi, n)
    sysm = System(two_s=np.full(n, 4, np.int32), J=ring_couplings(n, 0.5, 0.1),
                  d=np.full(n, -1.0), e=_tilted_axes(phi, math.radians(30.0)),
                  g=np.full(n, 2.0), B=np.array([0.0, 0.0, 2.0]), pos=pos, name="cfg4")
    return sysm, RunSpec(R=8, n_lanczos=200, seed=4000, T=t_grid())


def cfg4_hb() -> tuple[System, RunSpec]:
    s, r = cfg4()
    s = dataclasses.replace(s, d=None, pos=None, name="cfg4_hb")
    return s, r


def cfg5_params(n_sets: int, seed: int = 5000) -> np.ndarray:
    """Parameter draws for the surrogate data set: columns
    (J, d, tilt[rad], |B|, theta_B, phi_B)."""
    rng = np.random.default_rng(seed)
    J = rng.uniform(-3.0, 3.0, n_sets)
    d = rng.uniform(-5.0, 5.0, n_sets)
    tilt = rng.uniform(0.0, 0.5 * np.pi, n_sets)
    bmag = rng.uniform(0.0, 7.0, n_sets)
    u = unit_vectors(rng, n_sets)
    theta = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
    phi = np.mod(np.arctan2(u[:, 1], u[:, 0]), 2 * np.pi)
    return np.stack([J, d, tilt, bmag, theta, phi], axis=1)


def cfg5_system(p) -> System:
    """The N=8, s=3/2 ring for one parameter row of :func:`cfg5_params`."""
    J, d, tilt, bmag, theta, phi = [float(x) for x in p]
    n = 8
    phis = 2 * np.pi * np.arange(n) / n
    bdir = np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi),
                     math.cos(theta)])
    return System(two_s=np.full(n, 3, np.int32), J=ring_couplings(n, J),
                  d=np.full(n, d), e=_tilted_axes(phis, tilt), g=np.full(n, 2.0),
                  B=bmag * bdir, pos=None, name="cfg5")


def cfg5_runspec() -> RunSpec:
    return RunSpec(R=20, n_lanczos=100, seed=5000, T=t_grid())


def random_small_system(rng: np.random.Generator, n_sites: int, max_two_s: int = 4,
                        dipolar: bool = True, name: str = "random") -> System:
    """A random mixed-spin system with every term switched on and non-zero y
    components in axes, field and positions (for elementwise parity)."""
    two_s = rng.integers(1, max_two_s + 1, n_sites).astype(np.int32)
    J = np.triu(rng.uniform(-1.5, 1.5, (n_sites, n_sites)), 1)
    d = rng.uniform(-3.0, 3.0, n_sites)
    e = unit_vectors(rng, n_sites)
    g = rng.uniform(1.8, 2.2, n_sites)
    B = rng.uniform(-2.0, 2.0, 3)
    pos = 0.5 * rng.standard_normal((n_sites, 3)) if dipolar else None
    if pos is not None:
        # keep sites apart so that the dipolar strengths stay moderate
        pos = pos + 0.6 * np.arange(n_sites)[:, None] * np.array([1.0, 0.3, -0.2])
    return System(two_s=two_s, J=J, d=d, e=e, g=g, B=B, pos=pos, name=name)


def ring6(B: float = 0.1) -> tuple[System, RunSpec]:
    """Anisotropic ring of Sec. 3.2: N=6, s=5/2, nearest-neighbour J=0.02 K,
    d=-20 K, all-to-all dipolar, B along z (0.1 T or 1 T in the paper).  Readings:
    ring radius 0.5 nm in the xy-plane; non-collinear easy axes tilted 30 deg from
    z towards the radial directions (phi_i = 2 pi i/6); g = 2.  sFTLM with
    time-reversed pairs (R counts vectors)."""
    return ring_sftlm(6, B)


def ring_sftlm(n: int, B: float = 0.1) -> tuple[System, RunSpec]:
    """The ring of Sec. 3.2 with n sites (n = 6 is the paper's; n = 5, dim
    7776, is small enough for a dense exact spectrum), same readings."""
    ang = 2 * np.pi * np.arange(n) / n
    pos = 0.5 * np.stack([np.cos(ang), np.sin(ang), np.zeros(n)], axis=1)
    sysm = System(two_s=np.full(n, 5, np.int32), J=ring_couplings(n, 0.02), d=np.full(n, -20.0),
                  e=_tilted_axes(ang, math.radians(30.0)), g=np.full(n, 2.0),
                  B=np.array([0.0, 0.0, float(B)]), pos=pos, name="ring%d" % n)
    return sysm, RunSpec(R=20, n_lanczos=100, seed=6000, T=t_grid())


def dodecahedron_directions() -> np.ndarray:
    """The 10 directions of the 20 vertices of a regular dodecahedron (one of each
    antipodal pair), unit vectors: the powder-average grid of Sec. 3.3."""
    ph = (1 + math.sqrt(5)) / 2
    verts = [(x, y, z) for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)]
    for a in (-1, 1):
        for b in (-1, 1):
            verts += [(0, a / ph, b * ph), (a / ph, b * ph, 0), (a * ph, 0, b / ph)]
    v = np.asarray(verts, np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    keep = []
    for x in v:
        if not any(np.allclose(x, -y) for y in keep):
            keep.append(x)
    return np.asarray(keep)


def mn9(B: float = 1.0) -> tuple[System, RunSpec]:
    """Mn9-like centred cube of Sec. 3.3: site 0 = centre s=5/2, sites 1..8 =
    cube vertices s=2 (dimension 6 * 5^8 = 2,343,750).  Exchange J_c (centre to
    vertices), J_s (edges of the top and bottom squares), J_e (vertical edges);
    easy axis D on the vertices tilted 30 deg from z at azimuth +-10 deg from x
    (alternating).  The paper does not print J_c, J_s, J_e, D: the values here
    (J_c = 1.0, J_s = 0.5, J_e = 0.3, D = -2 K) are synthetic readings; no
    dipolar term; g = 2; fields: |B| times the 10 dodecahedron directions
    (powder average)."""
    corners = [(x, y, z) for z in (1, -1) for (x, y) in ((1, 1), (-1, 1), (-1, -1), (1, -1))]
    n = 9
    J = np.zeros((n, n))
    for v in range(1, 9):
        J[0, v] = 1.0
    for layer in (0, 4):
        for k in range(4):
            a, b = 1 + layer + k, 1 + layer + (k + 1) % 4
            J[min(a, b), max(a, b)] = 0.5
    for k in range(4):
        J[1 + k, 5 + k] = 0.3
    phi = np.array([math.radians(10.0 if v % 2 else -10.0) for v in range(8)])
    axes = np.zeros((n, 3))
    axes[0] = (0, 0, 1)
    axes[1:] = _tilted_axes(phi, math.radians(30.0))
    d = np.zeros(n)
    d[1:] = -2.0
    two_s = np.array([5] + [4] * 8, np.int32)
    dirs = dodecahedron_directions()
    sysm = System(two_s=two_s, J=J, d=d, e=axes, g=np.full(n, 2.0), B=float(B) * dirs[0],
                  pos=None, name="mn9")
    return sysm, RunSpec(R=20, n_lanczos=100, seed=7000, T=t_grid(), fields=float(B) * dirs)


WORKLOADS = {
    "cfg1": cfg1, "cfg2": cfg2, "cfg2_hb": cfg2_hb, "cfg4": cfg4, "cfg4_hb": cfg4_hb,
    "ring6": ring6, "mn9": mn9,
}
