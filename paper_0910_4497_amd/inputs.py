"""Seeded synthetic inputs: compressed fcc C60 crystals, the parameter record,
Maxwell velocities.

This module builds geometry and random draws only; it holds none of the
tight-binding arithmetic.  Both the GPU path and the CPU oracle are fed from
it, so that they see bit-identical inputs.

Workloads follow the paper's C60 setting (Sec. 4: a 2x2x2 fcc C60 crystal of
1920 atoms as the starting structure, compressed runs) with these recipes:

  * C60: truncated icosahedron obtained by cutting every edge of an
    icosahedron of edge 4.30 A at fraction t = 1.45/4.30 from both ends, giving
    pentagon bonds of 1.45 A and hexagon-hexagon bonds of 1.40 A.
  * molecular centres on the fcc conventional-cell sites
    (0,0,0), (0,1/2,1/2), (1/2,0,1/2), (1/2,1/2,0) * a, replicated k x k x k
    (cell loop x slowest, then y, then z, then the 4 basis sites);
  * one uniform random rotation per molecule (quaternion of 4 standard
    normals, normalised), drawn in the same loop order;
  * Gaussian jitter N(0, sigma) on every coordinate, then wrap into [0, L).
  * optional strain of the molecular centres along x (before rotation):
    x_c <- x_c + eps * (x_c^2 / L - x_c), a periodic displacement whose local
    strain runs linearly from -eps to +eps across the cell.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_XU = os.path.join(_HERE, "params", "xu1992.json")
PARAMS_LONG = os.path.join(_HERE, "params", "xu_longrange.json")   # hopping to 7 A

# Unit system: eV, Angstrom, fs, amu.
K_B = 8.617333262e-5            # eV / K
ACC_UNIT = 9.648533212e-3       # (eV / (A amu)) expressed in A / fs^2
MASS_C = 12.011                 # amu

PARAM_KEYS = ("eps_s", "eps_p", "v_sss", "v_sps", "v_pps", "v_ppp",
              "r0", "n", "nc", "rc", "r1", "rm", "s_tail",
              "phi0", "d0", "m", "mc", "dc", "d1", "dm", "phi_tail", "frep")


def load_params(path: str = PARAMS_XU) -> dict:
    """Parameter record as a plain dict (floats and float lists)."""
    with open(path) as fh:
        rec = json.load(fh)
    return {k: rec[k] for k in PARAM_KEYS}


def c60_ideal(edge: float = 4.30, bond_pent: float = 1.45) -> np.ndarray:
    """Ideal C60 centred at the origin, shape (60, 3), deterministic order."""
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    ico = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            ico.append((0.0, s1, s2 * phi))
            ico.append((s1, s2 * phi, 0.0))
            ico.append((s2 * phi, 0.0, s1))
    ico = np.array(ico) * (edge / 2.0)          # raw edge length is 2
    t = bond_pent / edge
    atoms = []
    for u in range(12):
        for v in range(u + 1, 12):
            if abs(np.linalg.norm(ico[u] - ico[v]) - edge) < 1e-9:
                atoms.append(ico[u] + t * (ico[v] - ico[u]))
                atoms.append(ico[v] + t * (ico[u] - ico[v]))
    out = np.array(atoms)
    assert out.shape == (60, 3)
    return out


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a normalised 4-vector of standard normals."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def fcc_c60(k: int, a: float, sigma: float, seed: int, strain: float = 0.0):
    """k x k x k conventional fcc cells of C60.  Returns (pos [N,3], L [3])."""
    rng = np.random.default_rng(seed)
    mol = c60_ideal()
    L = k * a
    basis = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]]) * a
    pos = []
    for ix in range(k):
        for iy in range(k):
            for iz in range(k):
                for b in basis:
                    c = np.array([ix * a, iy * a, iz * a]) + b
                    if strain:
                        c[0] = c[0] + strain * (c[0] * c[0] / L - c[0])
                    R = random_rotation(rng)
                    pos.append(c + mol @ R.T)
    pos = np.concatenate(pos, axis=0)
    if sigma > 0:
        pos = pos + rng.normal(0.0, sigma, pos.shape)
    pos = np.mod(pos, L)
    return pos, np.array([L, L, L]), rng


def cubic_diamond(k: int, a: float, sigma: float = 0.0, seed: int = 0):
    """k x k x k conventional cubic-diamond cells (8 atoms each: the fcc sites
    and the same shifted by (1/4, 1/4, 1/4) a), loop order x slowest, Gaussian
    jitter sigma (A), wrapped into the box. Returns (pos, cell lengths)."""
    fcc = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]], dtype=np.float64)
    basis = np.concatenate([fcc, fcc + 0.25], axis=0)
    pos = []
    for i in range(k):
        for j in range(k):
            for l in range(k):
                pos.append((basis + np.array([i, j, l], dtype=np.float64)) * a)
    pos = np.concatenate(pos, axis=0)
    L = k * a
    if sigma > 0:
        pos = pos + np.random.default_rng(seed).normal(0.0, sigma, pos.shape)
    return np.mod(pos, L), np.array([L, L, L])


@dataclass
class Workload:
    name: str
    pos: np.ndarray                 # [N,3] A, wrapped into the cell
    cell: np.ndarray                # [3] orthorhombic box lengths, A
    periodic: tuple = (1, 1, 1)
    r_cut: float = 7.0              # cluster radius, A
    r: int = 40                     # block-Krylov order (block steps)
    kT: float = 0.1                 # eV
    r_per_atom: np.ndarray | None = None
    extra: dict = field(default_factory=dict)
    params: str = PARAMS_XU         # parameter file
    hop_max: int = 24               # hop-list capacity the workload needs

    @property
    def n_atoms(self) -> int:
        return self.pos.shape[0]

    @property
    def n_electrons(self) -> float:
        return 4.0 * self.n_atoms


def workload(name: str) -> Workload:
    """The five C60 workloads (names 'c60_240' ... 'c60_15360'), the
    4 x 4 x 4 cubic-diamond cell 'diamond_512', 'c60_1920_long' (the
    1920-atom crystal with the long-range hopping of PARAMS_LONG) and the
    size series 'c60_scale_k<k>' (k x k x k cells, lattice constant, jitter,
    cutoff radius and Krylov order of c60_1920; k = 2 is c60_1920 itself)."""
    if name == "c60_240":           # one compressed conventional cell
        pos, L, _ = fcc_c60(1, 12.5, 0.02, 1001)
        return Workload(name, pos, L, r_cut=6.0, r=30)
    if name == "c60_1920":          # 2x2x2 cells, precision study
        pos, L, _ = fcc_c60(2, 12.0, 0.05, 1002)
        return Workload(name, pos, L, r_cut=7.0, r=40)
    if name == "c60_6480_strained":  # 3x3x3 cells, +-4% strain, mixed r
        pos, L, rng = fcc_c60(3, 11.8, 0.10, 1003, strain=0.04)
        rpa = rng.choice(np.array([30, 40, 50]), pos.shape[0]).astype(np.int32)
        return Workload(name, pos, L, r_cut=7.0, r=50, r_per_atom=rpa)
    if name == "c60_1920_hot":      # 2x2x2 cells, sigma 0.08 (FD / NVE study)
        pos, L, _ = fcc_c60(2, 12.0, 0.08, 1004)
        return Workload(name, pos, L, r_cut=7.0, r=40,
                        extra={"fd_seed": 3004, "md_seed": 2004, "T_K": 1500.0})
    if name == "c60_15360":         # 4x4x4 cells, full scale
        pos, L, _ = fcc_c60(4, 11.6, 0.10, 1005)
        return Workload(name, pos, L, r_cut=8.0, r=50)
    if name == "diamond_512":       # 4x4x4 cubic-diamond cells (pressure / EOS)
        pos, L = cubic_diamond(4, 3.567, 0.02, 1006)
        return Workload(name, pos, L, r_cut=6.0, r=30)
    if name == "c60_1920_long":     # the 1920-atom crystal with hopping to 7 A (dense local H)
        pos, L, _ = fcc_c60(2, 12.0, 0.05, 1002)
        return Workload(name, pos, L, r_cut=8.0, r=40, params=PARAMS_LONG, hop_max=256)
    if name.startswith("c60_scale_k"):  # k x k x k cells at the c60_1920 settings (N = 240 k^3)
        k = int(name[len("c60_scale_k"):])
        if not 1 <= k <= 8:
            raise KeyError(name)
        pos, L, _ = fcc_c60(k, 12.0, 0.05, 1002 if k == 2 else 1010 + k)
        return Workload(name, pos, L, r_cut=7.0, r=40)
    raise KeyError(name)


WORKLOADS = ("c60_240", "c60_1920", "c60_6480_strained", "c60_1920_hot", "c60_15360", "diamond_512",
             "c60_1920_long")


def maxwell_velocities(n: int, T: float, seed: int, mass: float = MASS_C) -> np.ndarray:
    """Maxwell-Boltzmann velocities (A/fs) at temperature T (K), zero centre-of-
    mass velocity, rescaled to exactly T over 3N-3 degrees of freedom."""
    rng = np.random.default_rng(seed)
    # variance of one component: kT/m in (eV/amu) -> A^2/fs^2 via ACC_UNIT
    sd = np.sqrt(K_B * T / mass * ACC_UNIT)
    v = rng.normal(0.0, sd, (n, 3))
    v -= v.mean(axis=0)
    ke = 0.5 * mass * np.sum(v * v) / ACC_UNIT          # eV
    t_now = 2.0 * ke / ((3 * n - 3) * K_B)
    return v * np.sqrt(T / t_now)


def kinetic_energy(v: np.ndarray, mass: float = MASS_C) -> float:
    """Kinetic energy in eV of velocities in A/fs."""
    return 0.5 * mass * float(np.sum(v * v)) / ACC_UNIT


def chain_positions(n_sites: int, spacing: float, axis: int = 2) -> np.ndarray:
    """Straight open chain of atoms centred on site n_sites//2 (small tests)."""
    pos = np.zeros((n_sites, 3))
    pos[:, axis] = (np.arange(n_sites) - n_sites // 2) * spacing
    return pos


def group_order(pos: np.ndarray, cell, periodic, m: int) -> np.ndarray:
    """Permutation that puts the atoms in compact groups of m consecutive
    indices (for the grouped form, whose groups are index blocks): recursive
    median bisection along the widest axis of the wrapped coordinates, the
    parts kept at multiples of m atoms; each leaf (m atoms, one ragged) is a
    group, its members in increasing index. pos[perm] is the reordered input;
    m = 1 keeps the order."""
    if m <= 1:
        return np.arange(np.asarray(pos).shape[0])
    x = np.array(pos, dtype=np.float64)
    cell = np.asarray(cell, dtype=np.float64)
    for a in range(3):
        if periodic[a]:
            x[:, a] -= cell[a] * np.floor(x[:, a] / cell[a])
    out, stack = [], [np.arange(x.shape[0])]
    while stack:
        idx = stack.pop()
        if len(idx) <= m:
            out.append(np.sort(idx))
            continue
        a = int(np.argmax(x[idx].max(axis=0) - x[idx].min(axis=0)))
        k = ((len(idx) // m + 1) // 2) * m
        o = idx[np.argsort(x[idx, a], kind="stable")]
        stack.append(o[k:])
        stack.append(o[:k])
    return np.concatenate(out)
