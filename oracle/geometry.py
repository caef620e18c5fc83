"""Minimum-image neighbour lists and cutoff-sphere clusters, by brute force.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 2 of the paper reaches linear scaling by solving each target atom with
only the atoms inside a cutoff radius around it (n atoms), cost O(n^3 N).
Here:
  d_ij   = minimum-image vector R_j - R_i (per periodic axis),
  hop(i) = {j != i : |d_ij| < r_m}  (r_m = hopping cutoff, 2.6 A for Xu),
  C_i    = {i} followed by {j != i : |d_ij| < R_cut} in increasing j,
  x_j    = d_ij, the position of j in the frame of the target atom i.
"""
from __future__ import annotations

import numpy as np


def min_image(d, cell, periodic):
    d = np.array(d, dtype=np.float64, copy=True)
    for ax in range(3):
        if periodic[ax]:
            d[..., ax] -= cell[ax] * np.round(d[..., ax] / cell[ax])
    return d


def displacements_from(i, pos, cell, periodic):
    """All d_ij = mic(R_j - R_i) for fixed i, shape (N, 3)."""
    return min_image(pos - pos[i], cell, periodic)


def neighbour_lists(pos, cell, periodic, cutoff):
    """For every atom: sorted indices j != i with |d_ij| < cutoff, and d_ij."""
    out_idx, out_d = [], []
    for i in range(pos.shape[0]):
        d = displacements_from(i, pos, cell, periodic)
        r = np.linalg.norm(d, axis=1)
        sel = np.nonzero(r < cutoff)[0]
        sel = sel[sel != i]
        out_idx.append(sel)
        out_d.append(d[sel])
    return out_idx, out_d


def cluster(i, pos, cell, periodic, r_cut):
    """C_i with the target first, and the cluster-frame positions x."""
    d = displacements_from(i, pos, cell, periodic)
    r = np.linalg.norm(d, axis=1)
    sel = np.nonzero(r < r_cut)[0]
    sel = sel[sel != i]
    idx = np.concatenate([[i], sel]).astype(np.int64)
    x = np.concatenate([np.zeros((1, 3)), d[sel]], axis=0)
    return idx, x


def group_of(i, m, n_atoms):
    """The group of atom i in the paper's grouped form (Sec. 3, Eqs. 6-9):
    consecutive index blocks {g m, ..., g m + m - 1} (the last one ragged)."""
    g0 = (i // m) * m
    return np.arange(g0, min(n_atoms, g0 + m))


def group_cluster(i, m, pos, cell, periodic, r_cut):
    """Union sphere C_G of the group G of atom i, shared by the group's chains
    (Sec. 3: the m atoms of a group run their recursions on one Hamiltonian):
    {i} followed by {j != i : min_{k in G} |d_kj| < R_cut} in increasing j,
    with positions x_j = d_ij in the frame of i.  Those are the right images
    only when |(d_ik)_a| + R_cut < L_a / 2 for every member k and periodic
    axis a; otherwise ValueError."""
    N = pos.shape[0]
    members = group_of(i, m, N)
    d_i = displacements_from(i, pos, cell, periodic)
    for ax in range(3):
        if periodic[ax] and np.any(np.abs(d_i[members, ax]) + r_cut >= 0.5 * cell[ax]):
            raise ValueError("group spread plus cutoff reaches half the cell: ambiguous images")
    inside = np.zeros(N, dtype=bool)
    for k in members:
        inside |= np.linalg.norm(displacements_from(k, pos, cell, periodic), axis=1) < r_cut
    sel = np.nonzero(inside)[0]
    sel = sel[sel != i]
    idx = np.concatenate([[i], sel]).astype(np.int64)
    x = np.concatenate([np.zeros((1, 3)), d_i[sel]], axis=0)
    return idx, x
