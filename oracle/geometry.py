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
