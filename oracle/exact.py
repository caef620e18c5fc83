"""Full diagonalisation of the whole Hamiltonian (the O(N^3) route of Sec. 2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

rho = sum_m |m> f(eps_m) <m| (Eq. 2) from numpy.linalg.eigh of the global
4N x 4N H; used on tiny systems as the exact limit the local Krylov solve
must reach once every cluster is the whole system and r reaches the grade.
"""
from __future__ import annotations

import numpy as np

from . import geometry, model, tb


def global_hamiltonian(pos, cell, periodic, p):
    N = pos.shape[0]
    H4 = np.zeros((N, 4, N, 4))
    nb, dv = geometry.neighbour_lists(pos, cell, periodic, p["rm"])
    for i in range(N):
        H4[i, :, i, :] = model.onsite_block(p)
        if len(nb[i]):
            H4[i, :, nb[i], :] = model.sk_blocks(dv[i], p)
    return H4.reshape(4 * N, 4 * N)


def solve(pos, cell, periodic, p, kT, n_electrons=None, mu=None):
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[0]
    H = global_hamiltonian(pos, cell, periodic, p)
    eps, U = np.linalg.eigh(H)
    if mu is None:
        mu = tb.chemical_potential([eps], [np.ones_like(eps)], n_electrons, kT)
    f = tb.fermi(eps, mu, kT)
    rho = (U * f[None, :]) @ U.T
    e_band = float(np.sum(eps * f))
    ent = float(np.sum(tb.entropy_per_level(eps, mu, kT)))
    e_rep, f_rep = tb.repulsion(pos, cell, periodic, p)
    nb, dv = geometry.neighbour_lists(pos, cell, periodic, p["rm"])
    rho4 = rho.reshape(N, 4, N, 4)
    grad = np.zeros((N, 3))
    for i in range(N):
        if len(nb[i]) == 0:
            continue
        dH = model.sk_blocks_grad(dv[i], p)                 # [p][c][beta][alpha]
        rji = rho4[nb[i], :, i, :]                           # [p][alpha][beta]
        g = np.einsum("pcba,pab->pc", dH, rji)
        grad[nb[i]] += g
        grad[i] -= g.sum(axis=0)
    return {"mu": mu, "eps": eps, "rho": rho, "e_band": e_band, "entropy": ent,
            "free_band": e_band - kT * ent, "e_rep": e_rep,
            "e_total": e_band - kT * ent + e_rep, "forces": -grad + f_rep, "H": H}
