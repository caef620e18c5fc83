"""Pins of the oracle's grouped form (Sec. 3, Eqs. 6-9): the m atoms of a group
run their scalar chains on one Hamiltonian, that of the union of their cutoff
spheres.

* exact limit: one group holding a whole isolated molecule, with cutoff
  spheres much smaller than the molecule, gives full diagonalisation once r
  passes every chain's grade; the per-atom form at the same cutoff does not;
* reach: on a uniform chain a recursion of order r equals the untruncated one
  exactly when the sphere reaches r - 1 sites past the seed (all r Lanczos
  vectors and the products forming T stay inside it); the union sphere of the
  middle member of a group of three reaches one site further than the
  member's own sphere, and the orders at which the two forms stop being exact
  differ by one;
* brute force: union membership and cluster-frame positions from an explicit
  loop over periodic images on a small box, and the error when the group's
  spread plus the cutoff reaches half the cell.
"""
import itertools

import numpy as np
import pytest

from paper_0910_4497_amd import inputs
from oracle import exact, geometry, krylov, tb

P = inputs.load_params()


def s_only_params(t=1.0, spacing=1.5):
    p = dict(P)
    p["v_sps"] = p["v_pps"] = p["v_ppp"] = 0.0
    p["eps_s"] = 0.0
    p["eps_p"] = 10.0
    p["v_sss"] = t / float(krylov.model.s_radial(spacing, P))
    return p


def test_group_exact_limit_whole_molecule():
    rng = np.random.default_rng(31)
    mol = inputs.c60_ideal() + rng.normal(0, 0.04, (60, 3))
    big = np.array([200.0, 200.0, 200.0])
    r_cut = 3.2                                           # own spheres: a few atoms
    sizes = [len(geometry.cluster(i, mol, big, (0, 0, 0), r_cut)[0]) for i in range(60)]
    assert max(sizes) < 20
    kw = dict(n_electrons=240.0, processes=8, seeds="orbital")
    grouped = tb.run(mol, big, (0, 0, 0), P, r_cut, 250, 0.1, group=60, **kw)
    ex = exact.solve(mol, big, (0, 0, 0), P, 0.1, n_electrons=240.0)
    assert abs(grouped["mu"] - ex["mu"]) < 1e-10
    assert abs(grouped["e_total"] - ex["e_total"]) < 1e-9 * abs(ex["e_total"])
    assert np.abs(grouped["forces"] - ex["forces"]).max() < 1e-9
    own = tb.run(mol, big, (0, 0, 0), P, r_cut, 250, 0.1, **kw)
    assert np.abs(own["forces"] - ex["forces"]).max() > 1e-3


def _chain_column(sol, mu, kT):
    """rho_{j s, i s} on the J rows of a solve (s orbitals only)."""
    return tb.rho_blocks_from(sol, mu, kT)[:, 0, 0]


def test_group_reach_on_uniform_chain():
    spacing, n_sites = 1.5, 41
    p = s_only_params(t=1.0, spacing=spacing)
    pos = inputs.chain_positions(n_sites, spacing)
    cell, per = np.array([1e3] * 3), (0, 0, 0)
    r_cut = 8.0                      # own sphere: 5 sites on each side (7.5 A < 8 < 9 A)
    c = 19                           # middle member of the group {18, 19, 20}
    assert list(geometry.group_of(c, 3, n_sites)) == [18, 19, 20]
    idx_u, _ = geometry.group_cluster(c, 3, pos, cell, per, r_cut)
    assert sorted(idx_u) == list(range(13, 26))          # 6 sites on each side
    mu, kT = 0.3, 0.5
    for r, own_exact, group_exact in ((6, True, True), (7, False, True), (8, False, False)):
        ref = tb.atom_solve(c, pos, cell, per, p, 100.0, r, seeds="orbital")      # untruncated
        own = tb.atom_solve(c, pos, cell, per, p, r_cut, r, seeds="orbital")
        grp = tb.atom_solve(c, pos, cell, per, p, r_cut, r, seeds="orbital", group=3)
        assert list(ref["J"]) == list(own["J"]) == list(grp["J"]) == [19, 18, 20]
        x_ref = _chain_column(ref, mu, kT)
        d_own = np.abs(_chain_column(own, mu, kT) - x_ref).max()
        d_grp = np.abs(_chain_column(grp, mu, kT) - x_ref).max()
        assert (d_own < 1e-13) == own_exact and (d_own > 1e-9 or own_exact), (r, d_own)
        assert (d_grp < 1e-13) == group_exact and (d_grp > 1e-9 or group_exact), (r, d_grp)


def test_group_cluster_brute_force_images():
    # 8 loose groups of 3 (members 0.8 A rms about a centre): most unions take
    # in part of another group, and a few groups are too spread for the box
    rng = np.random.default_rng(0)
    L = np.array([11.0, 12.0, 13.0])
    cen = rng.uniform(0, 1, (8, 3)) * L
    pos = (np.repeat(cen, 3, axis=0) + rng.normal(0, 0.8, (24, 3))) % L
    per = (1, 1, 1)
    m, r_cut = 3, 3.5
    n_checked = n_refused = n_partial = 0
    shifts = [np.array(s) * L for s in itertools.product((-1, 0, 1), repeat=3)]
    for i in range(24):
        members = [k for k in range(24) if k // m == i // m]
        spread_ok = True
        d_i = {}
        for j in range(24):
            best = min((pos[j] + s - pos[i] for s in shifts), key=np.linalg.norm)
            d_i[j] = best
        for k in members:
            if np.any(np.abs(d_i[k]) + r_cut >= 0.5 * L):
                spread_ok = False
        if not spread_ok:
            with pytest.raises(ValueError):
                geometry.group_cluster(i, m, pos, L, per, r_cut)
            n_refused += 1
            continue
        expect = []
        for j in range(24):
            if j == i:
                continue
            near = min(np.linalg.norm(pos[j] + s - pos[k]) for k in members for s in shifts)
            if near < r_cut:
                expect.append(j)
        idx, x = geometry.group_cluster(i, m, pos, L, per, r_cut)
        assert list(idx) == [i] + expect
        for a, j in enumerate(idx):
            assert np.abs(x[a] - d_i[int(j)]).max() < 1e-12
        n_checked += 1
        outside = {int(j) // m for j in idx if int(j) // m != i // m}
        n_partial += any(any(g * m + t not in idx for t in range(m)) for g in outside)
    assert n_checked >= 20 and n_refused >= 1 and n_partial >= 10, (n_checked, n_refused, n_partial)
    # a group whose spread plus the cutoff reaches half the cell is refused
    bad = np.zeros((4, 3))
    bad[1, 0] = 3.0
    with pytest.raises(ValueError):
        geometry.group_cluster(0, 4, bad, np.array([11.0, 50.0, 50.0]), per, 3.0)


@pytest.mark.parametrize("m", [1, 2, 4, 7])
def test_group_order_permutation_and_compactness(m):
    """inputs.group_order is a permutation whose index blocks of m are compact:
    on the 1920-atom crystal every group of 2 or 4 satisfies the image
    condition of the union spheres at R_cut = 7 A (spread + R_cut < L/2)."""
    w = inputs.workload("c60_1920")
    L = np.asarray(w.cell)
    perm = inputs.group_order(w.pos, L, (1, 1, 1), m)
    assert sorted(perm.tolist()) == list(range(w.n_atoms))
    pos = w.pos[perm]
    worst = 0.0
    for g0 in range(0, w.n_atoms, m):
        G = np.arange(g0, min(w.n_atoms, g0 + m))
        for i in G:
            d = geometry.min_image(pos[G] - pos[i], L, (1, 1, 1))
            worst = max(worst, float(np.abs(d).max()))
    if m in (2, 4):
        assert worst + w.r_cut < 0.5 * L.min(), worst
    if m == 1:
        assert list(perm) == list(range(w.n_atoms))
