"""Pins of the oracle's Krylov construction (no GPU).

  * Eq. (5) worked example: binomial expansion of H^r|0> on the uniform chain
    (tests/golden/chain_binomial.txt) and the Lanczos coefficients that follow
    from it (alpha = 0, beta_1 = sqrt 2, beta_k = 1), with the decoupled p
    seeds deflating at the first step;
  * block-Krylov structure: Q^T Q = I, Q^T H Q block-tridiagonal, block Gauss
    quadrature E1^T T^k E1 = Phi^T H^k Phi for k <= 2r - 1;
  * exactness once the Krylov space is invariant (Sec. 3: accuracy is complete
    at the degree of the minimal polynomial): rho column = f(H) Phi from the
    library eigensolver of the cluster Hamiltonian;
  * two independent basis constructions agree.
"""
import os

import numpy as np
import pytest

from paper_0910_4497_amd import inputs
from oracle import geometry, krylov, tb

P = inputs.load_params()
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def s_only_params(t=1.0, spacing=1.5):
    p = dict(P)
    p["v_sps"] = p["v_pps"] = p["v_ppp"] = 0.0
    p["eps_s"] = 0.0
    p["eps_p"] = 10.0
    p["v_sss"] = t / float(krylov.model.s_radial(spacing, P))
    return p


def chain_H(n_sites, p, spacing=1.5):
    pos = inputs.chain_positions(n_sites, spacing)
    c = n_sites // 2
    idx, x = geometry.cluster(c, pos, np.array([1e3] * 3), (0, 0, 0), 1e3)
    return krylov.cluster_hamiltonian(x, p), idx, pos


def test_eq5_binomial_chain():
    p = s_only_params()
    n = 21
    H, idx, pos = chain_H(n, p)
    site_of = {int(g): a for a, g in enumerate(idx)}
    c = n // 2
    rows = [list(map(int, l.split())) for l in open(os.path.join(GOLD, "chain_binomial.txt"))
            if l.strip() and not l.startswith("#")]
    v = np.zeros(H.shape[0])
    v[0] = 1.0                                        # s orbital of the centre atom
    for r_pow, *coef in rows:
        if r_pow > 0:
            v = H @ v
        expect = np.zeros(H.shape[0])
        for k, cval in enumerate(coef):
            g = c + (2 * k - r_pow)
            expect[4 * site_of[g]] = cval
        assert np.allclose(v, expect, atol=1e-9 * max(coef)), r_pow


def test_chain_lanczos_coefficients_and_deflation():
    p = s_only_params(t=1.0)
    M = 10
    H, _, _ = chain_H(2 * M + 1, p)
    r = M
    Q, T = krylov.block_lanczos(H, r)
    # seed block 4 wide, then the decoupled p seeds deflate: width 1 after
    widths = [4] + [1] * (r - 1)
    assert Q.shape[1] == sum(widths)
    # p orbitals: isolated on-site energy
    assert np.allclose(np.diag(T)[1:4], 10.0)
    s_idx = [0] + list(range(4, Q.shape[1]))
    Ts = T[np.ix_(s_idx, s_idx)]
    beta = np.abs(np.diag(Ts, -1))
    assert np.allclose(np.diag(Ts), 0.0, atol=1e-13)
    assert abs(beta[0] - np.sqrt(2.0)) < 1e-13
    assert np.allclose(beta[1:], 1.0, atol=1e-13)
    # same subspace through the other construction
    Q2, widths2 = krylov.block_krylov_basis(H, r)
    assert widths2 == widths
    assert np.allclose(Q2 @ Q2.T, Q @ Q.T, atol=1e-12)


def test_chain_moments_closed_form():
    """<s0|(H - E_s)^k|s0> = C(k, k/2) t^k for even k, 0 for odd k (walks on the
    chain), reproduced by the block Gauss quadrature of the Krylov T."""
    from math import comb
    t = 0.8
    p = s_only_params(t=t)
    M = 8
    H, _, _ = chain_H(2 * M + 1, p)
    r = M
    Q, T = krylov.block_lanczos(H, r)
    lam, Y = np.linalg.eigh(T)
    for k in range(0, 2 * r):
        mom = float(np.sum(Y[0, :] ** 2 * lam ** k))
        exp = comb(k, k // 2) * t ** k if k % 2 == 0 else 0.0
        assert abs(mom - exp) < 1e-10 * max(1.0, exp), k


@pytest.fixture(scope="module")
def cfg1_cluster():
    w = inputs.workload("c60_240")
    idx, x = geometry.cluster(7, w.pos, w.cell, (1, 1, 1), w.r_cut)
    return krylov.cluster_hamiltonian(x, P), w


def test_basis_orthonormal_and_block_tridiagonal(cfg1_cluster):
    H, w = cfg1_cluster
    r = w.r
    Q, widths = krylov.block_krylov_basis(H, r)
    assert widths == [4] * r
    assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() < 1e-13
    T = Q.T @ H @ Q
    band = np.abs(np.subtract.outer(np.arange(T.shape[0]) // 4, np.arange(T.shape[0]) // 4)) > 1
    assert np.abs(T[band]).max() < 1e-12 * np.linalg.norm(H)


def test_block_gauss_quadrature(cfg1_cluster):
    H, w = cfg1_cluster
    r = 6
    Q, _ = krylov.block_krylov_basis(H, r)
    T = Q.T @ H @ Q
    Hs = H / np.linalg.norm(H, 2)
    Ts = T / np.linalg.norm(H, 2)
    for k in range(2 * r):
        Mh_k = np.linalg.matrix_power(Hs, k)[:4, :4]
        Mt_k = np.linalg.matrix_power(Ts, k)[:4, :4]
        assert np.allclose(Mh_k, Mt_k, atol=1e-12), k
    # and it fails beyond: degree 2r is not integrated exactly
    k = 2 * r + 2
    assert np.abs(np.linalg.matrix_power(Hs, k)[:4, :4]
                  - np.linalg.matrix_power(Ts, k)[:4, :4]).max() > 1e-10


def test_routes_agree(cfg1_cluster):
    w = inputs.workload("c60_240")
    for i in (0, 101, 239):
        a = tb.atom_solve(i, w.pos, w.cell, (1, 1, 1), P, w.r_cut, w.r, route="arnoldi")
        b = tb.atom_solve(i, w.pos, w.cell, (1, 1, 1), P, w.r_cut, w.r, route="lanczos")
        assert np.allclose(a["lam"], b["lam"], atol=1e-11)
        for mu in (-2.0, 0.0, 1.5):
            ra, rb = tb.rho_blocks_from(a, mu, 0.1), tb.rho_blocks_from(b, mu, 0.1)
            assert np.abs(ra - rb).max() < 1e-11


def test_invariant_space_equals_cluster_solution():
    """Isolated jittered C60, small cutoff sphere: once r reaches the grade the
    Krylov rho column equals f(H^(i)) Phi_i from numpy.linalg.eigh."""
    rng = np.random.default_rng(11)
    mol = inputs.c60_ideal() + rng.normal(0, 0.03, (60, 3))
    cell = np.array([100.0] * 3)
    i, r_cut = 3, 3.2
    idx, x = geometry.cluster(i, mol, cell, (0, 0, 0), r_cut)
    H = krylov.cluster_hamiltonian(x, P)
    n4 = H.shape[0]
    r = n4 // 4 + 3                                   # beyond the grade
    Q, widths = krylov.block_krylov_basis(H, r)
    assert widths[-1] == 0 and Q.shape[1] <= n4       # invariant space reached
    sol = tb.atom_solve(i, mol, cell, (0, 0, 0), P, r_cut, r, full_column=True)
    ev, U = np.linalg.eigh(H)
    for mu in (-1.0, 0.5):
        exact = (U * tb.fermi(ev, mu, 0.1)) @ U[:4, :].T
        got = tb.rho_column_full(sol, mu, 0.1).reshape(-1, 4)
        assert np.abs(exact - got).max() < 1e-12


# ---------------------------------------------------- orbital seeds (Eqs. 6-9)
def test_orbital_chain_closed_form():
    """Uniform s-only chain, seed = the s orbital of the centre site: the
    scalar recursion of Eqs. (6)-(7) gives alpha_k = E_s = 0, beta_1 = sqrt(2)|t|
    and beta_k = |t| after; a p seed is an eigenvector (its chain stops at once)."""
    p = s_only_params(t=1.0)
    M = 10
    H, _, _ = chain_H(2 * M + 1, p)
    V, a, b = krylov.orbital_lanczos(H, M, 0)
    assert np.allclose(a, 0.0, atol=1e-13)
    assert abs(b[0] - np.sqrt(2.0)) < 1e-13 and np.allclose(b[1:], 1.0, atol=1e-13)
    assert np.abs(V.T @ V - np.eye(V.shape[1])).max() < 1e-13
    for c in (1, 2, 3):
        Vp, ap, bp = krylov.orbital_lanczos(H, M, c)
        assert len(bp) == 0 and abs(ap[0] - 10.0) < 1e-13


def test_orbital_routes_agree(cfg1_cluster):
    """Per orbital, the Ritz values of the Arnoldi basis of K_r(H, e_c) equal
    those of the three-term recursion (two independent constructions)."""
    H, w = cfg1_cluster
    for c in range(4):
        Q = krylov.orbital_krylov_basis(H, w.r, c)
        lam1 = np.linalg.eigvalsh(Q.T @ H @ Q)
        V, a, b = krylov.orbital_lanczos(H, w.r, c)
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        lam2 = np.linalg.eigvalsh(T)
        assert np.abs(lam1 - lam2).max() < 1e-10


def test_orbital_space_is_inside_block_space(cfg1_cluster):
    """K_r(H, e_c) is a subspace of the block space K_r(H, Phi)."""
    H, w = cfg1_cluster
    Qb, _ = krylov.block_krylov_basis(H, w.r)
    for c in range(4):
        Q = krylov.orbital_krylov_basis(H, w.r, c)
        assert np.abs(Q - Qb @ (Qb.T @ Q)).max() < 1e-9


def test_orbital_exact_limit_and_rotation():
    """Isolated C60 with every sphere the whole molecule: with r past every
    orbital's grade the orbital form equals full diagonalisation; at a finite
    r its energy changes under a rigid rotation of the molecule, while the
    block form's does not (its result depends on span(Phi) only)."""
    from oracle import exact
    rng = np.random.default_rng(21)
    mol = inputs.c60_ideal() + rng.normal(0, 0.04, (60, 3))
    big = np.array([200.0, 200.0, 200.0])
    kr = tb.run(mol, big, (0, 0, 0), P, 8.0, 250, 0.1, n_electrons=240.0, processes=8, seeds="orbital")
    ex = exact.solve(mol, big, (0, 0, 0), P, 0.1, n_electrons=240.0)
    assert abs(kr["mu"] - ex["mu"]) < 1e-10
    assert abs(kr["e_total"] - ex["e_total"]) < 1e-9 * abs(ex["e_total"])
    assert np.abs(kr["forces"] - ex["forces"]).max() < 1e-9
    Rm = inputs.random_rotation(np.random.default_rng(5))
    c0 = mol.mean(axis=0)
    rot = (mol - c0) @ Rm.T + c0
    e = {}
    for seeds in ("block", "orbital"):
        e[seeds] = [tb.run(x, big, (0, 0, 0), P, 6.0, 10, 0.1, n_electrons=240.0, processes=8,
                           seeds=seeds)["e_total"] for x in (mol, rot)]
    assert abs(e["block"][0] - e["block"][1]) < 1e-9 * abs(e["block"][0])
    assert abs(e["orbital"][0] - e["orbital"][1]) > 1e-6
