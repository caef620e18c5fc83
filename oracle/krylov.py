"""Local Hamiltonian, block-Krylov basis and the block Lanczos recursion.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 3 of the paper: the Hilbert space of the cutoff sphere (Eq. 3) is
replaced by the Krylov subspace K_r(H, phi) = span{phi, H phi, ...,
H^{r-1} phi} (Eq. 4), seeded with the atomic orbital(s) of the target atom.
Here the seed is the block of all four orbitals of the target atom (local
index 0), so K_r is spanned by the columns of Phi, H Phi, ..., H^{r-1} Phi
and has dimension <= 4r.  The projected matrix T = Q^T H Q over an
orthonormal basis Q of K_r is what the paper diagonalises (the tridiagonal
T of the Lanczos recursion, Eqs. 6-7; block-tridiagonal in block form).

Two independent constructions of an orthonormal basis of the same K_r are
given; every quantity computed from them depends only on the subspace:

  block_krylov_basis  -- block Arnoldi: H times the newest basis vectors,
                         two classical Gram-Schmidt passes against every
                         earlier vector, then sequential Gram-Schmidt (twice)
                         within the new block, dropping (deflating) any
                         column whose remaining norm is <= tol;
  block_lanczos       -- the three-term recursion of Eqs. (6)-(9) with full
                         4x4 blocks, L_k = H V_k - V_k A_k - V_{k-1} B_{k-1}^T,
                         V_{k+1} B_k = L_k, plus two full re-orthogonalisation
                         passes; the QR step is pivoted Householder, columns
                         with |R_cc| <= tol are dropped.

The paper's own seeding (Sec. 3, Eqs. 6-9) is one orbital at a time: one
scalar chain per orbital of the target atom, batched with diagonal A_k, B_k.
For that form:

  orbital_krylov_basis -- Arnoldi for K_r(H, e_c) with two classical
                          Gram-Schmidt passes (the scalar case of the above);
  orbital_lanczos      -- the scalar three-term recursion of Eqs. (6)-(7)
                          with two full re-orthogonalisation passes, giving
                          alpha_k, beta_k of the tridiagonal T directly.

Deflation threshold: tol = tau * ||H||_F with tau = 1e-12.  A column that is
dropped lies in the span already built, so the subspace is unchanged; if all
columns of a block drop, the space is invariant and the recursion stops.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import model

TAU_DEFLATE = 1e-12


def cluster_hamiltonian(x, p):
    """Dense 4n x 4n H restricted to the cluster (Eq. 1 on the atoms of Eq. 3).

    x: cluster-frame positions (n, 3), target at row 0.  Two cluster atoms a, b
    are coupled iff |x_b - x_a| < r_m, with the block taken from x_b - x_a.
    """
    n = x.shape[0]
    H4 = np.zeros((n, 4, n, 4))
    for a in range(n):
        H4[a, :, a, :] = model.onsite_block(p)
    a_idx, b_idx = np.nonzero(np.ones((n, n), dtype=bool))
    dvec = x[b_idx] - x[a_idx]
    r = np.linalg.norm(dvec, axis=1)
    sel = (a_idx != b_idx) & (r < p["rm"])
    a_idx, b_idx, dvec = a_idx[sel], b_idx[sel], dvec[sel]
    H4[a_idx, :, b_idx, :] = model.sk_blocks(dvec, p)
    return H4.reshape(4 * n, 4 * n)


def deflation_tol(H, tau=TAU_DEFLATE):
    return tau * np.linalg.norm(H)


def block_krylov_basis(H, r, tau=TAU_DEFLATE, reorth=True):
    """Orthonormal basis (columns) of K_r(H, Phi), Phi = first 4 unit vectors.

    Returns (Q, widths) where widths[k] is the number of columns kept at block
    step k (widths[0] = 4 for the seed block).
    """
    dim = H.shape[0]
    tol = deflation_tol(H, tau)
    Q = np.zeros((dim, 4 * r))
    Q[:4, :4] = np.eye(4)
    nq = 4
    newest = list(range(4))
    widths = [4]
    npass = 2 if reorth else 1
    for _k in range(1, r):
        W = H @ Q[:, newest]
        for _ in range(npass):                       # against earlier blocks
            W = W - Q[:, :nq] @ (Q[:, :nq].T @ W)
        kept = []
        for c in range(W.shape[1]):                  # within the new block
            w = W[:, c].copy()
            for _ in range(npass):
                if kept:
                    Qn = Q[:, kept]
                    w = w - Qn @ (Qn.T @ w)
            nrm = np.linalg.norm(w)
            if nrm > tol:
                Q[:, nq] = w / nrm
                kept.append(nq)
                nq += 1
        widths.append(len(kept))
        if not kept:
            break
        newest = kept
    return Q[:, :nq], widths


def block_lanczos(H, r, tau=TAU_DEFLATE, reorth=True):
    """Block three-term recursion (Eqs. 6-9 with full 4x4 blocks).

    Returns (Q, T): the basis [V_1 ... V_r] and the block-tridiagonal T
    assembled from the recursion coefficients A_k (diagonal blocks) and B_k
    (sub-diagonal blocks, transposed above the diagonal).
    """
    dim = H.shape[0]
    tol = deflation_tol(H, tau)
    V = np.zeros((dim, 4))
    V[:4, :4] = np.eye(4)
    V_prev = np.zeros((dim, 0))
    B_prev = np.zeros((4, 0))
    blocks, A_list, B_list = [V], [], []
    for k in range(r):
        W = H @ V
        A = V.T @ W
        A = 0.5 * (A + A.T)
        A_list.append(A)
        if k == r - 1:
            break
        W = W - V @ A - V_prev @ B_prev.T
        if reorth:
            Qall = np.hstack(blocks)
            for _ in range(2):
                W = W - Qall @ (Qall.T @ W)
        if W.shape[1] == 0:
            break
        Qw, Rw, piv = scipy.linalg.qr(W, mode="economic", pivoting=True)
        rank = int(np.sum(np.abs(np.diag(Rw)) > tol))
        if rank == 0:
            break
        Bfull = np.zeros_like(Rw)
        Bfull[:, piv] = Rw                      # W = Qw @ Bfull
        V_next = Qw[:, :rank]
        B = Bfull[:rank, :]
        B_list.append(B)
        V_prev, B_prev, V = V, B, V_next
        blocks.append(V)
    widths = [b.shape[1] for b in blocks]
    offs = np.concatenate([[0], np.cumsum(widths)])
    T = np.zeros((offs[-1], offs[-1]))
    for k, A in enumerate(A_list):
        T[offs[k]:offs[k + 1], offs[k]:offs[k + 1]] = A
    for k, B in enumerate(B_list):
        T[offs[k + 1]:offs[k + 2], offs[k]:offs[k + 1]] = B
        T[offs[k]:offs[k + 1], offs[k + 1]:offs[k + 2]] = B.T
    return np.hstack(blocks), T


def orbital_krylov_basis(H, r, c, tau=TAU_DEFLATE, reorth=True):
    """Orthonormal basis (columns) of K_r(H, e_c), e_c the c-th unit vector;
    stops when the new vector's norm after orthogonalisation is <= tol (the
    space is invariant)."""
    dim = H.shape[0]
    tol = deflation_tol(H, tau)
    Q = np.zeros((dim, r))
    Q[c, 0] = 1.0
    nq = 1
    npass = 2 if reorth else 1
    for _k in range(1, r):
        w = H @ Q[:, nq - 1]
        for _ in range(npass):
            w = w - Q[:, :nq] @ (Q[:, :nq].T @ w)
        nrm = np.linalg.norm(w)
        if nrm <= tol:
            break
        Q[:, nq] = w / nrm
        nq += 1
    return Q[:, :nq]


def orbital_lanczos(H, r, c, tau=TAU_DEFLATE, reorth=True):
    """Scalar three-term recursion (Eqs. 6-7) seeded with e_c:
    l_k = H v_k - alpha_k v_k - beta_{k-1} v_{k-1}, v_{k+1} = l_k / beta_k,
    alpha_k = v_k.H v_k, beta_k = |l_k|, with two full re-orthogonalisation
    passes of l_k. Returns (V, alpha, beta): the Lanczos vectors, the diagonal
    and the off-diagonal of T."""
    dim = H.shape[0]
    tol = deflation_tol(H, tau)
    v = np.zeros(dim)
    v[c] = 1.0
    V = [v]
    alpha, beta = [], []
    v_prev, b_prev = np.zeros(dim), 0.0
    for k in range(r):
        w = H @ v
        a = float(v @ w)
        alpha.append(a)
        if k == r - 1:
            break
        w = w - a * v - b_prev * v_prev
        if reorth:
            Vm = np.array(V).T
            for _ in range(2):
                w = w - Vm @ (Vm.T @ w)
        b = float(np.linalg.norm(w))
        if b <= tol:
            break
        beta.append(b)
        v_prev, b_prev, v = v, b, w / b
        V.append(v)
    return np.array(V).T, np.array(alpha), np.array(beta)

