"""Per-atom projected eigensolve, global chemical potential, density matrix,
band energy, entropy, repulsion and forces.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Following the paper (Secs. 2-3):
  * per target atom i: H^(i) on the cutoff sphere, orthonormal basis Q of
    K_r(H^(i), Phi_i), T = Q^T H^(i) Q, T = Y diag(lambda) Y^T (the small
    eigenproblem the paper hands to LAPACK);
  * the density matrix of Eq. (2), rho = sum_m |m> f(eps_m) <m|, is taken in
    the Krylov space: the column block of seed i is
        rho[:, i] = Q Y f(Lambda) Y[0:4, :]^T
    and its rows on atom j give rho_{j alpha, i beta};
  * occupation f(eps) = 2 / (1 + exp((eps - mu)/kT)) (spin factor 2);
  * one global mu with sum_i sum_m f(lambda_m^(i)) w_m^(i) = N_e, where
    w_m^(i) = sum_{beta<4} Y[beta, m]^2 is the weight of Ritz pair m on the
    seed block; found by 100 bisection steps on
    [min lambda - 50 kT, max lambda + 50 kT];
  * E_band = sum_i sum_m lambda_m f_m w_m = sum_i sum_j Tr[H_ij rho_ji];
    S/k_B = sum_i sum_m w_m 2 s(f_m/2), s(q) = -q ln q - (1-q) ln(1-q);
    A = E_band - kT S/k_B;  E_rep = sum_i F(sum_j phi(r_ij));  E = A + E_rep;
  * force (Sec. 2: <F_i> = Tr[rho F_i], F_i = -dH/dR_i):
        F_k = - sum_i sum_{j in hop(i)} Tr[(dH_ij/dR_k) rho_ji] - dE_rep/dR_k;
  * virial (Sec. 5 times the pressure of a diamond cell; the pair form is the
    standard one for energies of pair vectors d_ij = R_j - R_i, minimum
    image): with g_ij the derivative of the pair's energy terms with respect
    to d_ij (the same terms the forces sum),
        W_ab = sum over ordered pairs (i, j) of (d_ij)_a (g_ij)_b,
    stress sigma = W / V and pressure P = -tr(W) / (3 V); for an isolated
    system W = -sum_k R_k (x) F_k.
"""
from __future__ import annotations

import os
import multiprocessing as mp

import numpy as np

from . import geometry, krylov, model

N_BISECT = 100


# ------------------------------------------------------------ occupation
def fermi(eps, mu, kT):
    """2/(1+exp(x)), x = (eps-mu)/kT, evaluated without overflow."""
    x = (np.asarray(eps, dtype=np.float64) - mu) / kT
    e = np.exp(-np.abs(x))
    return np.where(x > 0, 2.0 * e / (1.0 + e), 2.0 / (1.0 + e))


def entropy_per_level(eps, mu, kT):
    """2 * s(f/2) with s(q) = -q ln q - (1-q) ln(1-q).

    With q = 1/(1+e^x): s = ln(1+e^{-|x|}) + |x| e^{-|x|}/(1+e^{-|x|}), which is
    the same function (s is symmetric under q <-> 1-q) with no cancellation.
    """
    x = np.abs((np.asarray(eps, dtype=np.float64) - mu) / kT)
    e = np.exp(-x)
    return 2.0 * (np.log1p(e) + x * e / (1.0 + e))


def electron_count(mu, lams, ws, kT):
    return float(sum(np.sum(fermi(l, mu, kT) * w) for l, w in zip(lams, ws)))


def chemical_potential(lams, ws, n_electrons, kT, n_iter=N_BISECT):
    lo = min(float(np.min(l)) for l in lams) - 50.0 * kT
    hi = max(float(np.max(l)) for l in lams) + 50.0 * kT
    for _ in range(n_iter):
        mid = 0.5 * (lo + hi)
        if electron_count(mid, lams, ws, kT) < n_electrons:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


# --------------------------------------------------------- per-atom solve
def orbital_solve(H, r, route="arnoldi", reorth=True):
    """The paper's per-orbital seeding (Sec. 3, Eqs. 6-9): one scalar Krylov
    space K_r(H, e_c) per orbital c of the target atom, T_c = Q_c^T H Q_c,
    T_c = Y_c diag(lambda_c) Y_c^T. Packed so that the column-block formulas
    of the block form apply: lam and the columns of Q Y are the four chains'
    concatenated, and Y1[c', m] is the seed component Y_c[0, m] of chain c's
    Ritz pair m in row c' = c, zero in the other rows (the density-matrix
    column of orbital c uses its own chain only)."""
    lams, QYs, Y1s = [], [], []
    for c in range(4):
        if route == "arnoldi":
            Q = krylov.orbital_krylov_basis(H, r, c, reorth=reorth)
            T = Q.T @ H @ Q
            T = 0.5 * (T + T.T)
        else:
            Q, a, b = krylov.orbital_lanczos(H, r, c, reorth=reorth)
            T = np.diag(a) + np.diag(b[:len(a) - 1], 1) + np.diag(b[:len(a) - 1], -1)
        lam, Y = np.linalg.eigh(T)
        lams.append(lam)
        QYs.append(Q @ Y)
        y1 = np.zeros((4, len(lam)))
        y1[c] = Y[0]
        Y1s.append(y1)
    return np.concatenate(lams), np.concatenate(QYs, axis=1), np.concatenate(Y1s, axis=1)


def atom_solve(i, pos, cell, periodic, p, r_cut, r, full_column=False,
               route="arnoldi", reorth=True, seeds="block", group=1):
    """Krylov solve for target atom i.

    Returns dict with lam [d], w [d], J (global ids: i then hop(i) sorted),
    P = (Q Y) restricted to the rows of J, shape (4|J|, d), Y1 = Y[0:4, :],
    and with full_column also the cluster ids and Q Y on all cluster rows.
    seeds="orbital": the paper's one scalar chain per orbital (orbital_solve).
    group=m > 1: the grouped form of Sec. 3 -- the recursion runs on the union
    sphere of the m-atom group of i (geometry.group_cluster) instead of i's own.
    """
    if group > 1:
        idx, x = geometry.group_cluster(i, group, pos, cell, periodic, r_cut)
    else:
        idx, x = geometry.cluster(i, pos, cell, periodic, r_cut)
    H = krylov.cluster_hamiltonian(x, p)
    if seeds == "orbital":
        lam, QY, Y1 = orbital_solve(H, r, route, reorth)
        w = np.sum(Y1 ** 2, axis=0)
        rloc = np.linalg.norm(x, axis=1)
        j_local = np.nonzero((rloc < p["rm"]) & (np.arange(len(idx)) > 0))[0]
        j_local = j_local[np.argsort(idx[j_local])]
        J_local = np.concatenate([[0], j_local])
        rows = (4 * J_local[:, None] + np.arange(4)[None, :]).ravel()
        out = {"i": i, "lam": lam, "w": w, "J": idx[J_local], "P": QY[rows, :],
               "Y1": Y1, "n_cluster": len(idx), "dim": len(lam)}
        if full_column:
            out["cluster"] = idx
            out["QY"] = QY
        return out
    if route == "arnoldi":
        Q, _w = krylov.block_krylov_basis(H, r, reorth=reorth)
        T = Q.T @ H @ Q
        T = 0.5 * (T + T.T)
    else:
        Q, T = krylov.block_lanczos(H, r, reorth=reorth)
    lam, Y = np.linalg.eigh(T)
    w = np.sum(Y[:4, :] ** 2, axis=0)
    rloc = np.linalg.norm(x, axis=1)
    j_local = np.nonzero((rloc < p["rm"]) & (np.arange(len(idx)) > 0))[0]
    j_local = j_local[np.argsort(idx[j_local])]
    J_local = np.concatenate([[0], j_local])
    rows = (4 * J_local[:, None] + np.arange(4)[None, :]).ravel()
    QY = Q @ Y
    out = {"i": i, "lam": lam, "w": w, "J": idx[J_local], "P": QY[rows, :],
           "Y1": Y[:4, :].copy(), "n_cluster": len(idx), "dim": Q.shape[1]}
    if full_column:
        out["cluster"] = idx
        out["QY"] = QY
    return out


def rho_blocks_from(sol, mu, kT):
    """rho_{j alpha, i beta} for j in J: array (|J|, 4, 4), [p][alpha][beta]."""
    f = fermi(sol["lam"], mu, kT)
    col = (sol["P"] * f[None, :]) @ sol["Y1"].T          # (4|J|, 4)
    return col.reshape(-1, 4, 4)


def rho_column_full(sol, mu, kT):
    f = fermi(sol["lam"], mu, kT)
    return ((sol["QY"] * f[None, :]) @ sol["Y1"].T).reshape(-1, 4, 4)


# ------------------------------------------------------------ repulsion
def repulsion(pos, cell, periodic, p):
    """E_rep and its forces -dE_rep/dR (N,3)."""
    N = pos.shape[0]
    nb, dv = geometry.neighbour_lists(pos, cell, periodic, p["dm"])
    xs = np.array([np.sum(model.phi_pair(np.linalg.norm(d, axis=1), p)) if len(d) else 0.0
                   for d in dv])
    e_rep = float(np.sum(model.f_embed(xs, p)))
    dF = model.f_embed_deriv(xs, p)
    grad = np.zeros((N, 3))
    for i in range(N):
        if len(nb[i]) == 0:
            continue
        rr = np.linalg.norm(dv[i], axis=1)
        g = (dF[i] * model.phi_pair_deriv(rr, p) / rr)[:, None] * dv[i]   # d/d(d_ij)
        grad[nb[i]] += g
        grad[i] -= g.sum(axis=0)
    return e_rep, -grad


def repulsion_virial(pos, cell, periodic, p):
    """W_rep = sum over ordered pairs (i, j) of d_ij (x) dF(x_i)/d d_ij, with
    dF(x_i)/d d_ij = F'(x_i) phi'(r_ij) d_ij / r_ij (each unordered pair
    appears twice, once for each embedding term)."""
    nb, dv = geometry.neighbour_lists(pos, cell, periodic, p["dm"])
    xs = np.array([np.sum(model.phi_pair(np.linalg.norm(d, axis=1), p)) if len(d) else 0.0
                   for d in dv])
    dF = model.f_embed_deriv(xs, p)
    W = np.zeros((3, 3))
    for i in range(pos.shape[0]):
        if len(nb[i]) == 0:
            continue
        rr = np.linalg.norm(dv[i], axis=1)
        g = (dF[i] * model.phi_pair_deriv(rr, p) / rr)[:, None] * dv[i]
        W += dv[i].T @ g
    return W


def pressure(virial, cell):
    """P = -tr(W) / (3 V) in eV/A^3 for an orthorhombic cell (lengths)."""
    V = float(np.prod(np.asarray(cell, dtype=np.float64)))
    return -float(np.trace(virial)) / (3.0 * V)


def _neighbours_of(k, pos, cell, periodic, cutoff):
    d = geometry.displacements_from(k, pos, cell, periodic)
    r = np.linalg.norm(d, axis=1)
    sel = np.nonzero(r < cutoff)[0]
    sel = sel[sel != k]
    return sel, d[sel]


def repulsion_forces_subset(pos, cell, periodic, p, atoms):
    """-dE_rep/dR_k for the listed atoms only: the same sum as repulsion(),
    F_k = sum_j (F'(x_k) + F'(x_j)) phi'(r_kj) d_kj / r_kj, evaluated from the
    neighbourhoods of k and of its neighbours."""
    xcache = {}

    def x_of(a):
        if a not in xcache:
            _, d = _neighbours_of(a, pos, cell, periodic, p["dm"])
            xcache[a] = float(np.sum(model.phi_pair(np.linalg.norm(d, axis=1), p))) if len(d) else 0.0
        return xcache[a]

    out = {}
    for k in atoms:
        nb, d = _neighbours_of(k, pos, cell, periodic, p["dm"])
        f = np.zeros(3)
        dFk = model.f_embed_deriv(x_of(k), p)
        for j, dj in zip(nb, d):
            r = np.linalg.norm(dj)
            f += (dFk + model.f_embed_deriv(x_of(int(j)), p)) * model.phi_pair_deriv(r, p) / r * dj
        out[int(k)] = f
    return out


def hop_closure(atoms, pos, cell, periodic, p):
    """atoms together with their hopping neighbours (the seeds their forces need)."""
    need = set(int(a) for a in atoms)
    for k in atoms:
        nb, _ = _neighbours_of(int(k), pos, cell, periodic, p["rm"])
        need.update(int(j) for j in nb)
    return sorted(need)


# ---------------------------------------------------------- parallel map
_G = {}


def _worker(i):
    g = _G
    return atom_solve(i, g["pos"], g["cell"], g["periodic"], g["p"], g["r_cut"],
                      int(g["r_of"](i)), full_column=g["full_column"],
                      route=g["route"], reorth=g["reorth"], seeds=g["seeds"], group=g["group"])


def _limit_blas():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def solve_atoms(atoms, pos, cell, periodic, p, r_cut, r, r_per_atom=None,
                full_column=False, route="arnoldi", reorth=True, processes=None, seeds="block",
                group=1):
    """atom_solve over a list of atoms, in worker processes (one BLAS thread each)."""
    r_of = (lambda i: r_per_atom[i]) if r_per_atom is not None else (lambda i: r)
    _G.update(pos=pos, cell=cell, periodic=periodic, p=p, r_cut=r_cut, r_of=r_of,
              full_column=full_column, route=route, reorth=reorth, seeds=seeds, group=group)
    atoms = list(atoms)
    if processes is None:
        processes = len(os.sched_getaffinity(0))
    processes = max(1, min(processes, len(atoms)))
    if processes == 1 or len(atoms) < 4:
        return [_worker(i) for i in atoms]
    ctx = mp.get_context("fork")
    with ctx.Pool(processes, initializer=_limit_blas) as pool:
        return pool.map(_worker, atoms, chunksize=max(1, len(atoms) // (4 * processes)))


# --------------------------------------------------------------- driver
def run(pos, cell, periodic, p, r_cut, r, kT, n_electrons=None, mu=None,
        r_per_atom=None, atoms=None, force_atoms=None, full_column=False,
        route="arnoldi", reorth=True, processes=None, seeds="block", group=1):
    """The whole path for one geometry.

    atoms=None solves every atom; mu must then be None (bisection on
    n_electrons) or given.  With a subset of atoms, mu must be given, and
    forces are returned for force_atoms (each needs itself and hop() solved).
    seeds: "block" (four-orbital seed block) or "orbital" (one scalar chain
    per orbital, Eqs. 6-9).  group: atoms per group of the grouped form
    (Sec. 3; union spheres, geometry.group_cluster), 1 = each atom's own sphere.
    """
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[0]
    all_atoms = atoms is None
    atoms = list(range(N)) if all_atoms else list(atoms)
    sols = solve_atoms(atoms, pos, cell, periodic, p, r_cut, r, r_per_atom,
                       full_column, route, reorth, processes, seeds, group)
    by_atom = {s["i"]: s for s in sols}
    if mu is None:
        if not all_atoms:
            raise ValueError("chemical potential by bisection needs every atom")
        mu = chemical_potential([s["lam"] for s in sols], [s["w"] for s in sols],
                                n_electrons, kT)
    rho = {s["i"]: rho_blocks_from(s, mu, kT) for s in sols}
    e_band = float(sum(np.sum(s["lam"] * fermi(s["lam"], mu, kT) * s["w"]) for s in sols))
    ent = float(sum(np.sum(s["w"] * entropy_per_level(s["lam"], mu, kT)) for s in sols))
    out = {"mu": mu, "sols": by_atom, "rho": rho, "e_band": e_band,
           "entropy": ent, "free_band": e_band - kT * ent}
    # trace identity check quantity: sum_i sum_j Tr[H_ij rho_ji]
    tr = 0.0
    for s in sols:
        i = s["i"]
        d = geometry.min_image(pos[s["J"][1:]] - pos[i], cell, periodic)
        blocks = np.concatenate([model.onsite_block(p)[None], model.sk_blocks(d, p)], axis=0)
        tr += float(np.einsum("pba,pab->", blocks, rho[i]))
    out["trace_HRho"] = tr
    if full_column:
        out["rho_full"] = {s["i"]: rho_column_full(s, mu, kT) for s in sols}
    # forces
    if all_atoms:
        e_rep, f_rep = repulsion(pos, cell, periodic, p)
        grad = np.zeros((N, 3))
        w_band = np.zeros((3, 3))
        for s in sols:
            i = s["i"]
            J = s["J"][1:]
            if len(J) == 0:
                continue
            d = geometry.min_image(pos[J] - pos[i], cell, periodic)
            dH = model.sk_blocks_grad(d, p)                  # (|J|, 3, 4, 4) [c][beta][alpha]
            g = np.einsum("pcba,pab->pc", dH, rho[i][1:])   # d Tr[H_ij rho_ji] / d d_c
            grad[J] += g
            grad[i] -= g.sum(axis=0)
            w_band += d.T @ g                                 # sum_p d_p (x) g_p
        forces = -grad + f_rep
        virial = w_band + repulsion_virial(pos, cell, periodic, p)
        out.update(e_rep=e_rep, forces=forces, virial=virial, virial_band=w_band,
                   e_total=e_band - kT * ent + e_rep)
    elif force_atoms is not None:
        need = hop_closure(force_atoms, pos, cell, periodic, p)
        missing = set(need) - set(by_atom)
        if missing:
            raise ValueError(f"forces on {list(force_atoms)} need solves of {sorted(missing)}")
        f_rep = repulsion_forces_subset(pos, cell, periodic, p, force_atoms)
        sampled = {}
        for k in force_atoms:
            k = int(k)
            f = f_rep[k].copy()
            sk = by_atom[k]
            for row, j in enumerate(sk["J"][1:], start=1):
                j = int(j)
                d = geometry.min_image(pos[j] - pos[k], cell, periodic)
                g_kj = np.einsum("cba,ab->c", model.sk_blocks_grad(d, p), rho[k][row])
                sj = by_atom[j]
                rowj = int(np.nonzero(sj["J"] == k)[0][0])
                g_jk = np.einsum("cba,ab->c", model.sk_blocks_grad(-d, p), rho[j][rowj])
                f += g_kj - g_jk            # F_k = -(grad_k): pair (k,j) gives -g_kj, pair (j,k) +g_jk
            sampled[k] = f
        out["forces_sampled"] = sampled
    return out
