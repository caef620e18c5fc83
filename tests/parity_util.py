"""Helpers shared by the GPU parity tests (imported by tests only)."""
from __future__ import annotations

import numpy as np

from paper_0910_4497_amd import inputs

P = inputs.load_params()


def gpu_run(ctx, pos_np, cell, periodic, r_cut, r, kT, n_electrons=None, mu=None,
            precision="fp64", r_per_atom=None, params=None):
    """One full pass through the C-ABI; returns numpy copies of everything."""
    import torch
    dev = ctx.device
    pos = torch.tensor(np.ascontiguousarray(pos_np), dtype=torch.float64, device=dev)
    ctx.build_local_H(pos, cell, periodic, P if params is None else params, r_cut)
    rpa = None
    if r_per_atom is not None:
        rpa = torch.tensor(np.asarray(r_per_atom, dtype=np.int32), device=dev)
    mu_t, rho = ctx.krylov_rho(r, kT, mu=mu, n_electrons=n_electrons, precision=precision,
                               r_per_atom=rpa)
    e, f = ctx.energy_forces()
    torch.cuda.synchronize()
    ctx.rho_layout()
    stats = ctx.stats()
    return {"mu": float(mu_t.item()), "rho": rho[:ctx.nnz].cpu().numpy(), "row_ptr": ctx.row_ptr.cpu().numpy(),
            "col_j": ctx.col_j.cpu().numpy(), "e": e.cpu().numpy(), "forces": f.cpu().numpy(),
            "stats": stats}


def rel_inf(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rho_blocks_gpu(res, i):
    s, e = res["row_ptr"][i], res["row_ptr"][i + 1]
    return res["col_j"][s:e], res["rho"][s:e]


def compare_rho(res, ora_rho, ora_sols, atoms):
    """max |rho_gpu - rho_oracle| over the listed target atoms, and max |rho|."""
    worst, scale = 0.0, 0.0
    for i in atoms:
        cj, blk = rho_blocks_gpu(res, i)
        J = ora_sols[i]["J"]
        assert np.array_equal(cj, J), (i, cj, J)
        worst = max(worst, float(np.abs(blk - ora_rho[i]).max()))
        scale = max(scale, float(np.abs(ora_rho[i]).max()))
    return worst, scale
