"""GPU parity of the grouped form (Sec. 3; tb_set_groups): groups of m
consecutive atoms share the union of their cutoff spheres. The atoms are put
in compact groups by inputs.group_order, on both sides.

* c60_1920, the paper's form (orbital seeds, m = 4), every atom, mu by
  bisection: FP64 to the parity bar, FP32 forces within 1e-3 eV/A;
* block seeds on union spheres (m = 2), sampled atoms at fixed mu;
* an isolated 8-atom cell in one group of 8 with a cutoff that leaves every
  own sphere partial: the union is the whole cell and the result is full
  diagonalisation;
* errors: a group too spread for the box (TB_ECUTOFF from the device flag)
  and group sizes outside [1, 8].
"""
import os

import numpy as np
import pytest

from paper_0910_4497_amd import inputs
from oracle import exact, geometry, tb as otb
from parity_util import P, compare_rho, gpu_run, rel_inf

pytestmark = pytest.mark.gpu
NPROC = min(16, len(os.sched_getaffinity(0)))
BIG = np.array([200.0, 200.0, 200.0])


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def grouped_input(name, m):
    w = inputs.workload(name)
    perm = inputs.group_order(w.pos, w.cell, (1, 1, 1), m)
    return w, np.ascontiguousarray(w.pos[perm])


def test_parity_grouped_orbital_c60_1920(torch_cuda):
    from paper_0910_4497_amd.tb import TBContext
    m = 4
    w, pos = grouped_input("c60_1920", m)
    ora = otb.run(pos, w.cell, (1, 1, 1), P, w.r_cut, w.r, w.kT, n_electrons=w.n_electrons,
                  processes=NPROC, seeds="orbital", group=m)
    n_union = max(s["n_cluster"] for s in ora["sols"].values())
    own = max(len(geometry.cluster(i, pos, w.cell, (1, 1, 1), w.r_cut)[0]) for i in range(0, w.n_atoms, 7))
    print(f"  union spheres up to {n_union} atoms (own spheres ~{own})")
    ctx = TBContext(w.n_atoms, n_union + 8, w.r)
    ctx.set_seeds("orbital")
    ctx.set_groups(m)
    res = gpu_run(ctx, pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, n_electrons=w.n_electrons)
    assert res["stats"]["max_cluster"] == n_union
    assert abs(res["mu"] - ora["mu"]) < 1e-9
    worst, scale = compare_rho(res, ora["rho"], ora["sols"], range(w.n_atoms))
    print(f"  rho max abs err {worst:.3e} (scale {scale:.3e})")
    assert worst <= 1e-8 * scale
    ef = rel_inf(res["forces"], ora["forces"])
    print(f"  force rel err {ef:.3e}")
    assert ef <= 1e-8
    e = res["e"]
    assert abs(e[3] - ora["e_total"]) <= 1e-10 * abs(ora["e_total"])
    r32 = gpu_run(ctx, pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, n_electrons=w.n_electrons,
                  precision="fp32")
    fe = float(np.abs(r32["forces"] - ora["forces"]).max())
    print(f"  fp32 max force err {fe:.3e} eV/A")
    assert fe <= 1e-3
    # back to own spheres: the same context gives the ungrouped result
    ctx.set_groups(1)
    r1 = gpu_run(ctx, pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, n_electrons=w.n_electrons)
    assert r1["stats"]["max_cluster"] < n_union
    ctx.close()


def test_parity_grouped_block_seeds_sampled(torch_cuda):
    from paper_0910_4497_amd.tb import TBContext
    m, mu = 2, 3.5
    w, pos = grouped_input("c60_1920", m)
    rng = np.random.default_rng(123)
    S = sorted(rng.choice(w.n_atoms, 10, replace=False).tolist())
    need = otb.hop_closure(S, pos, w.cell, (1, 1, 1), P)
    ora = otb.run(pos, w.cell, (1, 1, 1), P, w.r_cut, w.r, w.kT, mu=mu, atoms=need, force_atoms=S,
                  processes=NPROC, group=m)
    ctx = TBContext(w.n_atoms, 300, w.r)
    ctx.set_groups(m)
    res = gpu_run(ctx, pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, mu=mu)
    ctx.close()
    worst, scale = compare_rho(res, ora["rho"], ora["sols"], need)
    print(f"  rho max abs err {worst:.3e} (scale {scale:.3e}) over {len(need)} targets")
    assert worst <= 1e-8 * scale
    F = np.array([ora["forces_sampled"][k] for k in S])
    err = rel_inf(res["forces"][S], F)
    print(f"  sampled force rel err {err:.3e}")
    assert err <= 1e-8


def test_grouped_exact_limit_small_cell(torch_cuda):
    from paper_0910_4497_amd.tb import TBContext
    pos, _ = inputs.cubic_diamond(1, 3.567, 0.05, 78)
    pos = pos - pos.mean(axis=0) + 100.0
    r_cut = 2.7                                   # own spheres: an atom and a few neighbours
    assert max(len(geometry.cluster(i, pos, BIG, (0, 0, 0), r_cut)[0]) for i in range(8)) < 8
    ex = exact.solve(pos, BIG, (0, 0, 0), P, 0.1, n_electrons=32.0)
    errs = {}
    for m in (1, 8):
        ctx = TBContext(8, 8, 40)
        ctx.set_seeds("orbital")
        ctx.set_groups(m)
        res = gpu_run(ctx, pos, BIG, (0, 0, 0), r_cut, 40, 0.1, n_electrons=32.0)
        ctx.close()
        errs[m] = (abs(res["mu"] - ex["mu"]), float(np.abs(res["forces"] - ex["forces"]).max()))
        print(f"  m={m}: mu err {errs[m][0]:.2e}, force err {errs[m][1]:.2e}")
    assert errs[8][0] < 1e-9 and errs[8][1] < 1e-8
    assert errs[1][1] > 1e-4


def test_grouped_errors(torch_cuda):
    import torch
    from paper_0910_4497_amd.tb import TBContext, TBError
    w = inputs.workload("c60_240")                # L/2 = 6.25 A, R_cut = 6 A: no room for a spread
    ctx = TBContext(w.n_atoms, 200, 10)
    for bad in (0, 9):
        with pytest.raises(TBError) as e:
            ctx.set_groups(bad)
        assert e.value.name == "TB_EINVAL"
    pos = torch.tensor(w.pos, dtype=torch.float64, device="cuda")
    ctx.set_groups(2)
    ctx.build_local_H(pos, w.cell, (1, 1, 1), P, w.r_cut)
    torch.cuda.synchronize()
    with pytest.raises(TBError) as e:
        ctx.stats()
    assert e.value.name == "TB_ECUTOFF"
    ctx.set_groups(1)
    ctx.build_local_H(pos, w.cell, (1, 1, 1), P, w.r_cut)
    torch.cuda.synchronize()
    assert ctx.stats()["flags"] == 0
    ctx.close()
