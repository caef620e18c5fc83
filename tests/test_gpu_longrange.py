"""GPU parity under the long-range parameter set (hopping to 7 A,
inputs.PARAMS_LONG): hop lists of ~200 neighbours (tb_create_ex), local
Hamiltonians with a third of all atom pairs coupled, rho rows for every hop
neighbour.

* an isolated pair of C60 molecules (120 atoms, spheres of R_cut = 8 A):
  every atom, mu by bisection, FP64 to the parity bar and FP32 forces within
  1e-3 eV/A with each of the four FP32 H.V item layouts;
* c60_1920_long at fixed mu: rho blocks of sampled targets, and the forces
  on two atoms whose hop closures the oracle solves;
* a hop capacity too small for the geometry is reported (TB_ECAPACITY).
"""
import os

import numpy as np
import pytest

from paper_0910_4497_amd import inputs
from oracle import tb as otb
from parity_util import compare_rho, gpu_run, rel_inf

pytestmark = pytest.mark.gpu
NPROC = min(16, len(os.sched_getaffinity(0)))
BIG = np.array([200.0, 200.0, 200.0])
PL = inputs.load_params(inputs.PARAMS_LONG)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def c60_pair(seed=61, sep=10.0):
    rng = np.random.default_rng(seed)
    mols = []
    for k in range(2):
        R = inputs.random_rotation(rng)
        mols.append(inputs.c60_ideal() @ R.T + np.array([sep * k, 0.0, 0.0]) + 100.0)
    return np.concatenate(mols) + rng.normal(0, 0.03, (120, 3))


def test_parity_long_range_c60_pair(torch_cuda):
    from paper_0910_4497_amd.tb import TBContext
    pos = c60_pair()
    r_cut, r = 8.0, 30
    ora = otb.run(pos, BIG, (0, 0, 0), PL, r_cut, r, 0.1, n_electrons=480.0, processes=NPROC)
    n_cl = max(s["n_cluster"] for s in ora["sols"].values())
    n_hop = max(len(s["J"]) - 1 for s in ora["sols"].values())
    print(f"  spheres up to {n_cl} atoms, hop lists up to {n_hop}")
    ctx = TBContext(120, n_cl + 4, r, hop_max=n_hop + 8)
    res = gpu_run(ctx, pos, BIG, (0, 0, 0), r_cut, r, 0.1, n_electrons=480.0, params=PL)
    assert res["stats"]["max_hop"] == n_hop
    assert abs(res["mu"] - ora["mu"]) < 1e-9
    worst, scale = compare_rho(res, ora["rho"], ora["sols"], range(120))
    print(f"  rho max abs err {worst:.3e} (scale {scale:.3e})")
    assert worst <= 1e-8 * scale
    ef = rel_inf(res["forces"], ora["forces"])
    print(f"  force rel err {ef:.3e}")
    assert ef <= 1e-8
    assert abs(res["e"][3] - ora["e_total"]) <= 1e-10 * abs(ora["e_total"])
    for layout in (0, 1, 2, 3):
        ctx.set_shape("fp32", 512, 4, 1, wide=layout)
        r32 = gpu_run(ctx, pos, BIG, (0, 0, 0), r_cut, r, 0.1, n_electrons=480.0, precision="fp32", params=PL)
        fe = float(np.abs(r32["forces"] - ora["forces"]).max())
        print(f"  fp32 (H.V layout {layout}) max force err {fe:.3e} eV/A")
        assert fe <= 1e-3
    ctx.close()


def test_parity_long_range_c60_1920_sampled(torch_cuda):
    from paper_0910_4497_amd.tb import TBContext
    w = inputs.workload("c60_1920_long")
    mu = 3.0
    rng = np.random.default_rng(71)
    F_atoms = sorted(rng.choice(w.n_atoms, 2, replace=False).tolist())
    S = sorted(set(rng.choice(w.n_atoms, 8, replace=False).tolist()) | set(F_atoms))
    need = sorted(set(S) | set(otb.hop_closure(F_atoms, w.pos, w.cell, (1, 1, 1), PL)))
    ora = otb.run(w.pos, w.cell, (1, 1, 1), PL, w.r_cut, w.r, w.kT, mu=mu, atoms=need,
                  force_atoms=F_atoms, processes=NPROC)
    ctx = TBContext(w.n_atoms, 330, w.r, hop_max=w.hop_max)
    res = gpu_run(ctx, w.pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, mu=mu, params=PL)
    ctx.close()
    print(f"  max sphere {res['stats']['max_cluster']}, max hop {res['stats']['max_hop']}, "
          f"max couplings {res['stats']['max_couplings']}")
    worst, scale = compare_rho(res, ora["rho"], ora["sols"], S)
    print(f"  rho max abs err {worst:.3e} (scale {scale:.3e}) over {len(S)} targets")
    assert worst <= 1e-8 * scale
    F = np.array([ora["forces_sampled"][k] for k in F_atoms])
    err = rel_inf(res["forces"][F_atoms], F)
    print(f"  sampled force rel err {err:.3e}")
    assert err <= 1e-8


def test_long_range_hop_capacity_reported(torch_cuda):
    import torch
    from paper_0910_4497_amd.tb import TBContext, TBError
    pos = c60_pair()
    ctx = TBContext(120, 128, 10, hop_max=24)
    ctx.build_local_H(torch.tensor(pos, dtype=torch.float64, device="cuda"), BIG, (0, 0, 0), PL, 8.0)
    torch.cuda.synchronize()
    with pytest.raises(TBError) as e:
        ctx.stats()
    assert e.value.name == "TB_ECAPACITY"
    ctx.close()
