"""A whole MD step captured in a HIP graph: every replay must reproduce the
eagerly launched step exactly (the kernels are deterministic), with the
program's own eager work and synchronisations between the replays."""
import numpy as np
import pytest

from paper_0910_4497_amd import inputs

pytestmark = pytest.mark.gpu
P = inputs.load_params()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replays_match_eager(torch_cuda, precision):
    torch = torch_cuda
    from paper_0910_4497_amd.md import GraphedVerlet, TBForceField, TBSettings
    w = inputs.workload("c60_240")
    pos0 = torch.tensor(w.pos, dtype=torch.float64, device="cuda:0")
    vel0 = torch.tensor(inputs.maxwell_velocities(w.n_atoms, 600.0, seed=9), dtype=torch.float64,
                        device="cuda:0")
    stream = torch.cuda.Stream()
    settings = TBSettings(cell=tuple(w.cell), periodic=(1, 1, 1), params=P, r_cluster=w.r_cut, r=w.r,
                          n_electrons=w.n_electrons, precision=precision)
    with torch.cuda.stream(stream):
        ff = TBForceField.for_geometry(pos0, settings)
        gv = GraphedVerlet(ff, pos0, vel0, dt=0.5, stream=stream, warmup=1)
    n = 4
    gv.init_state(pos0, vel0)
    ref_pos, ref_e = [], []
    for _ in range(n):
        gv.eager_step()
        stream.synchronize()
        ref_pos.append(gv.pos.clone())
        ref_e.append(gv.e.clone())
    gv.init_state(pos0, vel0)
    stream.synchronize()
    for k in range(n):
        gv.step()
        stream.synchronize()
        assert torch.equal(gv.pos, ref_pos[k]), k
        assert torch.equal(gv.e, ref_e[k]), k
        # unrelated eager work and a device-wide synchronisation between replays
        x = torch.randn(4096, device="cuda:0")
        assert torch.isfinite(x.sum())
        torch.cuda.synchronize()
    assert ff.ctx.stats()["flags"] == 0
    print(f"  {precision}: {n} replays equal to the eager steps; E_tot {float(gv.e[3]):.6f} eV")
    ff.close()


@pytest.mark.parametrize("groups", [1, 4])
def test_graph_replays_match_eager_orbital_seeds(torch_cuda, groups):
    """The same with the paper's per-orbital seeding (per-chain eigensolver)
    and, for groups = 4, the grouped form (union spheres built on the device
    inside the captured step): an isolated pair of C60 molecules."""
    torch = torch_cuda
    from paper_0910_4497_amd.md import GraphedVerlet, TBForceField, TBSettings
    rng = np.random.default_rng(13)
    mols = [inputs.c60_ideal() @ inputs.random_rotation(rng).T + np.array([10.0 * k, 0.0, 0.0]) + 100.0
            for k in range(2)]
    pos = np.concatenate(mols) + rng.normal(0, 0.03, (120, 3))
    cell = (200.0, 200.0, 200.0)
    pos = np.ascontiguousarray(pos[inputs.group_order(pos, cell, (0, 0, 0), groups)])
    pos0 = torch.tensor(pos, dtype=torch.float64, device="cuda:0")
    vel0 = torch.tensor(inputs.maxwell_velocities(120, 600.0, seed=10), dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.Stream()
    settings = TBSettings(cell=cell, periodic=(0, 0, 0), params=P, r_cluster=6.0, r=20, n_electrons=480.0,
                          precision="fp64", seeds="orbital", groups=groups)
    with torch.cuda.stream(stream):
        ff = TBForceField.for_geometry(pos0, settings)
        gv = GraphedVerlet(ff, pos0, vel0, dt=0.5, stream=stream, warmup=1)
    n = 3
    gv.init_state(pos0, vel0)
    ref = []
    for _ in range(n):
        gv.eager_step()
        stream.synchronize()
        ref.append((gv.pos.clone(), gv.e.clone()))
    gv.init_state(pos0, vel0)
    stream.synchronize()
    for k in range(n):
        gv.step()
        stream.synchronize()
        assert torch.equal(gv.pos, ref[k][0]) and torch.equal(gv.e, ref[k][1]), k
        torch.cuda.synchronize()
    assert ff.ctx.stats()["flags"] == 0
    print(f"  orbital seeds, groups {groups}: {n} replays equal to the eager steps")
    ff.close()
