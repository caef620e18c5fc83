"""NPT molecular dynamics through the library (velocity Verlet, Berendsen
thermostat and isotropic barostat driven by the virial pressure) on the
4 x 4 x 4 perfect diamond cell stretched to a = 3.60 A (about -17 GPa):

* three steps driven by the library equal the same integrator driven by the
  FP64 oracle (positions, velocities, cell) to 1e-9;
* 200 steps toward P0 = 0 at 300 K: the cell shrinks and the pressure
  relaxes toward zero; the record is printed.
"""
import os

import numpy as np
import pytest

from paper_0910_4497_amd import inputs
from oracle import tb as otb

pytestmark = pytest.mark.gpu
P = inputs.load_params()
NPROC = min(16, len(os.sched_getaffinity(0)))
ARGS = dict(dt=0.5, T0=300.0, P0_GPa=0.0, tau_T=20.0, tau_P=100.0, compressibility=1.0 / 450.0)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def start(torch, device):
    pos, L = inputs.cubic_diamond(4, 3.60)
    vel = inputs.maxwell_velocities(len(pos), 300.0, seed=61)
    t = lambda x: torch.tensor(np.asarray(x, dtype=np.float64), device=device)
    return t(pos), t(vel), t(L)


def make_ff(torch, pos, cell):
    from paper_0910_4497_amd.md import TBForceField, TBSettings
    s = TBSettings(cell=tuple(cell.tolist()), periodic=(1, 1, 1), params=P, r_cluster=6.0, r=30,
                   n_electrons=4.0 * pos.shape[0])
    return TBForceField(pos.shape[0], 200, s)


def test_npt_library_equals_oracle(torch_cuda):
    torch = torch_cuda
    from paper_0910_4497_amd.md import library_evaluator, npt_berendsen
    pos, vel, cell = start(torch, "cuda:0")
    ff = make_ff(torch, pos, cell)
    g = npt_berendsen(library_evaluator(ff), pos, vel, cell, steps=3, **ARGS)
    ff.close()

    def ora_eval(p, c):
        o = otb.run(p.numpy(), c.numpy(), (1, 1, 1), P, 6.0, 30, 0.1, n_electrons=4.0 * p.shape[0],
                    processes=NPROC)
        return (torch.tensor(o["e_total"], dtype=torch.float64), torch.tensor(o["forces"]),
                torch.tensor(o["virial"]))

    pc, vc, cc = start(torch, "cpu")
    o = npt_berendsen(ora_eval, pc, vc, cc, steps=3, **ARGS)
    for name, a, b in (("pos", g[0], o[0]), ("vel", g[1], o[1]), ("cell", g[2], o[2]), ("record", g[3], o[3])):
        err = float((a.cpu() - b).abs().max() / b.abs().max())
        print(f"  {name}: rel err {err:.2e}")
        assert err <= 1e-9, name


def test_npt_relaxes_stretched_diamond(torch_cuda):
    torch = torch_cuda
    from paper_0910_4497_amd.md import library_evaluator, npt_berendsen
    pos, vel, cell = start(torch, "cuda:0")
    ff = make_ff(torch, pos, cell)
    _, _, cell_end, rec = npt_berendsen(library_evaluator(ff), pos, vel, cell, steps=200, **ARGS)
    st = ff.ctx.stats()
    ff.close()
    rec = rec.cpu().numpy()
    a_end = float(cell_end[0]) / 4
    for k in (0, 49, 99, 149, 199):
        print(f"  step {k + 1}: T {rec[k, 1]:7.1f} K, P {rec[k, 2]:8.3f} GPa, a {np.cbrt(rec[k, 3]) / 4:.4f} A")
    assert st["flags"] == 0
    assert a_end < 3.60 and abs(rec[-1, 2]) < 0.5 * abs(rec[0, 2])
