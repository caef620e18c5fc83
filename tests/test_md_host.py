"""Host logic of the NPT integrator (no GPU): with an evaluator that returns
no forces and no virial, one step must reproduce the Berendsen formulas by
hand: drift, thermostat factor, kinetic pressure and the cell scaling."""
import numpy as np
import torch

from paper_0910_4497_amd import inputs
from paper_0910_4497_amd.md import EV_A3_GPA, npt_berendsen


def test_npt_one_step_by_hand():
    N = 64
    rng = np.random.default_rng(3)
    L = 20.0
    pos0 = torch.tensor(rng.uniform(0, L, (N, 3)))
    vel0 = torch.tensor(inputs.maxwell_velocities(N, 600.0, seed=4))
    cell0 = torch.tensor([L, L, L], dtype=torch.float64)

    def evaluate(pos, cell):
        return torch.tensor(0.0, dtype=torch.float64), torch.zeros_like(pos), torch.zeros((3, 3), dtype=torch.float64)

    dt, T0, tau_T, tau_P, beta, P0 = 0.5, 300.0, 10.0, 50.0, 0.01, 1.0
    pos, vel, cell, rec = npt_berendsen(evaluate, pos0, vel0, cell0, dt, 1, T0, P0, tau_T, tau_P, beta)
    ke = 0.5 * inputs.MASS_C / inputs.ACC_UNIT * float((vel0 ** 2).sum())
    T = 2 * ke / ((3 * N - 3) * inputs.K_B)
    assert abs(T - 600.0) < 1e-9                      # the generator's exact rescale
    lam = np.sqrt(1 + dt / tau_T * (T0 / T - 1))
    P = (2 * ke / 3) / L ** 3 * EV_A3_GPA
    mu = (1 - beta * dt / tau_P * (P0 - P)) ** (1 / 3)
    assert abs(float(rec[0, 1]) - T) < 1e-9 and abs(float(rec[0, 2]) - P) < 1e-12
    assert torch.allclose(vel, vel0 * lam, rtol=1e-14, atol=0)
    assert torch.allclose(cell, cell0 * mu, rtol=1e-14, atol=0)
    drift = torch.remainder(pos0 + dt * vel0, cell0) * mu
    assert torch.allclose(pos, drift, rtol=1e-13, atol=1e-12)
