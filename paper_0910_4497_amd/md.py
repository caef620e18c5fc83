"""Energy/force evaluation as a PyTorch autograd Function, and velocity-Verlet
molecular dynamics on top of it (argument marshalling only: every step of the
evaluation runs in libtbkrylov's kernels).

Sec. 2: the force on an atom is the trace of the density matrix with the
derivative of the Hamiltonian, plus the repulsive pair term. TBEnergy returns
the total energy A + E_rep (A = E_band - T S, the Mermin free energy whose
exact-limit gradient the trace formula gives) and its backward hands back
-F * grad_out. At finite Krylov order or cutoff the local density matrix is
not variational, so -F is the method's force, not the exact derivative of the
returned energy; the gap shrinks as r and the cutoff grow.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import inputs
from .tb import TBContext

PROBE_CLUSTER_CAP = 560        # FP64 Krylov kernel: two 4n x 4 blocks in 160 KB of LDS


@dataclass
class TBSettings:
    """What one evaluation needs besides the positions."""
    cell: tuple
    periodic: tuple
    params: dict
    r_cluster: float
    r: int
    kT: float = 0.1
    n_electrons: float | None = None      # None: keep mu fixed at `mu`
    mu: float | None = None
    precision: str = "fp64"
    r_per_atom: torch.Tensor | None = None
    seeds: str = "block"                  # or "orbital": one scalar chain per orbital
    groups: int = 1                       # grouped form: atoms per union sphere (index blocks)
    hop_max: int = 24                     # hop-list capacity (neighbours within max(rm, dm))


class TBForceField:
    """One library context bound to fixed settings: pos -> (e[4], forces)."""

    def __init__(self, n_atoms: int, n_cluster_max: int, settings: TBSettings, device: int = 0):
        self.s = settings
        r_max = settings.r if settings.r_per_atom is None else max(settings.r, int(settings.r_per_atom.max()))
        self.ctx = TBContext(n_atoms, n_cluster_max, r_max, device=device, hop_max=settings.hop_max)
        self.ctx.set_seeds(settings.seeds)
        self.ctx.set_groups(settings.groups)
        self.mu = None

    @classmethod
    def from_context(cls, ctx: TBContext, settings: TBSettings) -> "TBForceField":
        """Wraps an existing context (its stream, capacities, buffers, and its own seeds
        and groups settings; those fields of `settings` are not applied)."""
        ff = cls.__new__(cls)
        ff.s, ff.ctx, ff.mu = settings, ctx, None
        return ff

    @classmethod
    def for_geometry(cls, pos: torch.Tensor, settings: TBSettings, margin: int = 24) -> "TBForceField":
        """Sizes the sphere capacity from the geometry itself (plus a margin for motion)."""
        s = settings
        cap = PROBE_CLUSTER_CAP
        probe = TBContext(pos.shape[0], cap, 1, device=pos.device.index or 0, hop_max=s.hop_max)
        probe.set_groups(s.groups)
        sizes = probe.build_local_H(pos, s.cell, s.periodic, s.params, s.r_cluster, want_sizes=True)
        n_max = int(sizes.max().item())
        probe.close()
        if n_max >= cap:
            raise ValueError(f"a cutoff sphere holds {cap} or more atoms; the Krylov kernel keeps two "
                             f"basis blocks of the sphere in LDS and supports fewer")
        return cls(pos.shape[0], min(cap, n_max + margin), s, device=pos.device.index or 0)

    def solve(self, pos: torch.Tensor):
        """Lists, local couplings and the density matrix at pos (no energies)."""
        s = self.s
        self.ctx.build_local_H(pos, s.cell, s.periodic, s.params, s.r_cluster)
        self.mu, _ = self.ctx.krylov_rho(s.r, s.kT, mu=s.mu, n_electrons=s.n_electrons,
                                         precision=s.precision, r_per_atom=s.r_per_atom)

    def __call__(self, pos: torch.Tensor):
        self.solve(pos)
        return self.ctx.energy_forces()

    def virial(self) -> torch.Tensor:
        """W [3][3] (eV) of the last evaluation (tb_virial)."""
        return self.ctx.virial()

    def pressure(self) -> torch.Tensor:
        """P = -tr(W) / (3 V) in eV/A^3 of the last evaluation (orthorhombic cell)."""
        cell = np.asarray(self.s.cell, dtype=np.float64)
        V = float(np.prod(np.diag(cell) if cell.ndim == 2 else cell))
        return -torch.trace(self.ctx.virial()) / (3.0 * V)

    def close(self):
        self.ctx.close()


class TBEnergy(torch.autograd.Function):
    """E_tot = E_band - T S + E_rep as a 0-d tensor.

    forward runs the solve and the energy sums only (no force contraction);
    backward launches the library's force kernel (tb_energy_backward: the
    contraction Tr[rho dH/dR] through the Slater-Koster radial derivatives plus
    the repulsive term, scaled by grad_out in the kernel) on the density matrix
    of this forward. If the context has solved another geometry since, the
    forward's solve is repeated first."""

    @staticmethod
    def forward(ctx, pos: torch.Tensor, ff: TBForceField):
        p = pos.detach().contiguous()
        ff.solve(p)
        e = ff.ctx.energy()
        ctx.ff = ff
        ctx.generation = ff.ctx.generation
        ctx.save_for_backward(p)
        return e[3].clone()

    @staticmethod
    def backward(ctx, grad_out):
        (p,) = ctx.saved_tensors
        ff = ctx.ff
        if ff.ctx.generation != ctx.generation:
            ff.solve(p)
        g = grad_out.detach().to(dtype=torch.float64).reshape(1)
        return ff.ctx.energy_backward(g), None


def velocity_verlet(ff: TBForceField, pos: torch.Tensor, vel: torch.Tensor, dt: float, steps: int,
                    mass: float = inputs.MASS_C, record_energy: bool = False):
    """NVE velocity Verlet (positions in A, velocities in A/fs, dt in fs).
    Positions are wrapped into the periodic cell on every step. Returns
    (pos, vel, energies) where energies is a [steps + 1][3] device tensor of
    (E_pot, E_kin, E_pot + E_kin) when record_energy is set, else None."""
    cell = torch.tensor(np.diag(np.asarray(ff.s.cell, dtype=np.float64)) if np.ndim(ff.s.cell) == 2
                        else np.asarray(ff.s.cell, dtype=np.float64), dtype=torch.float64, device=pos.device)
    per = torch.tensor([bool(x) for x in ff.s.periodic], device=pos.device)
    acc_unit = inputs.ACC_UNIT / mass
    ke_unit = 0.5 * mass / inputs.ACC_UNIT          # amu A^2/fs^2 -> eV
    e, f = ff(pos)
    acc = f * acc_unit
    rec = torch.empty((steps + 1, 3), dtype=torch.float64, device=pos.device) if record_energy else None

    def log(k, e):
        if rec is not None:
            ke = ke_unit * (vel * vel).sum()
            rec[k, 0] = e[3]
            rec[k, 1] = ke
            rec[k, 2] = e[3] + ke
    log(0, e)
    for k in range(steps):
        pos = pos + vel * dt + 0.5 * acc * dt * dt
        pos = torch.where(per, torch.remainder(pos, cell), pos)
        e, f = ff(pos)
        a_new = f * acc_unit
        vel = vel + 0.5 * (acc + a_new) * dt
        acc = a_new
        log(k + 1, e)
    return pos, vel, rec


EV_A3_GPA = 160.21766208      # 1 eV/A^3 in GPa


def npt_berendsen(evaluate, pos: torch.Tensor, vel: torch.Tensor, cell: torch.Tensor, dt: float,
                  steps: int, T0: float, P0_GPa: float, tau_T: float, tau_P: float,
                  compressibility: float, mass: float = inputs.MASS_C, periodic=(True, True, True)):
    """NPT molecular dynamics: velocity Verlet with a Berendsen thermostat and
    an isotropic Berendsen barostat (the compression runs of Sec. 4 need a
    pressure control; the paper does not say which, so a generic weak-coupling
    scheme is used).

    evaluate(pos, cell) -> (E_tot, forces [N][3], virial [3][3]) at the given
    positions and orthorhombic cell lengths (tensors on pos.device).
    Per step: half kick, drift, wrap, evaluate, half kick; then
      T = 2 K / (3N - 3) k_B,  velocities *= sqrt(1 + dt/tau_T (T0/T - 1)),
      P = (2 K / 3 - tr(W) / 3) / V,  scale = (1 - compressibility dt/tau_P (P0 - P))^(1/3),
      positions and cell *= scale
    (units: A, fs, eV, K; compressibility in 1/GPa, P in GPa). The forces are
    kept through the cell scaling (weak coupling). Returns (pos, vel, cell,
    record [steps][4] of E_tot, T, P in GPa, V)."""
    N = pos.shape[0]
    acc_unit = inputs.ACC_UNIT / mass
    ke_unit = 0.5 * mass / inputs.ACC_UNIT
    per = torch.tensor([bool(x) for x in periodic], device=pos.device)
    pos, vel, cell = pos.clone(), vel.clone(), cell.clone()
    e, f, W = evaluate(pos, cell)
    acc = f * acc_unit
    rec = torch.empty((steps, 4), dtype=torch.float64, device=pos.device)
    for k in range(steps):
        vel = vel + 0.5 * dt * acc
        pos = pos + dt * vel
        pos = torch.where(per, torch.remainder(pos, cell), pos)
        e, f, W = evaluate(pos, cell)
        acc = f * acc_unit
        vel = vel + 0.5 * dt * acc
        ke = ke_unit * (vel * vel).sum()
        T = 2.0 * ke / ((3 * N - 3) * inputs.K_B)
        vel = vel * torch.sqrt(1.0 + dt / tau_T * (T0 / T - 1.0))
        V = torch.prod(cell)
        P = (2.0 * ke / 3.0 - torch.trace(W) / 3.0) / V * EV_A3_GPA
        scale = (1.0 - compressibility * dt / tau_P * (P0_GPa - P)) ** (1.0 / 3.0)
        pos = pos * scale
        cell = cell * scale
        rec[k, 0] = e
        rec[k, 1] = T
        rec[k, 2] = P
        rec[k, 3] = V
    return pos, vel, cell, rec


def library_evaluator(ff: TBForceField):
    """evaluate(pos, cell) for npt_berendsen through the library (the cell
    lengths are read to the host for the list build)."""
    def evaluate(pos, cell):
        ff.s.cell = tuple(float(x) for x in cell.tolist())
        e, f = ff(pos)
        return e[3], f, ff.ctx.virial()
    return evaluate


class GraphedVerlet:
    """Velocity-Verlet MD with one whole step (position update, lists, Krylov
    solve, eigensolve, chemical potential, density matrix, forces, velocity
    update) captured in a HIP graph and replayed per step.

    The force field's context must enqueue on `stream` (a non-default stream
    of default priority): the library then launches into the capture. State
    lives in static device buffers (pos, vel, acc, e, forces) updated in place.

    fixed_start: every replay advances the state set by init_state() by one
    step instead of the previous replay's state (a throughput measurement on
    starts whose trajectory leaves the model's valid range; all work of the
    step is still done).
    """

    def __init__(self, ff: TBForceField, pos: torch.Tensor, vel: torch.Tensor, dt: float,
                 stream: torch.cuda.Stream, mass: float = inputs.MASS_C, warmup: int = 2,
                 fixed_start: bool = False):
        self.ff, self.dt, self.stream, self.fixed_start = ff, dt, stream, fixed_start
        s = ff.s
        cell = np.asarray(s.cell, dtype=np.float64)
        cell = np.diag(cell) if cell.ndim == 2 else cell
        with torch.cuda.stream(stream):
            self.L = torch.tensor(cell, dtype=torch.float64, device=pos.device)
            self.per = torch.tensor([bool(x) for x in s.periodic], device=pos.device)
            self.pos = pos.clone()
            self.vel = vel.clone()
            self.e = torch.empty(4, dtype=torch.float64, device=pos.device)
            self.f = torch.empty_like(self.pos)
            self.acc_unit = inputs.ACC_UNIT / mass
            self._forces()
            self.acc = self.f * self.acc_unit
            self.start = (self.pos.clone(), self.vel.clone(), self.acc.clone())
            for _ in range(warmup):
                self._step()
        stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=stream):
            self._step()
        stream.synchronize()

    def _forces(self):
        s = self.ff.s
        ctx = self.ff.ctx
        ctx.build_local_H(self.pos, s.cell, s.periodic, s.params, s.r_cluster)
        ctx.krylov_rho(s.r, s.kT, mu=s.mu, n_electrons=s.n_electrons, precision=s.precision,
                       r_per_atom=s.r_per_atom)
        ctx.energy_forces(forces=self.f, e_out=self.e)

    def _step(self):
        dt = self.dt
        if self.fixed_start:
            self.pos.copy_(self.start[0])
            self.vel.copy_(self.start[1])
            self.acc.copy_(self.start[2])
        self.pos.add_(self.vel * dt + 0.5 * self.acc * dt * dt)
        self.pos.copy_(torch.where(self.per, torch.remainder(self.pos, self.L), self.pos))
        self._forces()
        a_new = self.f * self.acc_unit
        self.vel.add_(0.5 * (self.acc + a_new) * dt)
        self.acc.copy_(a_new)

    def init_state(self, pos: torch.Tensor, vel: torch.Tensor):
        """Set positions and velocities; forces and accelerations are evaluated
        eagerly on the context's stream."""
        with torch.cuda.stream(self.stream):
            self.pos.copy_(pos)
            self.vel.copy_(vel)
            self._forces()
            self.acc.copy_(self.f * self.acc_unit)
            for buf, src in zip(self.start, (self.pos, self.vel, self.acc)):
                buf.copy_(src)

    def eager_step(self):
        """The same step as the graph, launched eagerly (reference for tests)."""
        with torch.cuda.stream(self.stream):
            self._step()

    def step(self):
        """One MD step: a replay of the captured graph (asynchronous)."""
        self.graph.replay()
