"""GPU parity: the HIP path through the C-ABI against the CPU FP64 oracle.

Bar (FP64 mode): normwise relative error <= 1e-8 for rho blocks and forces,
<= 1e-10 relative for the energies; mu to 1e-9 eV. FP32 mode: force error
<= 1e-3 eV/A (max-abs over all components), errors reported. BF16-operand
mode: errors reported, bounded by the BF16 perturbation (bf16_check); the
1e-3 eV/A bar is checked as an expected failure.
"""
import os

import numpy as np
import pytest

from paper_0910_4497_amd import inputs
from oracle import exact, tb as otb
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


def make_ctx(n_atoms, n_cluster, r_max):
    from paper_0910_4497_amd.tb import TBContext
    return TBContext(n_atoms, n_cluster, r_max)


def check_against_oracle(res, ora, atoms, tol_rho=1e-8, tol_f=1e-8, tol_e=1e-10):
    worst, scale = compare_rho(res, ora["rho"], ora["sols"], atoms)
    print(f"  rho max abs err {worst:.3e} (scale {scale:.3e})")
    assert worst <= tol_rho * scale
    ef = rel_inf(res["forces"], ora["forces"])
    print(f"  force rel err {ef:.3e}; mu gpu {res['mu']:.15f} oracle {ora['mu']:.15f}")
    assert ef <= tol_f
    e = res["e"]
    assert abs(e[0] - ora["e_band"]) <= tol_e * abs(ora["e_band"])
    assert abs(e[2] - ora["e_rep"]) <= tol_e * max(1.0, abs(ora["e_rep"]))
    assert abs(e[3] - ora["e_total"]) <= tol_e * abs(ora["e_total"])


def test_single_atom(torch_cuda):
    ctx = make_ctx(1, 4, 4)
    pos = np.zeros((1, 3))
    res = gpu_run(ctx, pos, BIG, (0, 0, 0), 3.0, 3, 0.1, n_electrons=4.0)
    assert abs(res["mu"] - (P["eps_p"] - 0.1 * np.log(2.0))) < 1e-12
    assert abs(np.trace(res["rho"][0]) - 4.0) < 1e-12
    assert res["stats"]["early_stop"] == 1


def test_s_only_chain_deflation(torch_cuda):
    p = dict(P)
    p["v_sps"] = p["v_pps"] = p["v_ppp"] = 0.0
    pos = inputs.chain_positions(15, 1.45)
    ctx = make_ctx(15, 16, 8)
    res = gpu_run(ctx, pos, BIG, (0, 0, 0), 9.0, 6, 0.1, n_electrons=60.0, params=p)
    ora = otb.run(pos, BIG, (0, 0, 0), p, 9.0, 6, 0.1, n_electrons=60.0, processes=1)
    assert res["stats"]["deflated"] >= 3 * 15
    check_against_oracle(res, ora, range(15))


@pytest.mark.parametrize("r", [3, 4, 5, 7, 8])
def test_exactly_degenerate_levels(torch_cuda, r):
    """s-only chain: the three p levels of every atom are exactly degenerate
    (and so are the deflated slots), so the projected matrix has clusters
    whose computed eigenvalue can equal diagonal entries of the tridiagonal
    exactly; the cluster eigenvectors must still be orthogonal (rho and mu to
    the parity bar at several Krylov orders)."""
    p = dict(P)
    p["v_sps"] = p["v_pps"] = p["v_ppp"] = 0.0
    pos = inputs.chain_positions(15, 1.45)
    ctx = make_ctx(15, 16, 8)
    res = gpu_run(ctx, pos, BIG, (0, 0, 0), 9.0, r, 0.1, n_electrons=60.0, params=p)
    ora = otb.run(pos, BIG, (0, 0, 0), p, 9.0, r, 0.1, n_electrons=60.0, processes=1)
    assert abs(res["mu"] - ora["mu"]) < 1e-9
    check_against_oracle(res, ora, range(15))


def test_isolated_c60_exact_limit(torch_cuda):
    rng = np.random.default_rng(21)
    mol = inputs.c60_ideal() + rng.normal(0, 0.04, (60, 3))
    ctx = make_ctx(60, 64, 72)
    res = gpu_run(ctx, mol, BIG, (0, 0, 0), 8.0, 70, 0.1, n_electrons=240.0)
    ex = exact.solve(mol, BIG, (0, 0, 0), P, 0.1, n_electrons=240.0)
    assert abs(res["mu"] - ex["mu"]) < 1e-9
    assert rel_inf(res["forces"], ex["forces"]) < 1e-8
    assert abs(res["e"][3] - ex["e_total"]) < 1e-10 * abs(ex["e_total"])
    rho4 = ex["rho"].reshape(60, 4, 60, 4)
    for i in range(60):
        s, e = res["row_ptr"][i], res["row_ptr"][i + 1]
        for p_, j in enumerate(res["col_j"][s:e]):
            assert np.abs(res["rho"][s + p_] - rho4[j, :, i, :]).max() < 1e-9


@pytest.fixture(scope="module")
def c60_240_oracle():
    w = inputs.workload("c60_240")
    ora = otb.run(w.pos, w.cell, (1, 1, 1), P, w.r_cut, w.r, w.kT, n_electrons=w.n_electrons,
                  processes=NPROC)
    return w, ora


def test_parity_c60_240_fp64(torch_cuda, c60_240_oracle):
    w, ora = c60_240_oracle
    ctx = make_ctx(w.n_atoms, 128, w.r)
    res = gpu_run(ctx, w.pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, n_electrons=w.n_electrons)
    assert abs(res["mu"] - ora["mu"]) < 1e-9
    check_against_oracle(res, ora, range(w.n_atoms))
    # bitwise reproducible
    res2 = gpu_run(ctx, w.pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, n_electrons=w.n_electrons)
    assert np.array_equal(res["forces"], res2["forces"]) and np.array_equal(res["e"], res2["e"])


def test_parity_c60_240_fp32(torch_cuda, c60_240_oracle):
    w, ora = c60_240_oracle
    ctx = make_ctx(w.n_atoms, 128, w.r)
    res = gpu_run(ctx, w.pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, n_electrons=w.n_electrons,
                  precision="fp32")
    fe = float(np.abs(res["forces"] - ora["forces"]).max())
    ee = abs(res["e"][3] - ora["e_total"]) / w.n_atoms
    print(f"  fp32: max force err {fe:.3e} eV/A, energy err {ee:.3e} eV/atom")
    assert fe <= 1e-3
    assert ee <= 1e-4


def bf16_check(res, ora, n_atoms, label, w):
    """Errors of a BF16-operand run against the FP64 oracle, reported, and
    bounded. Rounding both operands of every H.V product to 8 significand bits
    perturbs the local Hamiltonian seen by the recursion by a relative 2^-8 at
    most, so each Ritz value moves by at most 2^-8 of the local spectral
    width (~40 eV): with 4 electrons per atom the energy error per atom is at
    most 4 * 2^-8 * 40 eV. Force errors have no useful worst case (eigenvector
    perturbations scale with 1/kT); their typical size is bounded instead:
    rms error <= 2^-6 of the rms band force (the perturbation acts on the band
    part only -- the net force is small where band and pair forces cancel --;
    2^-8 for the operands, times the four terms of a pair force: rho_ji from
    two seeds, each through Ritz values and vectors). The max error is only
    reported."""
    d = res["forces"] - ora["forces"]
    fe = float(np.abs(d).max())
    frms = float(np.sqrt(np.mean(d ** 2)))
    band = ora["forces"] - otb.repulsion(w.pos, w.cell, (1, 1, 1), P)[1]
    f_scale = float(np.sqrt(np.mean(band ** 2)))
    ee = abs(res["e"][3] - ora["e_total"]) / n_atoms
    eb = abs(res["e"][0] - ora["e_band"]) / n_atoms
    st = res["stats"]
    print(f"  {label} bf16: max force err {fe:.3e} eV/A (rms {frms:.3e}, rms band force {f_scale:.3f}), "
          f"E_tot err {ee:.3e} eV/atom, E_band err {eb:.3e} eV/atom, mu err {abs(res['mu'] - ora['mu']):.3e} eV, "
          f"reorth steps/atom {st['reorth_steps'] / n_atoms:.1f}")
    assert st["flags"] == 0
    e_bound = 4 * 2.0 ** -8 * 40.0
    assert ee <= e_bound and eb <= e_bound
    assert frms <= 2.0 ** -6 * f_scale


def test_parity_c60_240_bf16(torch_cuda, c60_240_oracle):
    """BF16 V_k operand in H.V (FP32 Hamiltonian, FP32 accumulation, a pass at
    every step): errors within the BF16 perturbation bounds."""
    w, ora = c60_240_oracle
    ctx = make_ctx(w.n_atoms, 128, w.r)
    res = gpu_run(ctx, w.pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, n_electrons=w.n_electrons,
                  precision="bf16")
    bf16_check(res, ora, w.n_atoms, "c60_240", w)
    assert res["stats"]["reorth_steps"] == w.n_atoms * (w.r - 1)


@pytest.mark.xfail(strict=False, reason="no BF16-operand form meets 1e-3 eV/A: rounding V_k to 8 "
                                        "significand bits moves the forces by ~1e-1 eV/A (c60_240)")
def test_bf16_operand_force_bar_c60_240(torch_cuda, c60_240_oracle):
    """The mixed-precision force bar (max-abs <= 1e-3 eV/A) applied to the
    BF16-operand form: expected to fail, recorded so that the claim is checked."""
    w, ora = c60_240_oracle
    ctx = make_ctx(w.n_atoms, 128, w.r)
    res = gpu_run(ctx, w.pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, n_electrons=w.n_electrons,
                  precision="bf16")
    fe = float(np.abs(res["forces"] - ora["forces"]).max())
    print(f"  bf16 max force err {fe:.3e} eV/A")
    assert fe <= 1e-3


def test_parity_c60_1920_full(torch_cuda):
    """Precision workload at full size: every atom, mu by bisection."""
    w = inputs.workload("c60_1920")
    ora = otb.run(w.pos, w.cell, (1, 1, 1), P, w.r_cut, w.r, w.kT, n_electrons=w.n_electrons,
                  processes=NPROC)
    ctx = make_ctx(w.n_atoms, 240, w.r)
    res = gpu_run(ctx, w.pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, n_electrons=w.n_electrons)
    assert abs(res["mu"] - ora["mu"]) < 1e-9
    check_against_oracle(res, ora, range(w.n_atoms))
    r32 = gpu_run(ctx, w.pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, n_electrons=w.n_electrons,
                  precision="fp32")
    fe = float(np.abs(r32["forces"] - ora["forces"]).max())
    print(f"  fp32 max force err {fe:.3e} eV/A")
    assert fe <= 1e-3
    rbf = gpu_run(ctx, w.pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, n_electrons=w.n_electrons,
                  precision="bf16")
    bf16_check(rbf, ora, w.n_atoms, "c60_1920", w)


def sampled_parity(name, mu_fixed, n_sample, seed, n_cluster, precisions=("fp64",)):
    w = inputs.workload(name)
    rng = np.random.default_rng(seed)
    S = sorted(rng.choice(w.n_atoms, n_sample, replace=False).tolist())
    need = otb.hop_closure(S, w.pos, w.cell, (1, 1, 1), P)
    ora = otb.run(w.pos, w.cell, (1, 1, 1), P, w.r_cut, w.r, w.kT, mu=mu_fixed, atoms=need,
                  force_atoms=S, r_per_atom=w.r_per_atom, processes=NPROC)
    r_max = int(np.max(w.r_per_atom)) if w.r_per_atom is not None else w.r
    ctx = make_ctx(w.n_atoms, n_cluster, r_max)
    res = {prec: gpu_run(ctx, w.pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, mu=mu_fixed,
                         precision=prec, r_per_atom=w.r_per_atom) for prec in precisions}
    ctx.close()
    return w, S, need, ora, res


@pytest.mark.parametrize("name,n_cluster", [("c60_15360", 400), ("c60_6480_strained", 280)])
def test_parity_large_sampled_fixed_mu(torch_cuda, name, n_cluster):
    """Full-size launch, outputs sampled on seeded atoms the oracle solves one
    by one (chemical potential fixed at 3.5 eV on both sides). FP64: the parity
    bar; mixed precision (FP32 recursion): max-abs force error <= 1e-3 eV/A on
    the sampled atoms, the bar of the 15360-atom target."""
    w, S, need, ora, res = sampled_parity(name, 3.5, 12, 99, n_cluster, precisions=("fp64", "fp32"))
    r64, r32 = res["fp64"], res["fp32"]
    assert r64["stats"]["max_cluster"] <= n_cluster
    worst, scale = compare_rho(r64, ora["rho"], ora["sols"], need)
    print(f"  {name}: rho max abs err {worst:.3e} (scale {scale:.3e}) over {len(need)} seeds")
    assert worst <= 1e-8 * scale
    F = np.array([ora["forces_sampled"][k] for k in S])
    G = r64["forces"][S]
    err = rel_inf(G, F)
    print(f"  {name}: sampled force rel err {err:.3e}")
    assert err <= 1e-8
    w32, _ = compare_rho(r32, ora["rho"], ora["sols"], need)
    fe = float(np.abs(r32["forces"][S] - F).max())
    fe_all = float(np.abs(r32["forces"] - r64["forces"]).max())
    print(f"  {name} fp32: rho max abs err {w32:.3e}, sampled max force err {fe:.3e} eV/A "
          f"(|F| max {np.abs(F).max():.2f}); all {w.n_atoms} atoms against the FP64 path: {fe_all:.3e} eV/A")
    assert r32["stats"]["flags"] == 0
    assert fe <= 1e-3 and fe_all <= 1e-3


def test_parity_c60_240_orbital_seeds(torch_cuda):
    """The paper's per-orbital seeding (tb_set_seeds TB_SEEDS_ORBITAL) against
    the oracle's orbital mode: FP64 to the parity bar, FP32 within 1e-3 eV/A."""
    w = inputs.workload("c60_240")
    ora = otb.run(w.pos, w.cell, (1, 1, 1), P, w.r_cut, w.r, w.kT, n_electrons=w.n_electrons,
                  processes=NPROC, seeds="orbital")
    ctx = make_ctx(w.n_atoms, 128, w.r)
    ctx.set_seeds("orbital")
    res = gpu_run(ctx, w.pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, n_electrons=w.n_electrons)
    assert abs(res["mu"] - ora["mu"]) < 1e-9
    check_against_oracle(res, ora, range(w.n_atoms))
    r32 = gpu_run(ctx, w.pos, w.cell, (1, 1, 1), w.r_cut, w.r, w.kT, n_electrons=w.n_electrons,
                  precision="fp32")
    fe = float(np.abs(r32["forces"] - ora["forces"]).max())
    print(f"  orbital seeds: fp32 max force err {fe:.3e} eV/A; reorth steps/atom "
          f"{res['stats']['reorth_steps'] / w.n_atoms:.1f} (fp64)")
    assert fe <= 1e-3


def test_orbital_seeds_exact_limit_small_cluster(torch_cuda):
    """An isolated jittered 8-atom diamond cell, every sphere the whole cluster
    (32 orbitals), r = 40 past every orbital's grade: the orbital form equals
    full diagonalisation, as does the block form at r = 10."""
    pos, _ = inputs.cubic_diamond(1, 3.567, 0.05, 77)
    pos = pos - pos.mean(axis=0) + 100.0
    ex = exact.solve(pos, BIG, (0, 0, 0), P, 0.1, n_electrons=32.0)
    for seeds, r in (("orbital", 40), ("block", 10)):
        ctx = make_ctx(8, 8, r)
        ctx.set_seeds(seeds)
        res = gpu_run(ctx, pos, BIG, (0, 0, 0), 8.0, r, 0.1, n_electrons=32.0)
        ctx.close()
        print(f"  {seeds}: mu err {abs(res['mu'] - ex['mu']):.2e}, force err {np.abs(res['forces'] - ex['forces']).max():.2e}")
        assert abs(res["mu"] - ex["mu"]) < 1e-9
        assert rel_inf(res["forces"], ex["forces"]) < 1e-8
        assert abs(res["e"][3] - ex["e_total"]) < 1e-10 * abs(ex["e_total"])
