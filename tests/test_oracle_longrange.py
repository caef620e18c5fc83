"""Pins of the oracle under the long-range parameter set (hopping to 7 A,
inputs.PARAMS_LONG), the regime of the paper's second parameter set (Sec. 4)
where the local Hamiltonian is nearly dense:

* the stored cubic tail is re-derived from the C1 conditions at r1 and rm,
  and s(r) is continuous with its derivative across r1 and vanishes at rm;
* an isolated C60 whose cutoff sphere holds the whole molecule, at r past
  the grade, equals full diagonalisation (mu, energies, forces), and the
  forces equal central differences of the exact energy;
* inside a cutoff sphere about a third of all atom pairs are coupled (the
  product H.V is nearly dense), against ~5 % for Xu's 2.6 A set.
"""
import numpy as np
import pytest

from paper_0910_4497_amd import inputs
from oracle import exact, geometry, krylov, model, tb

PL = inputs.load_params(inputs.PARAMS_LONG)
PX = inputs.load_params()
BIG = np.array([200.0, 200.0, 200.0])
ISO = (0, 0, 0)


def test_long_range_tail_rederived():
    def head(r):
        return (PL["r0"] / r) ** PL["n"] * np.exp(PL["n"] * (-(r / PL["rc"]) ** PL["nc"]
                                                            + (PL["r0"] / PL["rc"]) ** PL["nc"]))
    h = PL["rm"] - PL["r1"]
    d = 1e-6
    slope = (head(PL["r1"] + d) - head(PL["r1"] - d)) / (2 * d)
    A = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [1, h, h * h, h ** 3], [0, 1, 2 * h, 3 * h * h]], dtype=np.float64)
    c = np.linalg.solve(A, np.array([head(PL["r1"]), slope, 0.0, 0.0]))
    assert np.allclose(c, PL["s_tail"], rtol=1e-6, atol=1e-15)
    assert PL["rm"] == 7.0 and PL["dm"] == PX["dm"]


def test_long_range_radial_continuity():
    a, b = PL["r1"], PL["rm"]
    e = 1e-9
    assert abs(model.s_radial(a - e, PL) - model.s_radial(a + e, PL)) < 1e-12
    assert abs(model.s_radial_deriv(a - e, PL) - model.s_radial_deriv(a + e, PL)) < 1e-9
    assert abs(model.s_radial(b - e, PL)) < 1e-14 and model.s_radial(b + 0.1, PL) == 0.0
    r = np.linspace(0.9, b - 0.01, 131)
    h = 1e-6
    fd = (model.s_radial(r + h, PL) - model.s_radial(r - h, PL)) / (2 * h)
    assert np.allclose(model.s_radial_deriv(r, PL), fd, rtol=1e-6, atol=1e-12)


@pytest.fixture(scope="module")
def molecule():
    rng = np.random.default_rng(41)
    return inputs.c60_ideal() + rng.normal(0, 0.04, (60, 3))


def test_long_range_exact_limit(molecule):
    mol = molecule
    assert max(len(geometry.cluster(i, mol, BIG, ISO, 8.0)[0]) for i in range(60)) == 60
    kr = tb.run(mol, BIG, ISO, PL, 8.0, 70, 0.1, n_electrons=240.0, processes=4)
    ex = exact.solve(mol, BIG, ISO, PL, 0.1, n_electrons=240.0)
    assert abs(kr["mu"] - ex["mu"]) < 1e-10
    for key in ("e_band", "e_rep", "e_total"):
        assert abs(kr[key] - ex[key]) < 1e-9 * max(1.0, abs(ex[key])), key
    assert np.abs(kr["forces"] - ex["forces"]).max() < 1e-9
    h = 1e-4
    for k, c in [(5, 1), (44, 0)]:
        es = []
        for sgn in (1, -1):
            x = mol.copy()
            x[k, c] += sgn * h
            es.append(exact.solve(x, BIG, ISO, PL, 0.1, n_electrons=240.0)["e_total"])
        fd = -(es[0] - es[1]) / (2 * h)
        assert abs(fd - kr["forces"][k, c]) < 1e-6 * max(1.0, abs(fd))


def test_long_range_local_H_is_dense():
    w = inputs.workload("c60_1920_long")
    frac = {}
    for name, p, rcut in (("long", PL, w.r_cut), ("xu", PX, 7.0)):
        idx, x = geometry.cluster(17, w.pos, w.cell, (1, 1, 1), rcut)
        H = krylov.cluster_hamiltonian(x, p).reshape(len(idx), 4, len(idx), 4)
        coupled = np.abs(H).max(axis=(1, 3)) > 0
        frac[name] = coupled.mean()
    assert frac["long"] > 0.3 and frac["long"] > 5 * frac["xu"] and frac["xu"] < 0.1, frac
