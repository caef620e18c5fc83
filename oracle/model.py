"""Tight-binding model: radial scaling, Slater-Koster sp3 blocks, repulsion.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper's Hamiltonian (Sec. 2, Eq. 1) is a non-self-consistent
tight-binding model with on-site energies and two-centre hoppings; it names
the Xu et al. carbon parameter set with a 2.6 A cutoff (Sec. 4).  The
functional forms below are the Xu-form ones:

  hopping scale  s(r) = (r0/r)^n exp{n[-(r/rc)^nc + (r0/rc)^nc]},  r < r1
                 s(r) = c0 + c1 (r-r1) + c2 (r-r1)^2 + c3 (r-r1)^3, r1 <= r < rm
                 s(r) = 0,                                           r >= rm
  pair term      phi(r): same form with (phi0, d0, m, mc, dc, d1, dm)
  repulsion      E_rep = sum_i F(sum_{j != i} phi(r_ij)), F a quartic.

Orbital order on every atom is (s, px, py, pz).  For the displacement
d = R_j - R_i with direction cosines h = d/|d|, the block H_ij[beta, alpha] =
<i beta|H|j alpha> is the Slater-Koster table:
  ss: V_sss s;  s-p_a: h_a V_sps s;  p_a-s: -h_a V_sps s;
  p_a-p_b: [h_a h_b V_pps + (delta_ab - h_a h_b) V_ppp] s.
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------- radial
def _scaled_form(r, pre, r0, ex, exc, rc):
    """pre * (r0/r)^ex * exp{ex[-(r/rc)^exc + (r0/rc)^exc]}"""
    return pre * (r0 / r) ** ex * np.exp(ex * (-(r / rc) ** exc + (r0 / rc) ** exc))


def _scaled_form_deriv(r, pre, r0, ex, exc, rc):
    """Derivative of _scaled_form with respect to r (product rule)."""
    val = _scaled_form(r, pre, r0, ex, exc, rc)
    return val * (-ex / r - ex * exc * (r / rc) ** exc / r)


def _cubic(x, c):
    return c[0] + x * (c[1] + x * (c[2] + x * c[3]))


def _cubic_deriv(x, c):
    return c[1] + x * (2.0 * c[2] + x * 3.0 * c[3])


def _piecewise(r, head, tail_c, r1, rm, deriv):
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    lo = r < r1
    mid = (r >= r1) & (r < rm)
    rl = np.where(lo, r, r1)            # keep the unused branch finite
    out = np.where(lo, head(rl), out)
    x = r - r1
    tail = _cubic_deriv(x, tail_c) if deriv else _cubic(x, tail_c)
    out = np.where(mid, tail, out)
    return out


def s_radial(r, p):
    head = lambda x: _scaled_form(x, 1.0, p["r0"], p["n"], p["nc"], p["rc"])
    return _piecewise(r, head, p["s_tail"], p["r1"], p["rm"], False)


def s_radial_deriv(r, p):
    head = lambda x: _scaled_form_deriv(x, 1.0, p["r0"], p["n"], p["nc"], p["rc"])
    return _piecewise(r, head, p["s_tail"], p["r1"], p["rm"], True)


def phi_pair(r, p):
    head = lambda x: _scaled_form(x, p["phi0"], p["d0"], p["m"], p["mc"], p["dc"])
    return _piecewise(r, head, p["phi_tail"], p["d1"], p["dm"], False)


def phi_pair_deriv(r, p):
    head = lambda x: _scaled_form_deriv(x, p["phi0"], p["d0"], p["m"], p["mc"], p["dc"])
    return _piecewise(r, head, p["phi_tail"], p["d1"], p["dm"], True)


def f_embed(x, p):
    c = p["frep"]
    return sum(c[k] * x ** k for k in range(5))


def f_embed_deriv(x, p):
    c = p["frep"]
    return sum(k * c[k] * x ** (k - 1) for k in range(1, 5))


# ------------------------------------------------------ Slater-Koster blocks
def sk_blocks(d, p):
    """H_ij blocks for displacement(s) d = R_j - R_i, shape (..., 4, 4)."""
    d = np.asarray(d, dtype=np.float64)
    r = np.linalg.norm(d, axis=-1)
    h = d / r[..., None]
    s = s_radial(r, p)
    out = np.zeros(d.shape[:-1] + (4, 4))
    out[..., 0, 0] = p["v_sss"] * s
    for a in range(3):
        out[..., 0, 1 + a] = h[..., a] * p["v_sps"] * s
        out[..., 1 + a, 0] = -h[..., a] * p["v_sps"] * s
        for b in range(3):
            hh = h[..., a] * h[..., b]
            delta = 1.0 if a == b else 0.0
            out[..., 1 + a, 1 + b] = (hh * p["v_pps"] + (delta - hh) * p["v_ppp"]) * s
    return out


def sk_blocks_grad(d, p):
    """d H_ij / d d_c for d = R_j - R_i, shape (..., 3, 4, 4) with c first.

    Written out by the chain rule: dh_a/dd_c = (delta_ac - h_a h_c)/r and
    ds/dd_c = s'(r) h_c.
    """
    d = np.asarray(d, dtype=np.float64)
    r = np.linalg.norm(d, axis=-1)
    h = d / r[..., None]
    s = s_radial(r, p)
    ds = s_radial_deriv(r, p)
    out = np.zeros(d.shape[:-1] + (3, 4, 4))
    eye = np.eye(3)
    for c in range(3):
        dh = [(eye[a, c] - h[..., a] * h[..., c]) / r for a in range(3)]
        dsc = ds * h[..., c]
        out[..., c, 0, 0] = p["v_sss"] * dsc
        for a in range(3):
            g = p["v_sps"] * (dh[a] * s + h[..., a] * dsc)
            out[..., c, 0, 1 + a] = g
            out[..., c, 1 + a, 0] = -g
            for b in range(3):
                hh = h[..., a] * h[..., b]
                dhh = dh[a] * h[..., b] + h[..., a] * dh[b]
                delta = 1.0 if a == b else 0.0
                val = (hh * p["v_pps"] + (delta - hh) * p["v_ppp"]) * dsc \
                    + (p["v_pps"] - p["v_ppp"]) * dhh * s
                out[..., c, 1 + a, 1 + b] = val
    return out


def onsite_block(p):
    return np.diag([p["eps_s"], p["eps_p"], p["eps_p"], p["eps_p"]])
