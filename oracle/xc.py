"""Perdew-Zunger (1981) LDA exchange-correlation, spin-unpolarised
(test infrastructure only).

The paper treats exchange-correlation with Perdew-Zunger LDA in the
adiabatic approximation (Methods, "Numerical calculations"): the
zero-temperature parametrisation is used at every T.

  rs   = (3 / (4 pi n))^{1/3}
  e_x  = -(3/(4 pi)) (9 pi/4)^{1/3} / rs,      v_x = 4/3 e_x
  e_c  = gamma / (1 + beta1 sqrt(rs) + beta2 rs)          rs >= 1
       = A ln rs + B + C rs ln rs + D rs                    rs < 1
  v_c  = e_c - (rs/3) de_c/drs

Two variants, selected by the same codes as the library's functional:

  XC_PZ81     the published fit as printed, branch rs >= 1 at rs = 1
              exactly. Its two correlation branches meet at rs = 1 with a
              jump of ~3e-5 Ha in e_c and v_c (the printed C and D are
              rounded).
  XC_PZ81_C1  the same branches joined C1 over 0.99 <= rs <= 1.01 with the
              weight w = 3t^2 - 2t^3, t = (rs - 0.99)/0.02,
              e_c = (1 - w) e_dense + w e_dilute, and v_c from that e_c
              exactly. Outside the window it equals XC_PZ81. A potential
              that jumps floors a minimiser's residual near 1e-4 when the
              density straddles rs = 1; with the join it converges.

Pins: the exchange closed form; v = d(n eps)/dn for both variants; the
branches on both sides of rs = 1; the size of the published fit's jump; the
log coefficient A against the Gell-Mann-Brueckner value (1 - ln 2)/pi^2.
The correlation constants themselves are "parity unpinned" against the 1981
publication, which is not available here (they are the standard published
values).
"""
from __future__ import annotations

import math

import numpy as np

XC_NONE, XC_PZ81, XC_PZ81_C1 = 0, 1, 2

PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116
CX = (3.0 / (4.0 * math.pi)) * (9.0 * math.pi / 4.0) ** (1.0 / 3.0)


RS_JOIN_LO, RS_JOIN_HI = 0.99, 1.01


def _dilute(r):
    """Correlation for rs >= 1: e_c and de_c/drs."""
    sq = np.sqrt(r)
    den = 1.0 + PZ_BETA1 * sq + PZ_BETA2 * r
    return PZ_GAMMA / den, -PZ_GAMMA * (0.5 * PZ_BETA1 / sq + PZ_BETA2) / den ** 2


def _dense(r):
    """Correlation for rs < 1: e_c and de_c/drs."""
    lr = np.log(r)
    return (PZ_A * lr + PZ_B + PZ_C * r * lr + PZ_D * r,
            PZ_A / r + PZ_C * lr + PZ_C + PZ_D)


def pz81(n, variant: int = XC_PZ81):
    """Energy per electron eps_xc(n) and potential v_xc(n); zero where n <= 0."""
    if variant not in (XC_PZ81, XC_PZ81_C1):
        raise ValueError("unknown PZ81 variant")
    n = np.asarray(n, dtype=np.float64)
    eps = np.zeros(n.shape)
    v = np.zeros(n.shape)
    pos = n > 0
    rs = (3.0 / (4.0 * math.pi * n[pos])) ** (1.0 / 3.0)
    ex = -CX / rs
    vx = 4.0 / 3.0 * ex
    ec = np.empty(rs.shape)
    dec = np.empty(rs.shape)
    if variant == XC_PZ81:
        hi = rs >= 1.0
        ec[hi], dec[hi] = _dilute(rs[hi])
        ec[~hi], dec[~hi] = _dense(rs[~hi])
    else:
        hi = rs >= RS_JOIN_HI
        lo = rs <= RS_JOIN_LO
        mid = ~(hi | lo)
        ec[hi], dec[hi] = _dilute(rs[hi])
        ec[lo], dec[lo] = _dense(rs[lo])
        r = rs[mid]
        e1, d1 = _dense(r)
        e2, d2 = _dilute(r)
        t = (r - RS_JOIN_LO) / (RS_JOIN_HI - RS_JOIN_LO)
        w = t * t * (3.0 - 2.0 * t)
        dw = 6.0 * t * (1.0 - t) / (RS_JOIN_HI - RS_JOIN_LO)
        ec[mid] = (1.0 - w) * e1 + w * e2
        dec[mid] = (1.0 - w) * d1 + w * d2 + dw * (e2 - e1)
    vc = ec - rs / 3.0 * dec
    eps[pos] = ex + ec
    v[pos] = vx + vc
    return eps, v
