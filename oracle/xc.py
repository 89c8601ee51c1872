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

Exchange is pinned by its closed form; the correlation constants are
"parity unpinned" against the 1981 publication, which is not available
here (they are the standard published values).
"""
from __future__ import annotations

import math

import numpy as np

PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116
CX = (3.0 / (4.0 * math.pi)) * (9.0 * math.pi / 4.0) ** (1.0 / 3.0)


def pz81(n):
    """Energy per electron eps_xc(n) and potential v_xc(n); zero where n <= 0."""
    n = np.asarray(n, dtype=np.float64)
    eps = np.zeros(n.shape)
    v = np.zeros(n.shape)
    pos = n > 0
    rs = (3.0 / (4.0 * math.pi * n[pos])) ** (1.0 / 3.0)
    ex = -CX / rs
    vx = 4.0 / 3.0 * ex
    ec = np.empty(rs.shape)
    vc = np.empty(rs.shape)
    hi = rs >= 1.0
    r = rs[hi]
    sq = np.sqrt(r)
    den = 1.0 + PZ_BETA1 * sq + PZ_BETA2 * r
    ec[hi] = PZ_GAMMA / den
    dec = -PZ_GAMMA * (0.5 * PZ_BETA1 / sq + PZ_BETA2) / den ** 2
    vc[hi] = ec[hi] - r / 3.0 * dec
    lo = ~hi
    r = rs[lo]
    lr = np.log(r)
    ec[lo] = PZ_A * lr + PZ_B + PZ_C * r * lr + PZ_D * r
    dec = PZ_A / r + PZ_C * lr + PZ_C + PZ_D
    vc[lo] = ec[lo] - r / 3.0 * dec
    eps[pos] = ex + ec
    v[pos] = vx + vc
    return eps, v
