"""Pressure of a configuration for the equation of state (test
infrastructure only).

The paper tabulates and plots the equation of state (Table 1, Fig. 3) but
prints no stress or pressure formula. Reading: the pressure of a snapshot at
fixed ion fractional positions is P = -dF/dV of the minimised total free
energy (electronic free energy plus the Ewald ion-ion energy); the ideal-gas
term of moving ions is the caller's. Closed forms used as pins:

  * uniform electron gas (no spatial terms): the density stays uniform, F/V
    = f(n0) with n0 = N_e / V, so P = n0 f'(n0) - f(n0);
      finite-T TF: P_TF = (2/3) n_T T I_{3/2}(eta0),
      PZ81 XC:     P_xc = n0 (v_xc(n0) - eps_xc(n0));
  * Ewald: at fixed fractional positions every term scales as 1/L, so
    E_ii(V) ~ V^{-1/3} and P_ii = E_ii / (3 V).

Parity pins: each closed form against a central difference of the oracle's
own energy in V (the free-energy density of `fermi`/`xc`, `ions.ewald` on a
scaled cell).
"""
from __future__ import annotations

import numpy as np

from . import fermi, ions, xc


def uniform_pressure(n0: float, T: float, with_xc: bool = True) -> float:
    """P_TF (+ P_xc) of the uniform electron gas at density n0."""
    eta = float(fermi.eta_from_ratio(np.array([n0 / fermi.density_scale(T)]))[0])
    i32 = float(fermi.fd_integrals(np.array([eta]), (1.5,))[0][0])
    p = (2.0 / 3.0) * fermi.density_scale(T) * T * i32
    if with_xc:
        eps, v = xc.pz81(np.array([n0]))
        p += n0 * (float(v[0]) - float(eps[0]))
    return p


def ewald_pressure(L: float, pos, zval) -> float:
    """P_ii = E_ii / (3 V) at fixed fractional positions."""
    return ions.ewald(L, pos, zval) / (3.0 * L ** 3)
