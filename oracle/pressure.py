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

For the full functional, `minimised_pressure` takes that reading literally:
two minimisations at V0 (1 -+ eps), fixed fractional ion positions.

Parity pins: each closed form against a central difference of the oracle's
own energy in V (the free-energy density of `fermi`/`xc`, `ions.ewald` on a
scaled cell); the minimised pressure against the closed forms where the
minimum is the uniform gas, and, for the full functional, against the
evaluation-only route `scaled_density_pressure` (stationarity of F at the
minimum).
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


# ----------------------------------------------------------------------------
# Full functional (reading of Table 1 / Fig. 3: P = -dF/dV of the minimised
# total free energy at fixed fractional ion positions)
# ----------------------------------------------------------------------------

def scaled_system(sys, V: float):
    """The system in the cube of volume V, ions at the same fractional
    positions, the same grid."""
    import dataclasses
    L = V ** (1.0 / 3.0)
    return dataclasses.replace(sys, L=L, pos=np.asarray(sys.pos) * (L / sys.L))


def minimised_pressure(sys, eps: float = 1e-4, gtol: float = 1e-10, phi0=None,
                       max_iter: int = 2000):
    """P = -(F(V0(1+eps)) - F(V0(1-eps))) / (2 eps V0), F the minimised total
    free energy (electronic + Ewald), each minimisation started from phi0
    (renormalised to the electron count in its cell). Returns (P, F_lo, F_hi)."""
    from .functional import Problem
    from .optimize import optimize
    V0 = sys.L ** 3
    F = []
    for sgn in (-1.0, 1.0):
        p = Problem(scaled_system(sys, V0 * (1.0 + sgn * eps)))
        res = optimize(p, phi0=phi0, gtol=gtol, max_iter=max_iter)
        if res["status"] != 0:
            raise RuntimeError("pressure solve did not converge")
        F.append(res["energy"]["total"])
    return -(F[1] - F[0]) / (2.0 * eps * V0), F[0], F[1]


def scaled_density_pressure(sys, n_min, eps: float = 1e-4):
    """-dF/dV by evaluations only: the minimising density n_min of the cell
    V0, carried with the cell (the same grid values times V0/V, so the
    electron count is kept), evaluated at V0(1 -+ eps). At a minimum F is
    stationary in n at fixed electron count, so this equals the minimised
    pressure to O(eps^2) -- an independent route to the same number."""
    from .functional import Problem
    V0 = sys.L ** 3
    F = []
    for sgn in (-1.0, 1.0):
        V = V0 * (1.0 + sgn * eps)
        p = Problem(scaled_system(sys, V))
        e, _ = p.evaluate(np.sqrt(np.asarray(n_min) * (V0 / V)), need_grad=False)
        F.append(e["total"])
    return -(F[1] - F[0]) / (2.0 * eps * V0)
