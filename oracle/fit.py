"""Kohn-Sham-assisted fit of beta (test infrastructure only).

Eq. (3) and Methods (optimisation of the beta parameter): for one ionic
configuration, beta minimises the integrated absolute density deviation

  D(beta) = integral |n_OF[beta](r) - n_ref(r)| dr,

n_OF[beta] the minimising density of the functional with that beta and n_ref
the reference (KSDFT in the paper; any density supplied by the caller here).
The paper runs Powell's method from SciPy; with one parameter it reduces to a
line minimisation, done here with SciPy's bounded Brent search. The
functional's beta over several configurations is the arithmetic mean of the
per-configuration values (the caller's mean).

Parity pin: with n_ref the oracle's own minimum at some beta*, the fit
returns beta* (D has its zero there).
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.optimize import minimize_scalar

from .functional import Problem
from .optimize import optimize


def density_deviation(L: float, dens_a, dens_b) -> float:
    """D = dV sum |a - b| on the grid (the integral of Eq. (3))."""
    a = np.asarray(dens_a, dtype=np.float64)
    return float(L ** 3 / a.size * np.sum(np.abs(a - np.asarray(dens_b, dtype=np.float64))))


def fit_beta(sys_, n_ref, lo: float, hi: float, xtol: float = 1e-4, gtol: float = 1e-9):
    """beta in [lo, hi] minimising D(beta) for the configuration sys_;
    returns (beta, D(beta), number of solves)."""
    count = [0]

    def D(beta):
        count[0] += 1
        p = Problem(dataclasses.replace(sys_, beta=float(beta)))
        res = optimize(p, gtol=gtol, max_iter=2000)
        return density_deviation(sys_.L, res["n"], n_ref)

    r = minimize_scalar(D, bounds=(lo, hi), method="bounded", options={"xatol": xtol})
    return float(r.x), float(r.fun), count[0]
