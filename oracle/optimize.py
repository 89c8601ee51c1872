"""Density optimisation on sqrt(n) under the electron-count constraint
(test infrastructure only).

The paper minimises the free energy over densities of fixed electron
number (its "SCF iterations", Methods, Table A caption) without stating the
algorithm. Reading: limited-memory BFGS on the sphere int phi^2 = N_e.

  r      = dE/dphi - 2 mu phi,  mu = int phi dE/dphi / (2 N_e)
  d      = -H r by the two-loop recursion over the last m pairs (s, y),
           H0 = gamma P with P(G) = 1/(G^2 + kappa) applied through the
           plane-wave expansion (kinetic preconditioner; kappa = 4 n0
           dmu0/dn, the Thomas-Fermi curvature in phi of the uniform gas)
           and gamma = s.y / y.P y of the newest pair (gamma = 1 without
           history)
  d     <- d - (int d phi / N_e) phi        (tangent to the sphere)
           reset to d = -P r (and drop the history) if d is not descent
  phi(t) = phi cos t + sqrt(N_e) d^ sin t,  d^ = d / ||d||
  t0     = min(||d|| / sqrt(N_e), t_max); backtracking Armijo in t with
           quadratic interpolation, accepting rounding-level energy
           changes once the predicted decrease is below the energy's
           rounding error
  stop   when ||r|| = (int r^2)^{1/2} < gtol, or after max_iter

All inner products are grid integrals (dV times the sum).
"""
from __future__ import annotations

import math

import numpy as np

from . import kernel
from .fft import fft3, ifft3

STATUS_OK, STATUS_NOT_CONVERGED = 0, 1


def make_preconditioner(prob):
    """P(G) = 1/(G^2 + kappa) as a function on grid fields."""
    _, dmudn = kernel.uniform_gas(prob.n0, prob.T)
    kappa = max(4.0 * prob.n0 * dmudn, 1e-3)
    mult = 1.0 / (prob.G2 + kappa)
    return lambda x: np.real(ifft3(mult * fft3(x)))


def optimize(prob, phi0=None, gtol: float = 1e-8, max_iter: int = 1000,
             m: int = 5, c1: float = 1e-4, theta_max: float = 0.5,
             max_trials: int = 20, precondition: bool = True, verbose: bool = False):
    ne = prob.ne
    dot = prob.dot
    P = make_preconditioner(prob) if precondition else (lambda x: x)
    if phi0 is None:
        phi = np.full(prob.n, math.sqrt(prob.n0))
    else:
        phi = np.array(phi0, dtype=np.float64)
    phi *= math.sqrt(ne / dot(phi, phi))
    e, g = prob.evaluate(phi)
    nevals = 1
    E = e["free_energy"]
    mu = dot(phi, g) / (2.0 * ne)
    r = g - 2.0 * mu * phi
    rn = math.sqrt(dot(r, r))
    S, Y = [], []
    it = 0
    history = [(E, rn)]
    status = STATUS_OK
    resets = 0
    while rn >= gtol and it < max_iter:
        # two-loop recursion
        q = r.copy()
        al = []
        for s, y in zip(reversed(S), reversed(Y)):
            rho = 1.0 / dot(y, s)
            a_ = rho * dot(s, q)
            q -= a_ * y
            al.append((a_, rho))
        gamma = dot(S[-1], Y[-1]) / dot(Y[-1], P(Y[-1])) if S else 1.0
        z = gamma * P(q)
        for (s, y), (a_, rho) in zip(zip(S, Y), reversed(al)):
            b = rho * dot(y, z)
            z += (a_ - b) * s
        d = -z
        d -= (dot(d, phi) / ne) * phi
        if dot(r, d) >= 0.0:
            d = -P(r)
            d -= (dot(d, phi) / ne) * phi
            S, Y = [], []
        dnorm = math.sqrt(dot(d, d))
        dh = d / dnorm
        g0 = math.sqrt(ne) * dot(r, dh)
        theta = min(dnorm / math.sqrt(ne), theta_max)
        tolE = 1e-12 * max(1.0, abs(E))
        accepted = False
        for _ in range(max_trials):
            pt = phi * math.cos(theta) + math.sqrt(ne) * math.sin(theta) * dh
            et, gt = prob.evaluate(pt)
            nevals += 1
            Et = et["free_energy"]
            if Et <= E + c1 * theta * g0 + tolE:
                accepted = True
                break
            den = 2.0 * (Et - E - g0 * theta)
            tn = -g0 * theta * theta / den if den > 0 else 0.5 * theta
            theta = min(max(tn, 0.1 * theta), 0.5 * theta)
        if not accepted:
            if S:
                S, Y = [], []
                resets += 1
                continue
            status = STATUS_NOT_CONVERGED
            break
        mut = dot(pt, gt) / (2.0 * ne)
        rt = gt - 2.0 * mut * pt
        s = pt - phi
        y = rt - r
        if dot(s, y) > 0.0:
            S.append(s)
            Y.append(y)
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
        phi, E, r, e, g, mu = pt, Et, rt, et, gt, mut
        rn = math.sqrt(dot(r, r))
        it += 1
        history.append((E, rn))
        if verbose:
            print(f"it {it:4d}  E {E:.15f}  |r| {rn:.3e}  theta {theta:.3e}")
    if rn >= gtol and status == STATUS_OK:
        status = STATUS_NOT_CONVERGED
    return dict(phi=phi, n=phi * phi, energy=e, iters=it, evals=nevals,
                gnorm=rn, mu=mu, status=status, history=history, resets=resets)
