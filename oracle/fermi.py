"""Fermi-Dirac integrals and the finite-temperature Thomas-Fermi term
(test infrastructure only).

Reading (the paper names the finite-temperature TF functional, Eq. (1) and
the sentence after it, but prints no formula): TF is the exact free energy
density of the uniform non-interacting electron gas at temperature T,
evaluated at the local density:

  I_nu(eta) = int_0^inf x^nu / (1 + exp(x - eta)) dx
  n         = (sqrt(2)/pi^2) T^{3/2} I_{1/2}(eta)             (spin 2)
  f_TF      = n T eta - (2 sqrt(2)/(3 pi^2)) T^{5/2} I_{3/2}(eta)
  v_TF      = dF_TF/dn = T eta

Quadrature: substitute x = t^2 (removes the x^-1/2 endpoint behaviour),
split the x axis at fixed offsets around the Fermi edge x = max(eta, 0),
and apply 32-point Gauss-Legendre on every panel in t. The tail beyond
max(eta,0)+50 is below 1e-19 relative. Pinned in the tests by the closed
forms at eta = 0 (Gamma(nu+1)(1-2^-nu)zeta(nu+1)), by the non-degenerate
series and the degenerate Sommerfeld limit, and by the uniform-gas numbers
fixed from the paper's density/temperature pairs.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy.special import expit

_GL_X, _GL_W = leggauss(32)
# panel edges in x, as offsets from the Fermi edge max(eta, 0)
_OFFSETS = (-36.0, -26.0, -16.0, -8.0, -4.0, -2.0, -1.0, 0.0,
            1.0, 2.0, 4.0, 8.0, 16.0, 26.0, 38.0, 50.0)

NT_COEF = math.sqrt(2.0) / math.pi ** 2          # n = NT_COEF T^1.5 I_1/2
GAMMA_3_2 = math.sqrt(math.pi) / 2.0


def fd_integrals(eta, orders=(0.5,), derivative=False, chunk=1 << 15):
    """I_nu(eta) for each nu in `orders` (nu > -1).

    With derivative=True the Fermi function F is replaced by
    dF/deta = F (1 - F), giving dI_nu/deta.
    Returns a list of arrays, one per order, shaped like `eta`.
    """
    eta = np.asarray(eta, dtype=np.float64)
    flat = eta.reshape(-1)
    outs = [np.zeros_like(flat) for _ in orders]
    for s in range(0, flat.size, chunk):
        e = flat[s:s + chunk]
        base = np.maximum(e, 0.0)
        edges = [np.zeros_like(e)] + [np.maximum(base + o, 0.0) for o in _OFFSETS]
        for a, b in zip(edges[:-1], edges[1:]):
            ta, tb = np.sqrt(a), np.sqrt(b)
            half = 0.5 * (tb - ta)
            if not np.any(half > 0):
                continue
            t = (0.5 * (ta + tb))[:, None] + half[:, None] * _GL_X[None, :]
            F = expit(e[:, None] - t * t)
            if derivative:
                F = F * (1.0 - F)
            for i, nu in enumerate(orders):
                g = 2.0 * t ** (2.0 * nu + 1.0) * F
                outs[i][s:s + chunk] += half * (g @ _GL_W)
    return [o.reshape(eta.shape) for o in outs]


def fd_half(eta):
    return fd_integrals(eta, (0.5,))[0]


def eta_from_ratio(u, tol=1e-12, max_iter=60):
    """Solve I_{1/2}(eta) = u (u > 0) by Newton on ln I_{1/2}.

    ln I_{1/2}(eta) is increasing and concave in eta, so Newton converges
    monotonically after at most one overshoot from any start. Iteration
    stops once the step is below `tol` (relative); one more step is then
    taken, which quadratic convergence carries to full double precision.
    """
    u = np.asarray(u, dtype=np.float64)
    flat = u.reshape(-1)
    if np.any(flat <= 0) or not np.all(np.isfinite(flat)):
        raise ValueError("density ratio must be positive and finite")
    eta = np.maximum(np.log(flat / GAMMA_3_2), (1.5 * flat) ** (2.0 / 3.0))
    active = np.arange(flat.size)
    lu = np.log(flat)
    for _ in range(max_iter):
        if active.size == 0:
            break
        e = eta[active]
        i_half, i_mhalf = fd_integrals(e, (0.5, -0.5))
        g = np.log(i_half) - lu[active]
        dg = i_mhalf / (2.0 * i_half)
        step = g / dg
        eta[active] = e - step
        done = np.abs(step) <= tol * np.maximum(1.0, np.abs(e))
        if np.any(done):
            fin = active[done]
            e2 = eta[fin]
            ih, imh = fd_integrals(e2, (0.5, -0.5))
            eta[fin] = e2 - (np.log(ih) - lu[fin]) / (imh / (2.0 * ih))
        active = active[~done]
    else:
        raise RuntimeError("Fermi-Dirac inversion did not converge")
    return eta.reshape(u.shape)


def density_scale(T: float) -> float:
    """n_T = (sqrt 2 / pi^2) T^{3/2}: the density at which I_{1/2}(eta) = 1."""
    return NT_COEF * T ** 1.5


def tf_density(eta, T):
    return density_scale(T) * fd_half(eta)


def tf_terms(n, T):
    """Pointwise eta, free-energy density f_TF and potential v_TF = T eta.

    n must be positive (the optimiser keeps it so); zero-density points
    contribute zero energy and the potential term 2 phi T eta -> 0.
    """
    n = np.asarray(n, dtype=np.float64)
    nT = density_scale(T)
    pos = n > 0
    eta = np.full(n.shape, -np.inf)
    f = np.zeros(n.shape)
    if np.any(pos):
        e = eta_from_ratio(n[pos] / nT)
        i32 = fd_integrals(e, (1.5,))[0]
        eta[pos] = e
        f[pos] = n[pos] * T * e - (2.0 / 3.0) * nT * T * i32
    return eta, f, T * eta
