"""Finite-temperature Lindhard response and the nonlocal kernels w, dw/dn0
(test infrastructure only).

Paper: F0 is a finite-temperature Wang-Teter functional whose kernel is the
second functional derivative at the mean valence density (Results, text
around Eq. (2)). Reading: the kernel is fixed by demanding that
TF + vW + F0 reproduce the non-interacting static response of the uniform
gas at (n0, T):

  chi0(q)   = -(1/(pi^2 q)) int_0^inf k f(k) ln|(2k+q)/(2k-q)| dk,
              f(k) = 1/(1 + exp(k^2/(2T) - eta0))
  K(q)      = -1/chi0(q) - dmu0/dn - q^2/(4 n0),
              dmu0/dn = sqrt(2) pi^2 / (T^{1/2} I_{-1/2}(eta0))
  w(q)      = K(q) n0^{2-2a} / (2 a^2),      w(0) = 0
  F0        = int int f(r) w(r-r') f(r'),    f = n^a

F1 reading (the paper describes it as a first-order inhomogeneity
correction obtained from line integrals, with no formula): the kernel's
density argument is expanded to first order along n0 + t(n - n0), which
needs w'(q) = dw(q; n0, T)/dn0 at fixed T.

chi0 is integrated directly (log singularity at k = q/2 kept as an
endpoint) with tanh-sinh quadrature on intervals split at q/2 and around
the Fermi edge. w' is a central difference in n0 with two Richardson
extrapolation levels. Pins: the T -> 0 closed-form Lindhard function, the
compressibility sum rule chi0(0) = -dn/dmu, K(q -> 0) -> 0, and the
Sommerfeld (T/E_F)^2 approach to the zero-temperature limit.
"""
from __future__ import annotations

import math

import numpy as np

from . import fermi

_TS_H = 1.0 / 48.0
_TS_T = np.arange(-173, 174) * _TS_H          # |t| <= 3.6
_TS_U = 0.5 * math.pi * np.sinh(_TS_T)
_TS_W = 0.5 * math.pi * np.cosh(_TS_T) / np.cosh(_TS_U) ** 2
# fraction of the interval from the left end, and from the right end, both
# computed without cancellation near the ends
_TS_FL = 1.0 / (1.0 + np.exp(-2.0 * _TS_U))
_TS_FR = 1.0 / (1.0 + np.exp(2.0 * _TS_U))


def chi0(q, T: float, eta0: float) -> np.ndarray:
    """Static finite-temperature Lindhard function for wave numbers q > 0."""
    q = np.atleast_1d(np.asarray(q, dtype=np.float64))
    if np.any(q <= 0):
        raise ValueError("chi0 needs q > 0")
    kmax = math.sqrt(2.0 * T * (max(eta0, 0.0) + 50.0))
    half = np.minimum(0.5 * q, kmax)
    if eta0 > 0:
        kf = math.sqrt(2.0 * T * eta0)
        wid = 3.0 * T / kf
        extra = [max(kf - wid, 0.0), kf, min(kf + wid, kmax)]
    else:
        extra = []
    nq = q.size
    pts = np.stack([np.zeros(nq), half] + [np.full(nq, e) for e in extra]
                   + [np.full(nq, kmax)], axis=1)
    pts = np.sort(pts, axis=1)
    total = np.zeros(nq)
    for c in range(pts.shape[1] - 1):
        a = pts[:, c][:, None]
        b = pts[:, c + 1][:, None]
        L = b - a
        k = a + L * _TS_FL[None, :]
        da = L * _TS_FL[None, :]        # k - a
        db = L * _TS_FR[None, :]        # b - k
        qq = q[:, None]
        # |2k - q| measured from whichever end is the singular point
        left_sing = (a == 0.5 * qq)
        right_sing = (b == 0.5 * qq)
        d = np.where(left_sing, 2.0 * da,
                     np.where(right_sing, 2.0 * db, np.abs(2.0 * k - qq)))
        f = 1.0 / (1.0 + np.exp(k * k / (2.0 * T) - eta0))
        with np.errstate(divide="ignore", invalid="ignore"):
            g = k * f * (np.log(2.0 * k + qq) - np.log(d))
        g = np.where((k > 0) & (d > 0), g, 0.0)
        total += 0.5 * L[:, 0] * (g @ _TS_W) * _TS_H
    return -total / (math.pi ** 2 * q)


def uniform_gas(n0: float, T: float):
    """eta0 and dmu/dn of the uniform gas at density n0."""
    nT = fermi.density_scale(T)
    eta0 = float(fermi.eta_from_ratio(np.array([n0 / nT]))[0])
    imh = float(fermi.fd_integrals(np.array([eta0]), (-0.5,))[0][0])
    dmudn = math.sqrt(2.0) * math.pi ** 2 / (math.sqrt(T) * imh)
    return eta0, dmudn


def kernel_K(q, n0: float, T: float) -> np.ndarray:
    """K(q) = -1/chi0 - dmu0/dn - q^2/(4 n0); K(0) = 0."""
    q = np.asarray(q, dtype=np.float64)
    eta0, dmudn = uniform_gas(n0, T)
    out = np.zeros(q.shape)
    pos = q > 0
    if np.any(pos):
        c = chi0(q[pos], T, eta0)
        out[pos] = -1.0 / c - dmudn - q[pos] ** 2 / (4.0 * n0)
    return out


def kernel_w(q, n0: float, T: float, a: float) -> np.ndarray:
    return kernel_K(q, n0, T) * n0 ** (2.0 - 2.0 * a) / (2.0 * a * a)


def kernel_wprime(q, n0: float, T: float, a: float, rel_h: float = 0.01) -> np.ndarray:
    """dw/dn0 at fixed T and q by central differences, Richardson x2."""
    def D(h):
        return (kernel_w(q, n0 + h, T, a) - kernel_w(q, n0 - h, T, a)) / (2.0 * h)
    h = rel_h * n0
    d1, d2, d3 = D(h), D(h / 2), D(h / 4)
    r1 = (4.0 * d2 - d1) / 3.0
    r2 = (4.0 * d3 - d2) / 3.0
    return (16.0 * r2 - r1) / 15.0


def shell_tables(L: float, n, n0: float, T: float, a: float, need_wprime=True):
    """w and w' on integer shells s = g1^2+g2^2+g3^2 of a cubic cell."""
    smax = sum((m // 2) ** 2 for m in n)
    s = np.arange(smax + 1, dtype=np.float64)
    q = (2.0 * math.pi / L) * np.sqrt(s)
    w = kernel_w(q, n0, T, a)
    wp = kernel_wprime(q, n0, T, a) if need_wprime else np.zeros_like(w)
    w[0] = 0.0
    wp[0] = 0.0
    return w, wp
