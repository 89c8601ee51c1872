"""Forces on the ions (test infrastructure only).

The paper drives its ions by molecular dynamics in the NVT ensemble
(Methods, molecular dynamics and static structure factors), which needs the
force on every ion at the minimising density. The paper prints no force
formula. Reading: the force is minus the derivative of the total energy with
respect to the ion position. At the minimum the energy is stationary in the
density at fixed electron count, so only the terms that depend explicitly on
the positions contribute (Hellmann-Feynman): the local pseudopotential
energy E_loc and the ion-ion Ewald energy.

Local part. With the plane-wave convention of `fft` and the local potential
of `ions.vloc_spectrum`,

  E_loc = V Re sum_m V(G_m) conj(n~(m))
        = Re sum_m sum_I v_I(G_m) exp(-i G_m.R_I) conj(n~(m)),

summed over every grid index m with G_m from the index map (Nyquist ->
-n/2); the Hermitian symmetrisation of V does not change this real part.
Differentiating the phase gives

  F_I = -dE_loc/dR_I = sum_m G_m v_I(G_m) Im[exp(i G_m.R_I) n~(m)].

The G = 0 term carries no force.

Ewald part (same split as `ions.ewald`): with d = R_I - R_J + L t, r = |d|,

  real:        F_I = Z_I sum_{J,t}' Z_J [erfc(a r)/r^2 + 2a/sqrt(pi) exp(-a^2 r^2)/r] d/r
  reciprocal:  F_I = (4 pi Z_I / V) sum_{G != 0} G exp(-G^2/4a^2)/G^2 Im[exp(i G.R_I) conj(S(G))],
               S(G) = sum_J Z_J exp(i G.R_J);

the self and background terms do not depend on the positions.

Parity pins: both parts against central finite differences of the pinned
energies (`ions.vloc_spectrum` through E_loc, `ions.ewald`), the Ewald force
against Newton's third law (the forces sum to zero), its independence of the
split parameter, the zero force on every ion of a simple-cubic lattice and
the Coulomb force of a close pair in a large cell; the local force against the
closed-form attraction of a Gaussian electron cloud.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from . import fft, ions


def local_forces(L: float, n, dens, pos, zval, rc) -> np.ndarray:
    """F_I = sum_m G_m v_I(G_m) Im[exp(i G_m.R_I) n~(m)] for every ion, from
    the density on the grid (shape n). Returns [nions][3]."""
    nt = fft.fft3(np.asarray(dens, dtype=np.float64))
    (g1, g2, g3), G2 = ions.gvectors(L, n)
    k = 2.0 * math.pi / L
    nz = G2 > 0
    out = np.zeros((len(pos), 3))
    for I, (R, Z, r) in enumerate(zip(np.asarray(pos), np.asarray(zval), np.asarray(rc))):
        vG = np.zeros(G2.shape)
        vG[nz] = -4.0 * math.pi * Z * np.exp(-G2[nz] * r * r / 4.0) / G2[nz]
        phase = k * (g1 * R[0] + g2 * R[1] + g3 * R[2])
        im = np.imag(np.exp(1j * phase) * nt) * vG
        out[I] = [k * np.sum(g1 * im), k * np.sum(g2 * im), k * np.sum(g3 * im)]
    return out


def local_energy(L: float, n, dens, pos, zval, rc) -> float:
    """E_loc = V sum_m Re(n~(m) conj V(m)) with the oracle's local potential."""
    nt = fft.fft3(np.asarray(dens, dtype=np.float64))
    vl = ions.vloc_spectrum(L, n, pos, zval, rc)
    return float(L ** 3 * np.sum(np.real(nt * np.conj(vl))))


def ewald_forces(L: float, pos, zval, alpha: float | None = None, idx=None) -> np.ndarray:
    """Minus the gradient of `ions.ewald` with respect to every position
    (only the rows idx when given, the others left zero)."""
    pos = np.asarray(pos, dtype=np.float64)
    Z = np.asarray(zval, dtype=np.float64)
    V = L ** 3
    if alpha is None:
        alpha = 3.2 / L
    rcut = 6.5 / alpha
    nimg = int(math.ceil(rcut / L)) + 1
    rng = np.arange(-nimg, nimg + 1)
    T = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), -1).reshape(-1, 3) * L
    out = np.zeros((len(Z), 3))
    c = 2.0 * alpha / math.sqrt(math.pi)
    rows = range(len(Z)) if idx is None else idx
    for i in rows:
        d = (pos[i][None, :] - pos)[:, None, :] + T[None, :, :]      # (N, nT, 3)
        r = np.linalg.norm(d, axis=-1)
        mask = (r > 0) & (r < rcut)
        rr = np.where(mask, r, 1.0)
        mag = np.where(mask, erfc(alpha * rr) / rr ** 2 + c * np.exp(-(alpha * rr) ** 2) / rr, 0.0)
        out[i] += Z[i] * np.sum((Z[:, None] * mag / rr)[..., None] * d, axis=(0, 1))
    gcut = 2.0 * alpha * math.sqrt(44.0)
    mmax = int(math.ceil(gcut * L / (2.0 * math.pi)))
    m = np.arange(-mmax, mmax + 1)
    gg = np.stack(np.meshgrid(m, m, m, indexing="ij"), -1).reshape(-1, 3)
    gg = gg[np.any(gg != 0, axis=1)]
    G = gg * (2.0 * math.pi / L)
    G2 = np.sum(G * G, axis=1)
    keep = G2 < gcut * gcut
    G, G2 = G[keep], G2[keep]
    ph = np.exp(1j * (G @ pos.T))                                    # (nG, N)
    S = ph @ Z
    wG = np.exp(-G2 / (4.0 * alpha ** 2)) / G2
    im = np.imag(ph * np.conj(S)[:, None])                            # (nG, N)
    rec = (4.0 * math.pi / V) * Z[:, None] * ((wG[:, None] * im).T @ G)
    if idx is None:
        return out + rec
    out[list(idx)] += rec[list(idx)]
    return out
