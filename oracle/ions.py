"""Local pseudopotential through the ionic structure factor, and the Ewald
ion-ion energy (test infrastructure only).

The paper uses local pseudopotentials (Heine-Abarenkov for H, a local
s-channel norm-conserving one for Be; Methods). Their parameters are not
printed, so an erf-smeared Coulomb potential stands in:

  v(r)   = -Z erf(r/rc) / r
  v(G)   = -4 pi Z exp(-G^2 rc^2 / 4) / G^2              (G != 0)
  V(G)   = (1/V) sum_I v_I(G) exp(-i G.R_I)
  V(0)   = (1/V) sum_I pi Z_I rc_I^2     (the non-Coulomb G -> 0 limit)

Reading for even grids: the local potential on the grid is the real part
of its plane-wave sum, i.e. the full spectrum is replaced by its Hermitian
part V_s(m) = (V(m) + conj V(-m mod n)) / 2. G components use the index
map m -> m for m < n/2, m - n otherwise (Nyquist -> -n/2).

Ewald: point charges in a neutralising background, standard split with
screening alpha; the result does not depend on alpha (pinned in tests,
together with the simple-cubic Madelung constant).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc


def gvectors(L: float, n):
    """Integer g per axis and |G|^2 on the full grid."""
    gs = [np.where(np.arange(m) < m // 2, np.arange(m), np.arange(m) - m) for m in n]
    g1, g2, g3 = np.meshgrid(*gs, indexing="ij")
    G2 = (2.0 * math.pi / L) ** 2 * (g1 ** 2 + g2 ** 2 + g3 ** 2)
    return (g1, g2, g3), G2


def shells(n):
    (g1, g2, g3), _ = gvectors(1.0, n)
    return (g1 * g1 + g2 * g2 + g3 * g3).astype(np.int64)


def vloc_spectrum(L: float, n, pos, zval, rc) -> np.ndarray:
    """Hermitian-symmetrised plane-wave coefficients of the local potential."""
    (g1, g2, g3), G2 = gvectors(L, n)
    V = L ** 3
    k = 2.0 * math.pi / L
    out = np.zeros(G2.shape, dtype=np.complex128)
    nz = G2 > 0
    for R, Z, r in zip(np.asarray(pos), np.asarray(zval), np.asarray(rc)):
        vG = np.zeros(G2.shape)
        vG[nz] = -4.0 * math.pi * Z * np.exp(-G2[nz] * r * r / 4.0) / G2[nz]
        phase = k * (g1 * R[0] + g2 * R[1] + g3 * R[2])
        out += vG * np.exp(-1j * phase)
    out /= V
    out[0, 0, 0] = np.sum(math.pi * np.asarray(zval) * np.asarray(rc) ** 2) / V
    neg = out[tuple(np.meshgrid(*[(-np.arange(m)) % m for m in n], indexing="ij"))]
    return 0.5 * (out + np.conj(neg))


def ewald(L: float, pos, zval, alpha: float | None = None) -> float:
    """Ewald energy of point charges Z_I at R_I plus a uniform neutralising
    background in a cube of side L (Hartree units)."""
    pos = np.asarray(pos, dtype=np.float64)
    Z = np.asarray(zval, dtype=np.float64)
    V = L ** 3
    if alpha is None:
        alpha = 3.2 / L
    # real space: images with |r + L t| < rcut, erfc(alpha rcut) ~ 1e-18
    rcut = 6.5 / alpha
    nimg = int(math.ceil(rcut / L)) + 1
    rng = np.arange(-nimg, nimg + 1)
    T = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), -1).reshape(-1, 3) * L
    e_real = 0.0
    for i in range(len(Z)):
        d = pos[i][None, :] - pos                       # (N,3)
        r = np.linalg.norm(d[:, None, :] + T[None, :, :], axis=-1)  # (N, nT)
        mask = (r > 0) & (r < rcut)
        rr = np.where(mask, r, 1.0)
        e_real += 0.5 * Z[i] * np.sum(Z[:, None] * np.where(mask, erfc(alpha * rr) / rr, 0.0))
    # reciprocal space: |G| < Gcut with exp(-G^2/(4 alpha^2)) ~ 1e-19
    gcut = 2.0 * alpha * math.sqrt(44.0)
    mmax = int(math.ceil(gcut * L / (2.0 * math.pi)))
    m = np.arange(-mmax, mmax + 1)
    gg = np.stack(np.meshgrid(m, m, m, indexing="ij"), -1).reshape(-1, 3)
    gg = gg[np.any(gg != 0, axis=1)]
    G = gg * (2.0 * math.pi / L)
    G2 = np.sum(G * G, axis=1)
    keep = G2 < gcut * gcut
    G, G2 = G[keep], G2[keep]
    S = np.exp(1j * (G @ pos.T)) @ Z
    e_rec = (2.0 * math.pi / V) * np.sum(np.abs(S) ** 2 * np.exp(-G2 / (4.0 * alpha ** 2)) / G2)
    e_self = -alpha / math.sqrt(math.pi) * np.sum(Z * Z)
    e_bg = -math.pi * np.sum(Z) ** 2 / (2.0 * V * alpha ** 2)
    return float(e_real + e_rec + e_self + e_bg)
