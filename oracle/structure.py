"""Static structure factors of one snapshot (test infrastructure only).

The paper's key observable (Methods, static structure factors) is

  S_ab(q) = <n_a(q) n_b*(q)> / sqrt(N_a N_b),

averaged over the wave vectors of equal magnitude and over sampled MD steps,
with n_a(q) the reciprocal-space density of species a. Readings for one
snapshot on the periodic grid:

  * electrons: n_e(q) = integral n(r) exp(-i q.r) dr = V n~(q) with the
    plane-wave coefficients of `fft` (1/M normalised); N_e = number of
    electrons (sum of the ionic charges);
  * ions (all ions as one species, the paper's systems are single-element):
    n_i(q) = sum_I exp(-i q.R_I), N_i = number of ions;
  * shells: the grid's wave vectors G_m (index map, Nyquist -> -n/2) grouped
    by s = g1^2 + g2^2 + g3^2 (|q| = 2 pi sqrt(s) / L in the cubic cell);
    every grid index counts once;
  * the shell average takes the real part of n_a n_b* (on the grid the
    imaginary parts cancel between q and -q except on Nyquist indices, whose
    partner is not on the grid).

The average over MD steps is the caller's mean of these per-snapshot values.

Parity pins: a uniform electron gas has S_ei = S_ee = 0 off q = 0; a single
ion has S_ii = 1; a simple-cubic ion lattice has S_ii = N_i on its
reciprocal lattice and 0 elsewhere; Gaussian electron clouds of width s on
every ion give S_ei(q) = Z exp(-q^2 s^2 / 4) sqrt(N_i / N_e) S_ii(q) and
S_ee = Z^2 exp(-q^2 s^2 / 2) (N_i / N_e) S_ii; the shell sums against a
brute-force loop over grid indices with a direct DFT.
"""
from __future__ import annotations

import math

import numpy as np

from . import fft, ions


def structure_factors(L: float, n, dens, pos, nelec: float):
    """Shell-averaged S_ei, S_ee, S_ii and the number of grid wave vectors
    per shell, for shells s = 0 .. (n1/2)^2 + (n2/2)^2 + (n3/2)^2."""
    V = L ** 3
    ne = V * fft.fft3(np.asarray(dens, dtype=np.float64))
    (g1, g2, g3), _ = ions.gvectors(L, n)
    k = 2.0 * math.pi / L
    ni = np.zeros(ne.shape, dtype=np.complex128)
    for R in np.asarray(pos):
        ni += np.exp(-1j * k * (g1 * R[0] + g2 * R[1] + g3 * R[2]))
    s = (g1 * g1 + g2 * g2 + g3 * g3).ravel()
    smax = sum((m // 2) ** 2 for m in n)
    cnt = np.bincount(s, minlength=smax + 1).astype(np.int64)
    nI = len(pos)
    def shell_mean(x):
        tot = np.bincount(s, weights=x.ravel(), minlength=smax + 1)
        return np.divide(tot, cnt, out=np.zeros(smax + 1), where=cnt > 0)
    s_ei = shell_mean(np.real(ne * np.conj(ni))) / math.sqrt(nelec * nI)
    s_ee = shell_mean(np.abs(ne) ** 2) / nelec
    s_ii = shell_mean(np.abs(ni) ** 2) / nI
    return s_ei, s_ee, s_ii, cnt


def structure_factors_at(L: float, n, dens, pos, nelec: float, shells):
    """The same shell averages for the listed shells only (every grid index
    of those shells summed directly): S_ei, S_ee, S_ii and counts."""
    V = L ** 3
    ne = V * fft.fft3(np.asarray(dens, dtype=np.float64))
    (g1, g2, g3), _ = ions.gvectors(L, n)
    s = g1 * g1 + g2 * g2 + g3 * g3
    k = 2.0 * math.pi / L
    pos = np.asarray(pos)
    nI = len(pos)
    out = []
    for sh in shells:
        sel = s == sh
        G = np.stack([g1[sel], g2[sel], g3[sel]], -1) * k             # (count, 3)
        ni = np.exp(-1j * (G @ pos.T)).sum(axis=1)
        e = ne[sel]
        c = int(np.count_nonzero(sel))
        out.append((float(np.sum(np.real(e * np.conj(ni)))) / c / math.sqrt(nelec * nI),
                    float(np.sum(np.abs(e) ** 2)) / c / nelec,
                    float(np.sum(np.abs(ni) ** 2)) / c / nI, c))
    return out
