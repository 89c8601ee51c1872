"""Pins of the oracle's static structure factors (one snapshot).

Uniform gas, single ion and simple-cubic lattice limits, Gaussian clouds on
the ions (closed-form ratio to S_ii) and a brute-force loop over grid
indices with the textbook DFT.
"""
import math

import numpy as np

from oracle import structure
from oracle.fft import direct_dft3


def test_uniform_gas_and_single_ion():
    L, n = 6.0, (8, 10, 12)
    pos = np.array([[1.3, 2.2, 0.4]])
    s_ei, s_ee, s_ii, cnt = structure.structure_factors(L, n, np.full(n, 0.3), pos, 1.0)
    assert cnt.sum() == np.prod(n)
    assert cnt[0] == 1
    occ = cnt > 0
    assert np.max(np.abs(s_ei[1:])) < 1e-13 and np.max(np.abs(s_ee[1:])) < 1e-13
    assert np.max(np.abs(s_ii[occ] - 1.0)) < 1e-13
    N_e = 0.3 * L ** 3
    assert abs(s_ei[0] - N_e * 1 / math.sqrt(1.0 * 1)) < 1e-12 * N_e


def test_simple_cubic_lattice():
    L, n, a = 8.0, (16, 16, 16), 4
    g = np.arange(a) * (L / a)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    _, _, s_ii, cnt = structure.structure_factors(L, n, np.ones(n), pos, float(len(pos)))
    s = np.arange(len(cnt))
    # reciprocal lattice: g_c all multiples of a, i.e. s = a^2 (h^2 + k^2 + l^2)
    gs = np.arange(-8, 8)
    G = np.stack(np.meshgrid(gs, gs, gs, indexing="ij"), -1).reshape(-1, 3)
    on = np.zeros(len(cnt), bool)
    for v in G[np.all(G % a == 0, axis=1)]:
        on[int(np.sum(v * v))] = True
    occ = cnt > 0
    # shells mixing lattice and non-lattice vectors average to N * fraction
    frac = np.zeros(len(cnt))
    for v in G:
        if np.all(v % a == 0):
            frac[int(np.sum(v * v))] += 1
    frac = np.divide(frac, cnt, out=np.zeros(len(cnt)), where=occ)
    assert np.max(np.abs(s_ii[occ] - len(pos) * frac[occ])) < 1e-9
    assert np.all(s_ii[occ & ~on] < 1e-20 + 1e-9)


def test_gaussian_clouds_on_the_ions():
    L, N, sw, Z = 10.0, 40, 0.9, 1.0
    rng = np.random.default_rng(3)
    pos = rng.random((5, 3)) * L
    x = np.arange(N) * L / N
    X, Y, Zg = np.meshgrid(x, x, x, indexing="ij")
    dens = np.zeros((N, N, N))
    for R in pos:
        for t in (-1, 0, 1):
            for u in (-1, 0, 1):
                for w in (-1, 0, 1):
                    r2 = ((X - R[0] + t * L) ** 2 + (Y - R[1] + u * L) ** 2
                          + (Zg - R[2] + w * L) ** 2)
                    dens += Z * (math.pi * sw * sw) ** -1.5 * np.exp(-r2 / (sw * sw))
    ne = Z * len(pos)
    s_ei, s_ee, s_ii, cnt = structure.structure_factors(L, (N, N, N), dens, pos, ne)
    q2 = (2 * math.pi / L) ** 2 * np.arange(len(cnt))
    occ = (cnt > 0) & (q2 < 16.0)      # resolved shells (exp(-q^2 s^2/4) > 1e-3)
    ratio = math.sqrt(len(pos) / ne)
    ei = Z * np.exp(-q2 * sw * sw / 4) * ratio * s_ii
    ee = Z * Z * np.exp(-q2 * sw * sw / 2) * (len(pos) / ne) * s_ii
    assert np.max(np.abs(s_ei[occ] - ei[occ])) < 1e-9 * np.max(np.abs(ei[occ]))
    assert np.max(np.abs(s_ee[occ] - ee[occ])) < 1e-9 * np.max(np.abs(ee[occ]))


def test_shell_sums_by_brute_force():
    L, n = 5.0, (4, 6, 4)
    rng = np.random.default_rng(9)
    dens = 0.1 + rng.random(n)
    pos = rng.random((3, 3)) * L
    ne = 2.5
    s_ei, s_ee, s_ii, cnt = structure.structure_factors(L, n, dens, pos, ne)
    nt = direct_dft3(dens, -1) / dens.size * L ** 3
    acc = {}
    for a in range(n[0]):
        for b in range(n[1]):
            for c in range(n[2]):
                g = [m if 2 * m < N else m - N for m, N in zip((a, b, c), n)]
                q = [2 * math.pi / L * v for v in g]
                ni = sum(np.exp(-1j * np.dot(q, R)) for R in pos)
                s = g[0] ** 2 + g[1] ** 2 + g[2] ** 2
                e = acc.setdefault(s, [0.0, 0.0, 0.0, 0])
                e[0] += (nt[a, b, c] * np.conj(ni)).real
                e[1] += abs(nt[a, b, c]) ** 2
                e[2] += abs(ni) ** 2
                e[3] += 1
    for s, (ei, ee, ii, c) in acc.items():
        assert cnt[s] == c
        assert abs(s_ei[s] - ei / c / math.sqrt(ne * 3)) < 1e-12 * max(1.0, abs(s_ei[s]))
        assert abs(s_ee[s] - ee / c / ne) < 1e-12 * max(1.0, abs(s_ee[s]))
        assert abs(s_ii[s] - ii / c / 3) < 1e-12 * max(1.0, abs(s_ii[s]))


def test_selected_shells_equal_the_full_computation():
    L, n = 6.0, (10, 12, 8)
    rng = np.random.default_rng(12)
    dens = 0.1 + rng.random(n)
    pos = rng.random((4, 3)) * L
    full = structure.structure_factors(L, n, dens, pos, 3.0)
    for sh, (ei, ee, ii, c) in zip((1, 2, 9, 41), structure.structure_factors_at(
            L, n, dens, pos, 3.0, (1, 2, 9, 41))):
        assert c == full[3][sh]
        assert abs(ei - full[0][sh]) < 1e-12 * max(1.0, abs(ei))
        assert abs(ee - full[1][sh]) < 1e-12 * max(1.0, abs(ee))
        assert abs(ii - full[2][sh]) < 1e-12 * max(1.0, abs(ii))
