"""Pins of the oracle's ionic forces (local pseudopotential and Ewald).

Each test compares the force oracle with something it does not share a
formula with: central finite differences of the separately pinned energies,
Newton's third law, lattice symmetry, the independence of the Ewald split
parameter, and the closed-form attraction between an erf-smeared ion and a
Gaussian electron cloud.
"""
import math

import numpy as np
from scipy.special import erf

from oracle import forces, ions


def _random_density(n, seed):
    rng = np.random.default_rng(seed)
    return 0.05 + rng.random(n)


def test_local_force_is_minus_the_energy_gradient():
    L, n = 7.0, (12, 16, 10)
    rng = np.random.default_rng(4)
    pos = rng.random((3, 3)) * L
    zval, rc = [1.0, 4.0, 1.0], [0.3, 0.5, 0.45]
    dens = _random_density(n, 5)
    F = forces.local_forces(L, n, dens, pos, zval, rc)
    h = 1e-4
    fd = np.zeros_like(F)
    for I in range(3):
        for a in range(3):
            p = pos.copy(); p[I, a] += h
            m = pos.copy(); m[I, a] -= h
            fd[I, a] = -(forces.local_energy(L, n, dens, p, zval, rc)
                         - forces.local_energy(L, n, dens, m, zval, rc)) / (2 * h)
    assert np.max(np.abs(F - fd)) < 1e-6 * np.max(np.abs(F))


def test_local_force_vanishes_in_a_uniform_density():
    L, n = 6.0, (8, 8, 8)
    pos = np.array([[0.3, 1.7, 2.2], [4.1, 0.2, 5.0]])
    F = forces.local_forces(L, n, np.full(n, 0.2), pos, [1.0, 4.0], [0.3, 0.5])
    assert np.max(np.abs(F)) < 1e-13


def test_local_force_of_a_gaussian_cloud():
    # An erf-smeared ion (charge density a Gaussian of width rc) and a
    # Gaussian electron cloud of width s attract like two Gaussian charges:
    # E(d) = -Z q erf(d / sigma) / d with sigma^2 = s^2 + rc^2. In the
    # periodic cell the neutralising background inside radius d pushes the
    # ion outward by Z (4 pi / 3) (q / V) d; the cubic image terms are
    # O(d^3 / L^5), about 2e-5 of the force here.
    L, N = 24.0, 96
    Z, rc, q, s, d = 1.0, 0.5, 1.0, 1.0, 1.5
    C = np.array([11.0, 12.0, 12.0])
    x = np.arange(N) * L / N
    X, Y, Zg = np.meshgrid(x, x, x, indexing="ij")
    dens = np.zeros((N, N, N))
    for t in (-1, 0, 1):
        for u in (-1, 0, 1):
            for w in (-1, 0, 1):
                r2 = (X - C[0] + t * L) ** 2 + (Y - C[1] + u * L) ** 2 + (Zg - C[2] + w * L) ** 2
                dens += q * (math.pi * s * s) ** -1.5 * np.exp(-r2 / (s * s))
    R = C + np.array([d, 0.0, 0.0])
    F = forces.local_forces(L, (N, N, N), dens, R[None, :], [Z], [rc])[0]
    sig = math.sqrt(s * s + rc * rc)
    dEdd = -Z * q * (2 / math.sqrt(math.pi) * math.exp(-(d / sig) ** 2) / (sig * d)
                     - erf(d / sig) / (d * d))
    expect = -dEdd + Z * (4 * math.pi / 3) * (q / L ** 3) * d
    assert abs(F[0] - expect) < 5e-5 * abs(expect)
    assert abs(F[1]) < 1e-10 and abs(F[2]) < 1e-10


def test_ewald_force_is_minus_the_energy_gradient():
    L = 6.0
    rng = np.random.default_rng(7)
    pos = rng.random((5, 3)) * L
    Z = np.array([1.0, 4.0, 1.0, 1.0, 4.0])
    F = forces.ewald_forces(L, pos, Z)
    h = 1e-5
    fd = np.zeros_like(F)
    for I in range(5):
        for a in range(3):
            p = pos.copy(); p[I, a] += h
            m = pos.copy(); m[I, a] -= h
            fd[I, a] = -(ions.ewald(L, p, Z) - ions.ewald(L, m, Z)) / (2 * h)
    assert np.max(np.abs(F - fd)) < 1e-6 * np.max(np.abs(F))


def test_ewald_forces_obey_newtons_third_law_and_ignore_alpha():
    L = 8.0
    rng = np.random.default_rng(8)
    pos = rng.random((7, 3)) * L
    Z = rng.choice([1.0, 4.0], 7)
    F1 = forces.ewald_forces(L, pos, Z, alpha=2.6 / L)
    F2 = forces.ewald_forces(L, pos, Z, alpha=4.1 / L)
    scale = np.max(np.abs(F1))
    assert np.max(np.abs(F1.sum(axis=0))) < 1e-11 * scale * len(Z)
    assert np.max(np.abs(F1 - F2)) < 1e-9 * scale


def test_ewald_force_vanishes_on_a_cubic_lattice():
    L = 9.0
    g = np.arange(3) * (L / 3)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    bcc = np.concatenate([pos, pos + L / 6])
    for p in (pos, bcc):
        F = forces.ewald_forces(L, p, np.ones(len(p)))
        assert np.max(np.abs(F)) < 1e-10


def test_ewald_force_of_a_close_pair_is_coulomb():
    L = 30.0
    pos = np.array([[15.0, 15.0, 15.0], [16.0, 15.0, 15.0]])
    F = forces.ewald_forces(L, pos, [1.0, 2.0])
    assert abs(F[0, 0] + 2.0) < 2e-3 and abs(F[1, 0] - 2.0) < 2e-3
    assert np.max(np.abs(F[:, 1:])) < 1e-12


def test_ewald_force_rows_equal_the_full_computation():
    L = 7.0
    rng = np.random.default_rng(9)
    pos = rng.random((6, 3)) * L
    Z = rng.choice([1.0, 4.0], 6)
    full = forces.ewald_forces(L, pos, Z)
    part = forces.ewald_forces(L, pos, Z, idx=[1, 4])
    assert np.array_equal(part[[1, 4]], full[[1, 4]])
    assert np.all(part[[0, 2, 3, 5]] == 0.0)
