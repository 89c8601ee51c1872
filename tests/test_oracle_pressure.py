"""Pins of the oracle's pressure closed forms against central differences
of the oracle's own energies in the volume."""
import numpy as np

from oracle import fermi, ions, pressure, xc


def _uniform_free_energy(V, N, T, with_xc):
    n0 = N / V
    _, f, _ = fermi.tf_terms(np.array([n0]), T)
    F = V * float(f[0])
    if with_xc:
        eps, _ = xc.pz81(np.array([n0]))
        F += V * n0 * float(eps[0])
    return F


def test_uniform_gas_pressure_is_minus_dF_dV():
    for (N, V, T) in ((8.0, 268.0, 1.0), (64.0, 270.0, 0.5), (16.0, 2000.0, 8.0)):
        for with_xc in (False, True):
            h = 1e-4 * V
            fd = -(_uniform_free_energy(V + h, N, T, with_xc)
                   - _uniform_free_energy(V - h, N, T, with_xc)) / (2 * h)
            p = pressure.uniform_pressure(N / V, T, with_xc)
            assert abs(p - fd) < 1e-7 * abs(p)


def test_ewald_pressure_is_minus_dE_dV():
    rng = np.random.default_rng(4)
    L = 7.0
    frac = rng.random((5, 3))
    Z = np.array([1.0, 4.0, 1.0, 1.0, 4.0])
    V = L ** 3
    h = 1e-4 * V
    Lp, Lm = (V + h) ** (1 / 3), (V - h) ** (1 / 3)
    fd = -(ions.ewald(Lp, frac * Lp, Z) - ions.ewald(Lm, frac * Lm, Z)) / (2 * h)
    p = pressure.ewald_pressure(L, frac * L, Z)
    assert abs(p - fd) < 1e-7 * abs(p)
