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


def _system(nions, n, seed, terms, beta=0.7, rs=2.0, T=1.0):
    from paper_2601_23002_amd import workloads as W
    return W.uniform_system(nions, 1.0, 0.4, rs, T, n, seed=seed, beta=beta, terms=terms)


def test_minimised_pressure_of_the_uniform_gas_is_the_closed_form():
    """With no spatial terms the minimum is the uniform density, so the
    minimised-energy pressure is the closed-form TF + XC + Ewald value."""
    from paper_2601_23002_amd import workloads as W
    s = _system(4, 12, 91, W.TERM_TF | W.TERM_XC)
    P, lo, hi = pressure.minimised_pressure(s, eps=1e-4, gtol=1e-11)
    ref = pressure.uniform_pressure(s.nelec / s.L ** 3, s.T, True) + pressure.ewald_pressure(
        s.L, s.pos, s.zval)
    assert abs(P - ref) < 1e-7 * abs(ref)
    assert (lo > hi) == (P > 0)


def test_minimised_pressure_equals_the_scaled_density_route():
    """Full functional (beta != 0, every term): two minimisations at
    V0 (1 -+ eps) against two evaluations of the V0 minimum carried with the
    cell. F is stationary in n at the minimum, so the two routes agree to
    O(eps^2); a wrong sign, scaling or volume in either fails."""
    from paper_2601_23002_amd import workloads as W
    from oracle.functional import Problem
    from oracle.optimize import optimize
    s = _system(5, 12, 93, W.TERM_ALL, beta=0.7)
    res = optimize(Problem(s), gtol=1e-11, max_iter=2000)
    assert res["status"] == 0
    P_min, _, _ = pressure.minimised_pressure(s, eps=1e-4, gtol=1e-11, phi0=np.sqrt(res["n"]))
    P_sc = pressure.scaled_density_pressure(s, res["n"], eps=1e-4)
    assert abs(P_min - P_sc) < 1e-8 * abs(P_min), (P_min, P_sc)
    # and the pressure is not dominated by one term: the Ewald part alone differs
    assert abs(P_min - pressure.ewald_pressure(s.L, s.pos, s.zval)) > 1e-3 * abs(P_min)
