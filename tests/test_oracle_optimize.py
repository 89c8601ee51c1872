"""Pins of the oracle's constrained minimisation: charge conservation,
stationarity, and the linear-response limit of the functional."""
import math

import numpy as np

from oracle import kernel
from oracle.functional import Problem, TERM_TF, TERM_VW, TERM_NL0, TERM_NL1, TERM_LOCPP
from oracle.optimize import optimize, STATUS_OK
from paper_2601_23002_amd import workloads as W


def test_optimize_small_system_conserves_charge_and_converges():
    s = W.uniform_system(6, 1.0, 0.4, 2.0, 1.0, 12, seed=41)
    p = Problem(s)
    res = optimize(p, gtol=1e-9, max_iter=400)
    assert res["status"] == STATUS_OK
    assert res["gnorm"] < 1e-9
    assert abs(p.dV * np.sum(res["n"]) - p.ne) < 1e-13 * p.ne
    # energies never rise by more than the rounding tolerance
    E = np.array([h[0] for h in res["history"]])
    assert np.all(np.diff(E) <= 1e-12 * np.abs(E[1:]))
    # stationarity: dE/dphi = 2 mu phi
    e, g = p.evaluate(res["phi"])
    r = g - 2 * e["mu"] * res["phi"]
    assert math.sqrt(p.dot(r, r)) < 1e-9


def test_warm_start_from_solution_stays():
    s = W.uniform_system(6, 1.0, 0.4, 2.0, 1.0, 12, seed=42)
    p = Problem(s)
    res = optimize(p, gtol=1e-9, max_iter=400)
    res2 = optimize(p, phi0=np.sqrt(res["n"]), gtol=1e-9, max_iter=50)
    assert res2["iters"] <= 2
    assert abs(res2["energy"]["free_energy"] - res["energy"]["free_energy"]) < 1e-12 * abs(
        res["energy"]["free_energy"])


def _response_problem(terms, beta=1.0, a=5 / 6):
    L, n, n0, T = 8.0, 16, 0.03, 1.0
    s = W.System(L=L, n=(n, n, n), pos=np.zeros((1, 3)), zval=np.array([n0 * L ** 3]),
                 rc=np.array([0.5]), T=T, beta=beta, alpha=a, terms=terms | TERM_LOCPP)
    return Problem(s, with_ewald=False)


def test_linear_response_reproduces_lindhard():
    # with a weak v_ext = eps cos(G x), the minimising density has
    # n~(G) = chi0(G) eps / 2 + O(eps^3): the functional's kernel makes
    # TF + vW + F0 respond exactly like the free gas; F1 (cubic in dn)
    # must not change the linear response for any beta
    eps, g = 1e-3, 2
    for terms, beta in ((TERM_TF | TERM_VW | TERM_NL0, 1.0),
                        (TERM_TF | TERM_VW | TERM_NL0 | TERM_NL1, 2.5)):
        p = _response_problem(terms, beta)
        v = np.zeros(p.n, dtype=complex)
        v[g, 0, 0] = v[-g, 0, 0] = eps / 2
        p.vloc = v
        res = optimize(p, gtol=1e-12, max_iter=600)
        assert res["status"] == STATUS_OK
        nt = np.fft.fftn(res["n"]) / p.M
        G = 2 * math.pi * g / p.L
        eta0, _ = kernel.uniform_gas(p.n0, p.T)
        chi = kernel.chi0(np.array([G]), p.T, eta0)[0]
        assert abs(nt[g, 0, 0].real / (chi * eps / 2) - 1) < 2e-5, (terms, nt[g, 0, 0], chi)
