"""Pins of the oracle's beta fit (Eq. (3)): the deviation integral against
its plain definition on a constant offset, and recovery of the beta that
generated the reference density."""
import dataclasses

import numpy as np
import pytest

from oracle import fit
from oracle.functional import Problem
from oracle.optimize import optimize
from paper_2601_23002_amd import workloads as W


def test_density_deviation_of_an_offset():
    rng = np.random.default_rng(1)
    a = rng.random((6, 8, 10))
    # |a - (a + c)| = c everywhere: D = c V
    assert abs(fit.density_deviation(3.0, a, a + 0.25) - 0.25 * 27.0) < 1e-13


@pytest.mark.slow
def test_fit_recovers_the_generating_beta():
    s = W.uniform_system(3, 1.0, 0.4, 2.0, 1.0, 12, seed=71, beta=0.6)
    ref = optimize(Problem(s), gtol=1e-10, max_iter=2000)["n"]
    beta, dev, nsolve = fit.fit_beta(dataclasses.replace(s, beta=1.0), ref, 0.0, 2.0, xtol=1e-4)
    assert abs(beta - 0.6) < 2e-3
    assert dev < 1e-3 * fit.density_deviation(s.L, ref, np.zeros_like(ref))
