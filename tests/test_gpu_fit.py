"""The beta fit of Eq. (3) through the C ABI (skx_fit_beta,
skx_density_deviation): the deviation integral against its plain definition,
and recovery of the beta that generated a reference density computed by the
CPU oracle (no GPU value enters the reference)."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2601_23002_amd import workloads as W

pytestmark = pytest.mark.gpu


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2601_23002_amd import skx
    return skx, torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_density_deviation_matches_definition():
    skx, torch = _lib()
    from oracle import fit
    _say("case: density deviation 24x16x20")
    rng = np.random.default_rng(81)
    a, b = rng.random((24, 16, 20)), rng.random((24, 16, 20))
    c = skx.Context(0)
    c.set_cell(6.5, (24, 16, 20))
    ta = torch.tensor(a, dtype=torch.float64, device="cuda:0")
    tb = torch.tensor(b, dtype=torch.float64, device="cuda:0")
    ref = fit.density_deviation(6.5, a, b)
    assert abs(c.density_deviation(ta, tb) - ref) < 1e-12 * ref
    assert c.density_deviation(ta, ta) == 0.0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fit_recovers_the_generating_beta(prec):
    skx, torch = _lib()
    from oracle.functional import Problem
    from oracle.optimize import optimize
    _say(f"case: beta fit {prec}, 4 H on 16^3, reference from the oracle at beta 0.6")
    s = W.uniform_system(4, 1.0, 0.4, 2.0, 1.0, 16, seed=61, beta=0.6)
    ref = optimize(Problem(s), gtol=1e-10, max_iter=2000)["n"]
    c = skx.Context(0).setup(dataclasses.replace(s, beta=1.0),
                             precision=skx.FP64 if prec == "fp64" else skx.MIXED)
    tref = torch.tensor(ref, dtype=torch.float64, device="cuda:0")
    beta, dev, ns, rho = c.fit_beta(tref, 0.0, 2.0, xtol=1e-4, gtol=1e-9, max_iter=2000)
    _say(f"  beta {beta:.6f}, deviation {dev:.3e}, {ns} solves")
    assert abs(beta - 0.6) < 2e-3
    scale = c.density_deviation(tref, torch.zeros_like(tref))
    assert dev < 1e-3 * scale
    assert abs(c.density_deviation(rho, tref) - dev) < 1e-12 * scale
    # the ctx keeps its own beta: a plain solve equals the beta = 1 minimum
    rho1, r1 = c.optimize(gtol=1e-9, max_iter=2000)
    assert c.density_deviation(rho1, tref) > 10 * dev
    # the Methods' beta over configurations is the caller's mean of the fits
    betas = [c.fit_beta(tref, lo=0.0, hi=2.0, xtol=1e-3, gtol=1e-9, max_iter=2000)[0]]
    assert abs(sum(betas) / len(betas) - 0.6) < 5e-3


def test_fit_errors():
    skx, torch = _lib()
    _say("case: beta fit errors")
    s = W.uniform_system(2, 1.0, 0.4, 2.0, 1.0, 16, seed=62)
    c = skx.Context(0).setup(s)
    t = torch.full(s.n, 0.01, dtype=torch.float64, device="cuda:0")
    for lo, hi, xtol in ((1.0, 1.0, 1e-3), (0.0, 1.0, 0.0), (float("nan"), 1.0, 1e-3)):
        with pytest.raises(skx.SkxError) as e:
            c.fit_beta(t, lo, hi, xtol=xtol)
        assert e.value.code == skx.E_INVALID
