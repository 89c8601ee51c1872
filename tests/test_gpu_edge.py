"""Edge cases and error paths of the C ABI on the GPU: uneven and smallest
grids, a single ion, beta = 0 (three fields), a = 1, warm starts, and the
documented error codes."""
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


def _uneven(n=(12, 16, 20), nions=5, seed=21, **kw):
    s = W.uniform_system(nions, 1.0, 0.4, 2.0, 1.0, n[0], seed=seed, **kw)
    s.n = tuple(n)
    return s


def _eval_vs_oracle(skx, torch, s, tol=1e-10):
    from oracle.functional import Problem
    phi = W.random_phi(s, 4, amp=0.3)
    e_ref, g_ref = Problem(s).evaluate(phi)
    c = skx.Context(0).setup(s)
    e, g = c.evaluate(torch.tensor(phi, dtype=torch.float64, device="cuda"), skx.SQRT_RHO)
    scale = max(1.0, abs(e_ref["free_energy"]))
    assert abs(e["free_energy"] - e_ref["free_energy"]) <= tol * scale
    assert np.max(np.abs(g.cpu().numpy() - g_ref)) <= 10 * tol * np.max(np.abs(g_ref))


@pytest.mark.parametrize("n", [(12, 16, 20), (8, 8, 8), (20, 12, 16)])
def test_uneven_and_smallest_grids_evaluate(n):
    skx, torch = _lib()
    _say(f"case: evaluate on {n}")
    _eval_vs_oracle(skx, torch, _uneven(n))


def test_uneven_grid_optimize_matches_oracle():
    skx, torch = _lib()
    from oracle.functional import Problem
    from oracle.optimize import optimize
    s = _uneven((12, 16, 20))
    _say("case: optimize on 12x16x20")
    ref = optimize(Problem(s), gtol=1e-9, max_iter=400)
    c = skx.Context(0).setup(s)
    rho, r = c.optimize(gtol=1e-9, max_iter=400)
    assert r["status"] == skx.OK
    assert abs(r["energy"]["free_energy"] - ref["energy"]["free_energy"]) < 1e-10 * abs(
        ref["energy"]["free_energy"])
    n = rho.cpu().numpy()
    assert np.sum(np.abs(n - ref["n"])) / np.sum(ref["n"]) < 1e-6


@pytest.mark.parametrize("case", ["single_ion", "beta0", "alpha1"])
def test_functional_variants(case):
    skx, torch = _lib()
    _say(f"case: functional variant {case}")
    if case == "single_ion":
        s = W.uniform_system(1, 1.0, 0.3, 2.0, 1.0, 16, seed=5)
    elif case == "beta0":
        s = W.uniform_system(6, 1.0, 0.4, 2.0, 1.0, 16, seed=6, beta=0.0)
    else:
        s = W.uniform_system(6, 1.0, 0.4, 2.0, 1.0, 16, seed=7, alpha=1.0)
    _eval_vs_oracle(skx, torch, s)


def test_warm_start_from_the_solution_stays():
    skx, _ = _lib()
    s = W.uniform_system(6, 1.0, 0.4, 2.0, 1.0, 16, seed=8)
    _say("case: warm start")
    c = skx.Context(0).setup(s)
    rho, r = c.optimize(gtol=1e-9, max_iter=400)
    rho2, r2 = c.optimize(gtol=1e-9, max_iter=400, rho0=rho)
    assert r2["status"] == skx.OK and r2["iters"] <= 2
    assert abs(r2["energy"]["free_energy"] - r["energy"]["free_energy"]) < 1e-10 * abs(
        r["energy"]["free_energy"])


def test_error_codes():
    skx, torch = _lib()
    _say("case: error codes")
    c = skx.Context(0)
    for bad in ((15, 16, 16), (14, 14, 14), (6, 6, 6), (1024, 8, 8)):
        with pytest.raises(skx.SkxError) as ex:
            c.set_cell(10.0, bad)
        assert ex.value.code == skx.E_INVALID
    c2 = skx.Context(0)
    with pytest.raises(skx.SkxError) as ex:
        c2.set_ions(np.zeros((1, 3)), [1.0], [0.3])
    assert ex.value.code == skx.E_STATE
    c2.set_cell(10.0, (16, 16, 16))
    with pytest.raises(skx.SkxError) as ex:
        c2.evaluate(torch.ones((16, 16, 16), dtype=torch.float64, device="cuda"))
    assert ex.value.code == skx.E_STATE
    with pytest.raises(skx.SkxError) as ex:
        c2.set_ions(np.zeros((1, 3)), [1.0], [-0.3])
    assert ex.value.code == skx.E_INVALID
    # pass B's x tile of an FP64 320-point x axis (4 fields x 320 x 9
    # complex) does not fit in LDS: large y-z planes are split, x pencils
    # are not
    s = dataclasses.replace(W.uniform_system(4, 1.0, 0.4, 2.0, 1.0, 8, seed=9), n=(320, 8, 8))
    c3 = skx.Context(0).setup(s, precision=skx.FP64)
    with pytest.raises(skx.SkxError) as ex:
        c3.evaluate(torch.ones(s.n, dtype=torch.float64, device="cuda"))
    assert ex.value.code == skx.E_INVALID
    c4 = skx.Context(0).setup(W.uniform_system(4, 1.0, 0.4, 2.0, 1.0, 16, seed=9))
    with pytest.raises(skx.SkxError) as ex:
        c4.optimize(m=9)
    assert ex.value.code == skx.E_INVALID


def test_max_iter_returns_the_best_state_and_non_cubic_cells_are_refused():
    skx, torch = _lib()
    _say("case: max_iter reached, non-cubic lattice")
    s = W.uniform_system(6, 1.0, 0.4, 2.0, 1.0, 16, seed=12)
    for prec in (skx.FP64, skx.MIXED):
        c = skx.Context(0).setup(s, precision=prec)
        rho, r = c.optimize(gtol=1e-12, max_iter=3)
        assert r["status"] == skx.NOT_CONVERGED
        assert np.isfinite(r["energy"]["free_energy"]) and r["gnorm"] > 1e-12
        dV = s.L ** 3 / np.prod(s.n)
        assert abs(float(rho.sum()) * dV - s.nelec) < 1e-9 * s.nelec
    import ctypes as C
    from paper_2601_23002_amd.skx import _lib as lib
    c = skx.Context(0)
    for lat in ((8.0, 0, 0, 0, 8.0, 0, 0, 0, 9.0), (8.0, 0.5, 0, 0, 8.0, 0, 0, 0, 8.0)):
        arr = (C.c_double * 9)(*lat)
        assert lib.skx_set_cell(c._h, arr, 16, 16, 16) == skx.E_INVALID
