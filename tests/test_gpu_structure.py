"""Static structure factors through the C ABI (skx_structure_factors)
against the oracle on the same FP64 densities and ions: shell counts exact,
S_ei, S_ee, S_ii to 1e-10 of each array's largest value (the FP64 target of
the path), on non-cubic and cubic grids with Nyquist planes in every axis,
and on the GPU minimum of the 64-ion 64^3 scan case.
"""
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


def _compare(got, ref):
    ei, ee, ii, cnt = got
    rei, ree, rii, rcnt = ref
    assert np.array_equal(cnt, rcnt)
    for a, b in ((ei, rei), (ee, ree), (ii, rii)):
        assert np.max(np.abs(a - b)) < 1e-10 * np.max(np.abs(b))


@pytest.mark.parametrize("n", [(16, 24, 20), (24, 24, 24)])
def test_structure_factors_match_oracle(n):
    skx, torch = _lib()
    from oracle import structure
    _say(f"case: structure factors grid {n}")
    rng = np.random.default_rng(51)
    zval = rng.choice([1.0, 4.0], 5)
    rc = np.where(zval > 1.0, 0.5, 0.3)
    L = W.cell_side(float(np.sum(zval)), 1.5)
    pos = rng.uniform(0.0, L, size=(5, 3))
    dens = 0.02 + 0.3 * rng.random(n)
    c = skx.Context(0)
    c.set_cell(L, n)
    c.set_ions(pos, zval, rc)
    rho = torch.tensor(dens, dtype=torch.float64, device="cuda:0")
    got = c.structure_factors(rho, kind=skx.RHO)
    _compare(got, structure.structure_factors(L, n, dens, pos, float(np.sum(zval))))
    got2 = c.structure_factors(torch.sqrt(rho), kind=skx.SQRT_RHO)
    for a, b in zip(got, got2):
        assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(a)))


def test_structure_factors_of_the_scan_minimum():
    skx, torch = _lib()
    from oracle import structure
    _say("case: structure factors 64 ions 64^3 at the GPU minimum")
    s = W.uniform_system(64, 1.0, 0.3, 2.0, 2.0, 64, seed=2)
    c = skx.Context(0).setup(s, precision=skx.FP64)
    rho, r = c.optimize(gtol=1e-8, max_iter=500)
    assert r["status"] == skx.OK
    got = c.structure_factors(rho)
    ref = structure.structure_factors(s.L, s.n, rho.cpu().numpy(), s.pos, float(np.sum(s.zval)))
    _compare(got, ref)
    # the screening cloud: S_ei is positive on the first shells
    assert got[0][1] > 0 and got[0][2] > 0


def test_structure_factor_errors():
    skx, torch = _lib()
    _say("case: structure factor errors")
    from paper_2601_23002_amd.skx import _lib as lib, _VP
    c = skx.Context(0)
    c.set_cell(7.0, (16, 16, 16))
    rho = torch.full((16, 16, 16), 0.1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(skx.SkxError) as e:
        c.structure_factors(rho)
    assert e.value.code == skx.E_STATE
    c.set_ions(np.array([[1.0, 2.0, 3.0]]), [1.0], [0.3])
    ns = lib.skx_num_shells(c._h)
    out = np.zeros(ns)
    import ctypes as C
    p = out.ctypes.data_as(C.POINTER(C.c_double))
    assert lib.skx_structure_factors(c._h, _VP(rho.data_ptr()), skx.RHO, p, None, None, None,
                                     ns - 1) == skx.E_INVALID
    assert lib.skx_structure_factors(c._h, _VP(rho.data_ptr()), skx.RHO, None, None, None, None,
                                     ns) == skx.E_INVALID
    assert lib.skx_structure_factors(c._h, None, skx.RHO, p, None, None, None, ns) == skx.E_INVALID


def test_structure_factors_at_the_largest_serving_size_on_sampled_shells():
    """192^3 with 1024 ions: every shell from the GPU, a sample of shells
    (small and large |q|) from the oracle's direct sums."""
    skx, torch = _lib()
    from oracle import structure
    _say("case: structure factors 1024 ions 192^3, sampled shells")
    n = (192, 192, 192)
    rng = np.random.default_rng(96)
    zval = np.where(rng.random(1024) < 0.5, 1.0, 4.0)
    rc = np.where(zval > 1.0, 0.5, 0.3)
    L = W.cell_side(float(np.sum(zval)), 2.5)
    pos = rng.uniform(0.0, L, size=(1024, 3))
    dens = 0.01 + 0.05 * rng.random(n)
    c = skx.Context(0)
    c.set_cell(L, n)
    c.set_ions(pos, zval, rc)
    rho = torch.tensor(dens, dtype=torch.float64, device="cuda:0")
    ei, ee, ii, cnt = c.structure_factors(rho)
    shells = (1, 2, 3, 14, 200, 9216, 27648)
    for sh, (rei, ree, rii, rc_) in zip(shells, structure.structure_factors_at(
            L, n, dens, pos, float(np.sum(zval)), shells)):
        assert cnt[sh] == rc_
        assert abs(ei[sh] - rei) < 1e-10 * max(abs(rei), 1e-3 * np.max(np.abs(ei[1:])))
        assert abs(ee[sh] - ree) < 1e-10 * max(abs(ree), 1e-3 * np.max(np.abs(ee[1:])))
        assert abs(ii[sh] - rii) < 1e-10 * abs(rii)
