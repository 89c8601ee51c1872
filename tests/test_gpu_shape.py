"""The compile-time-shaped pass kernels (36^3-80^3 grids, and pass B alone at
the large serving lengths 144^3-192^3) against the oracle and against the
runtime-shaped kernels.

Passes A and C fold the real DC and Nyquist columns of each plane into one
complex y transform, so they round differently from the runtime-shaped
kernels; both must meet the oracle tolerances (FP64 1e-10 relative on every
energy term, FP32 2e-5), and whole optimisations must reach the same
minimum.
"""
import sys

import numpy as np
import pytest

from paper_2601_23002_amd import workloads as W

pytestmark = pytest.mark.gpu

TERMS = ("f_tf", "e_vw", "f_nl0", "f_nl1", "e_h", "e_loc", "e_xc")


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2601_23002_amd import skx
    return skx, torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _eval(skx, torch, s, phi, prec, shape):
    old = skx.set_shape_kernels(shape)
    try:
        c = skx.Context(0).setup(s, precision=prec)
        dt = torch.float32 if prec == skx.FP32 else torch.float64
        e, g = c.evaluate(torch.tensor(phi, dtype=dt, device="cuda"), skx.SQRT_RHO)
        return e, g.double().cpu().numpy()
    finally:
        skx.set_shape_kernels(old)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shape64_evaluation_matches_oracle(precision):
    skx, torch = _lib()
    from oracle.functional import Problem
    prec = skx.FP64 if precision == "fp64" else skx.FP32
    tol = 1e-10 if precision == "fp64" else 2e-5
    s = W.uniform_system(64, 1.0, 0.3, 2.0, 2.0, 64, seed=21, beta=1.3)
    phi = W.random_phi(s, 22, amp=0.4)
    _say(f"case: 64^3 evaluation, shape kernels, {precision}")
    e_ref, g_ref = Problem(s).evaluate(phi)
    scale = sum(abs(e_ref[k]) for k in TERMS)
    for shape in (7, 1, 2, 4, 0):                 # all, each pass alone, none
        e, g = _eval(skx, torch, s, phi, prec, shape)
        for k in TERMS:
            assert abs(e[k] - e_ref[k]) <= tol * max(abs(e_ref[k]), 1e-3 * scale), (shape, k)
        assert abs(e["mu"] - e_ref["mu"]) <= tol * max(1.0, abs(e_ref["mu"])) * 10, shape
        assert np.max(np.abs(g - g_ref)) <= tol * np.max(np.abs(g_ref)) * 10, shape


@pytest.mark.parametrize("beta,terms", [(0.0, W.TERM_ALL),
                                        (1.3, W.TERM_ALL & ~W.TERM_VW),
                                        (1.3, W.TERM_TF | W.TERM_HARTREE | W.TERM_LOCPP)])
def test_shape64_field_subsets_match_oracle(beta, terms):
    """Absent fields (no h with beta = 0, no phi without vW, neither f nor h
    without the nonlocal terms) leave spectrum slots unused; every pass of
    the shape kernels must skip them consistently (FP64 1e-10, FP32 2e-5;
    FP32 pass C streams the next present field's plane while transforming
    the current one)."""
    skx, torch = _lib()
    from oracle.functional import Problem
    s = W.uniform_system(64, 1.0, 0.3, 2.0, 2.0, 64, seed=27, beta=beta, terms=terms)
    phi = W.random_phi(s, 28, amp=0.4)
    _say(f"case: 64^3 shape kernels, beta={beta}, terms={terms}")
    e_ref, g_ref = Problem(s).evaluate(phi)
    scale = sum(abs(e_ref[k]) for k in TERMS)
    for prec, tol in ((skx.FP64, 1e-10), (skx.FP32, 2e-5)):
        e, g = _eval(skx, torch, s, phi, prec, 7)
        for k in TERMS:
            assert abs(e[k] - e_ref[k]) <= tol * max(abs(e_ref[k]), 1e-3 * scale), (prec, k, e[k], e_ref[k])
        assert np.max(np.abs(g - g_ref)) <= tol * 10 * np.max(np.abs(g_ref)), prec


def test_shape64_sampled_gradient_points():
    """Every point class of the register-resident assembly (each lane's two
    rows and R1 z offsets, every wavefront's row pairs) on one plane: the
    FP64 gradient of the shape kernel equals the runtime-shaped kernel's to
    rounding on all 64 x 64 points of several planes."""
    skx, torch = _lib()
    s = W.uniform_system(64, 1.0, 0.3, 1.0, 0.5, 64, seed=23)
    phi = W.random_phi(s, 24, amp=0.5)
    _say("case: 64^3 shape vs runtime kernels, all points")
    _, g1 = _eval(skx, torch, s, phi, skx.FP64, True)
    _, g0 = _eval(skx, torch, s, phi, skx.FP64, False)
    scale = np.max(np.abs(g0))
    assert np.max(np.abs(g1 - g0)) <= 1e-12 * scale


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_shape64_optimisation_reaches_same_minimum(precision):
    skx, torch = _lib()
    prec = skx.FP64 if precision == "fp64" else skx.MIXED
    s = W.uniform_system(64, 1.0, 0.3, 2.0, 2.0, 64, seed=25)
    out = {}
    for shape in (True, False):
        _say(f"case: 64^3 optimise {precision}, shape kernels {shape}")
        old = skx.set_shape_kernels(shape)
        try:
            c = skx.Context(0).setup(s, precision=prec)
            rho, res = c.optimize(gtol=1e-8)
        finally:
            skx.set_shape_kernels(old)
        assert res["status"] == 0, res
        out[shape] = (res["energy"]["free_energy"], rho.cpu().numpy())
    (e1, r1), (e0, r0) = out[True], out[False]
    assert abs(e1 - e0) / 64 <= 1e-9              # far inside 1e-6 Ha/atom
    assert np.max(np.abs(r1 - r0)) <= 1e-5 * np.max(np.abs(r0))


# ----------------------------------------------------------------------------
# The other compile-time lengths (radix orders 4-3-3, 8-5, 8-3-2, 2-5-5,
# 2-3-3-3, 4-3-5, 8-3-3, 8-5-2; pass B on the shaped kernel with whole column
# blocks below the Nyquist column at 48 and 80, and ragged blocks whose last
# one holds the Nyquist column at 36, 40, 50, 54, 60, 72)
# ----------------------------------------------------------------------------
SHAPED = [36, 40, 48, 50, 54, 60, 72, 80]
_ORACLE = {}


def _shaped_case(n):
    if n not in _ORACLE:
        from oracle.functional import Problem
        s = W.uniform_system(max(8, n * n * n // 4096), 1.0, 0.3, 2.0, 2.0, n, seed=30 + n,
                             beta=1.3)
        phi = W.random_phi(s, 31 + n, amp=0.4)
        _ORACLE[n] = (s, phi) + Problem(s).evaluate(phi)
    return _ORACLE[n]


@pytest.mark.parametrize("n", SHAPED)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shaped_lengths_match_oracle(n, precision):
    skx, torch = _lib()
    prec = skx.FP64 if precision == "fp64" else skx.FP32
    tol = 1e-10 if precision == "fp64" else 2e-5
    _say(f"case: {n}^3 evaluation, shape kernels, {precision}")
    s, phi, e_ref, g_ref = _shaped_case(n)
    scale = sum(abs(e_ref[k]) for k in TERMS)
    for shape in (7, 5, 0):                       # all, passes A and C, none
        e, g = _eval(skx, torch, s, phi, prec, shape)
        for k in TERMS:
            assert abs(e[k] - e_ref[k]) <= tol * max(abs(e_ref[k]), 1e-3 * scale), (shape, k)
        assert abs(e["mu"] - e_ref["mu"]) <= tol * max(1.0, abs(e_ref["mu"])) * 10, shape
        assert np.max(np.abs(g - g_ref)) <= tol * np.max(np.abs(g_ref)) * 10, shape


@pytest.mark.parametrize("n", SHAPED)
def test_shaped_lengths_equal_runtime_kernels_at_every_point(n):
    """FP64 gradient of the shaped kernels against the runtime-shaped ones on
    every grid point (1e-12 of the gradient's scale), with beta = 0 and no
    vW term as well (absent fields skipped consistently)."""
    skx, torch = _lib()
    for beta, terms in ((1.3, W.TERM_ALL), (0.0, W.TERM_ALL & ~W.TERM_VW)):
        s = W.uniform_system(16, 1.0, 0.3, 2.0, 2.0, n, seed=40 + n, beta=beta, terms=terms)
        phi = W.random_phi(s, 41 + n, amp=0.5)
        _say(f"case: {n}^3 shape vs runtime kernels, beta {beta}, terms {terms}")
        e1, g1 = _eval(skx, torch, s, phi, skx.FP64, 7)
        e0, g0 = _eval(skx, torch, s, phi, skx.FP64, 0)
        assert np.max(np.abs(g1 - g0)) <= 1e-12 * np.max(np.abs(g0))
        for k in TERMS:
            assert abs(e1[k] - e0[k]) <= 1e-12 * max(1.0, abs(e0[k])), k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_shaped_lengths_optimisation_reaches_same_minimum(precision):
    """A batch over every kernel family (36, 54, 72, 80 shaped; 90 runtime):
    solved with the shaped kernels on and off, each solve reaches the same
    minimum (far inside 1e-6 Ha/atom)."""
    skx, torch = _lib()
    prec = skx.FP64 if precision == "fp64" else skx.MIXED
    systems = [W.uniform_system(12, 1.0, 0.3, 2.0, 2.0, n, seed=50 + n) for n in (36, 54, 72, 80, 90)]
    out = {}
    for shape in (7, 0):
        _say(f"case: shaped lengths, batched {precision} solves, shape kernels {shape}")
        old = skx.set_shape_kernels(shape)
        try:
            ctxs = [skx.Context(0).setup(x, precision=prec) for x in systems]
            rhos = [torch.empty(x.n, dtype=torch.float64, device="cuda") for x in systems]
            res = skx.run_batch(ctxs, rhos, gtol=1e-8, max_iter=1000)
        finally:
            skx.set_shape_kernels(old)
        assert all(r["status"] == skx.OK for r in res), res
        out[shape] = [(r["energy"]["free_energy"], x.cpu().numpy()) for r, x in zip(res, rhos)]
    for (e1, r1), (e0, r0), x in zip(out[7], out[0], systems):
        assert abs(e1 - e0) / len(x.zval) <= 1e-9
        assert np.max(np.abs(r1 - r0)) <= 1e-5 * np.max(np.abs(r0))


# ----------------------------------------------------------------------------
# Larger serving lengths (90, 96, 100, 108, 120, 128, 144, 150, 160, 162,
# 180, 192): pass B
# alone on the compile-time-shaped kernel (FP64 blocks of 4, FP32 of 16 up
# to 144 and 8 beyond; ragged where the width does not divide N/2 or the
# Nyquist column's first stage would not fit, else whole blocks and the
# Nyquist column on its own workgroups), passes A and C on the in-LDS
# runtime-shaped or the split kernels. The oracle takes minutes per
# evaluation at the largest sizes, so the shaped pass B is held to the
# runtime-shaped one, which the oracle pins on large planes
# (test_gpu_bigplane.py), at every grid point.
# ----------------------------------------------------------------------------
LARGE_B = [90, 96, 100, 108, 120, 128, 144, 150, 160, 162, 180, 192]


@pytest.mark.parametrize("n", LARGE_B)
def test_large_shaped_pass_b_equals_runtime_kernel_at_every_point(n):
    """FP64: gradient within 1e-12 of its scale, every energy term within
    1e-12 relative; FP32: within 2e-5 of the FP64 runtime result (both
    precisions' shaped pass B against the runtime one), with beta = 0 and no
    vW term as well."""
    skx, torch = _lib()
    for beta, terms in ((1.3, W.TERM_ALL), (0.0, W.TERM_ALL & ~W.TERM_VW)):
        s = W.uniform_system(16, 1.0, 0.3, 2.0, 2.0, n, seed=60 + n, beta=beta, terms=terms)
        phi = W.random_phi(s, 61 + n, amp=0.4)
        _say(f"case: {n}^3 shaped pass B vs runtime, beta {beta}, terms {terms}")
        e1, g1 = _eval(skx, torch, s, phi, skx.FP64, 7)
        e0, g0 = _eval(skx, torch, s, phi, skx.FP64, 0)
        scale = np.max(np.abs(g0))
        assert np.max(np.abs(g1 - g0)) <= 1e-12 * scale
        for k in TERMS:
            assert abs(e1[k] - e0[k]) <= 1e-12 * max(1.0, abs(e0[k])), k
        escale = sum(abs(e0[k]) for k in TERMS)
        for shape in (7, 0):
            e, g = _eval(skx, torch, s, phi, skx.FP32, shape)
            for k in TERMS:
                assert abs(e[k] - e0[k]) <= 2e-5 * max(abs(e0[k]), 1e-3 * escale), (shape, k)
            assert np.max(np.abs(g - g0)) <= 2e-4 * scale, shape


def test_large_shaped_pass_b_optimisation_reaches_same_minimum():
    """A mixed-precision batch of a 144^3 and a 160^3 solve with the shaped
    pass B on and off reaches the same minimum (far inside 1e-6 Ha/atom);
    the preconditioner's pass B runs on the shaped kernel too."""
    skx, torch = _lib()
    systems = [W.uniform_system(16, 1.0, 0.3, 2.0, 2.0, n, seed=70 + n) for n in (144, 160)]
    out = {}
    for shape in (7, 0):
        _say(f"case: 144^3 + 160^3 mixed batch, shape kernels {shape}")
        old = skx.set_shape_kernels(shape)
        try:
            ctxs = [skx.Context(0).setup(x, precision=skx.MIXED) for x in systems]
            rhos = [torch.empty(x.n, dtype=torch.float64, device="cuda") for x in systems]
            res = skx.run_batch(ctxs, rhos, gtol=1e-8, max_iter=1000)
        finally:
            skx.set_shape_kernels(old)
        assert all(r["status"] == skx.OK for r in res), res
        out[shape] = [(r["energy"]["free_energy"], x.cpu().numpy()) for r, x in zip(res, rhos)]
    for (e1, r1), (e0, r0), x in zip(out[7], out[0], systems):
        assert abs(e1 - e0) / len(x.zval) <= 1e-9
        assert np.max(np.abs(r1 - r0)) <= 1e-5 * np.max(np.abs(r0))


@pytest.mark.parametrize("n", [160, 192])
def test_large_grid_potential_matches_energy_finite_difference(n):
    """At the large serving lengths (split passes A and C, shaped pass B)
    the FP64 potential is the derivative of the FP64 energy: dV sum(dE/dphi d)
    against a fourth-order central difference of E along a smooth direction
    d, to 1e-7 of its scale (the difference quotient's rounding is about
    1e-9 of it here). A property that holds at any size, checked where the
    oracle would need minutes per evaluation."""
    skx, torch = _lib()
    s = W.uniform_system(32, 1.0, 0.3, 2.0, 2.0, n, seed=90 + n, beta=1.3)
    phi = W.random_phi(s, 91 + n, amp=0.4)
    d = W.random_phi(s, 92 + n, amp=0.5) - W.random_phi(s, 93 + n, amp=0.5)
    _say(f"case: {n}^3 FP64 potential against energy differences")
    c = skx.Context(0).setup(s, precision=skx.FP64)

    def ev(x, grad=True):
        return c.evaluate(torch.tensor(x, dtype=torch.float64, device="cuda"), skx.SQRT_RHO,
                          want_grad=grad)

    e, g = ev(phi)
    an = s.volume / s.M * float(np.sum(g.double().cpu().numpy() * d))
    eps = 2e-4
    E = lambda t: ev(phi + t * d, grad=False)[0]["free_energy"]
    fd = (-E(2 * eps) + 8 * E(eps) - 8 * E(-eps) + E(-2 * eps)) / (12 * eps)
    scale = max(abs(an), 1e-3 * abs(e["free_energy"]))
    assert abs(fd - an) <= 1e-7 * scale, (n, fd, an)
