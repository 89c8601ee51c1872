"""Passes A and C on the split kernels (z transforms over row-pair chunks and
y transforms over column chunks, in separate launches), for planes whose
half spectrum does not fit in LDS (FP64 beyond 128 x 128, FP32 beyond
192 x 192) and the sizes where they were measured faster.

The split kernels are checked against the oracle on small grids with the
split forced (one and several row-pair chunks per plane, ragged last column
chunks, absent fields), on planes that need it (FP64 8 x 144 x 144, FP32
8 x 216 x 216: large planes at an oracle cost of seconds), and through whole
optimisations (forced against natural on 32^3; mixed against FP64 on
8 x 144 x 144, which exercises the split preconditioner passes too).
"""
import dataclasses
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


def _flat_system(n1, n, seed, nions=24, rs=2.0, T=2.0):
    s = W.uniform_system(nions, 1.0, 0.3, rs, T, n, seed=seed, beta=1.3)
    return dataclasses.replace(s, n=(n1, n, n))


def _check(skx, torch, s, phi, prec, tol):
    from oracle.functional import Problem
    e_ref, g_ref = Problem(s).evaluate(phi)
    c = skx.Context(0).setup(s, precision=prec)
    dt = torch.float32 if prec == skx.FP32 else torch.float64
    e, g = c.evaluate(torch.tensor(phi, dtype=dt, device="cuda"), skx.SQRT_RHO)
    g = g.double().cpu().numpy()
    scale = sum(abs(e_ref[k]) for k in TERMS)
    for k in TERMS:
        assert abs(e[k] - e_ref[k]) <= tol * max(abs(e_ref[k]), 1e-3 * scale), (k, e[k], e_ref[k])
    assert abs(e["mu"] - e_ref["mu"]) <= tol * max(1.0, abs(e_ref["mu"])) * 10
    assert np.max(np.abs(g - g_ref)) <= tol * np.max(np.abs(g_ref)) * 10


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_forced_chunking_matches_oracle(precision):
    skx, torch = _lib()
    prec = skx.FP64 if precision == "fp64" else skx.FP32
    tol = 1e-10 if precision == "fp64" else 2e-5
    for n in (24, 30):
        s = W.uniform_system(6, 1.0, 0.4, 2.0, 1.0, n, seed=n, beta=1.3)
        phi = W.random_phi(s, n + 1, amp=0.4)
        _say(f"case: split planes forced, {precision}, {n}^3")
        old = skx.set_plane_chunking(True)
        try:
            _check(skx, torch, s, phi, prec, tol)
        finally:
            skx.set_plane_chunking(old)


@pytest.mark.parametrize("beta,terms", [(0.0, W.TERM_ALL & ~W.TERM_VW),
                                        (1.3, W.TERM_TF | W.TERM_HARTREE | W.TERM_LOCPP)])
def test_forced_split_field_subsets_match_oracle(beta, terms):
    """Absent fields (no h with beta = 0, no phi without vW, neither f nor h
    without the nonlocal terms) leave spectrum slots unused; the split
    kernels' field loops and column-chunk items must skip them consistently.
    A 40-point z axis gives two row-pair chunks per plane (16 and 4 row pairs)
    and a ragged last column chunk (21 columns: 8 + 8 + 5 in FP64, 16 + 5 in
    FP32)."""
    skx, torch = _lib()
    for n1, prec, tol in ((40, skx.FP64, 1e-10), (16, skx.FP32, 2e-5)):
        s = dataclasses.replace(W.uniform_system(8, 1.0, 0.4, 2.0, 1.0, 40, seed=51, beta=beta,
                                                 terms=terms), n=(n1, 40, 40))
        phi = W.random_phi(s, 52, amp=0.4)
        _say(f"case: split planes forced, {n1}x40x40, beta={beta}, terms={terms}, prec {prec}")
        old = skx.set_plane_chunking(True)
        try:
            _check(skx, torch, s, phi, prec, tol)
        finally:
            skx.set_plane_chunking(old)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_forced_split_uneven_grid_matches_oracle(precision):
    """Rows, columns and x pencils of three different lengths (10 x 24 x 40:
    z transforms of 40 points in one row-pair chunk of 12 pairs, y transforms
    of 24 points over column chunks of 21 columns)."""
    skx, torch = _lib()
    prec = skx.FP64 if precision == "fp64" else skx.FP32
    tol = 1e-10 if precision == "fp64" else 2e-5
    s = dataclasses.replace(W.uniform_system(6, 1.0, 0.4, 2.0, 1.0, 24, seed=53, beta=1.3),
                            n=(10, 24, 40))
    phi = W.random_phi(s, 54, amp=0.4)
    _say(f"case: split planes forced, 10x24x40, {precision}")
    old = skx.set_plane_chunking(True)
    try:
        _check(skx, torch, s, phi, prec, tol)
    finally:
        skx.set_plane_chunking(old)


def test_forced_chunking_optimisation_same_minimum():
    skx, torch = _lib()
    s = W.uniform_system(16, 1.0, 0.3, 2.0, 1.0, 32, seed=31)
    out = {}
    for force in (True, False):
        _say(f"case: 32^3 FP64 optimise, split forced {force}")
        old = skx.set_plane_chunking(force)
        try:
            c = skx.Context(0).setup(s, precision=skx.FP64)
            rho, res = c.optimize(gtol=1e-8)
        finally:
            skx.set_plane_chunking(old)
        assert res["status"] == 0, res
        out[force] = (res["energy"]["free_energy"], rho.cpu().numpy())
    (e1, r1), (e0, r0) = out[True], out[False]
    assert abs(e1 - e0) / 16 <= 1e-9
    assert np.max(np.abs(r1 - r0)) <= 1e-6 * np.max(np.abs(r0))


@pytest.mark.parametrize("precision,n", [("fp64", 144), ("fp32", 216)])
def test_large_plane_matches_oracle(precision, n):
    skx, torch = _lib()
    prec = skx.FP64 if precision == "fp64" else skx.FP32
    tol = 1e-10 if precision == "fp64" else 2e-5
    s = _flat_system(8, n, seed=41)
    phi = W.random_phi(s, 42, amp=0.4)
    _say(f"case: large plane {precision} 8x{n}x{n}")
    _check(skx, torch, s, phi, prec, tol)


def test_large_plane_mixed_optimisation():
    skx, torch = _lib()
    s = _flat_system(8, 144, seed=43)
    out = {}
    for name, prec in (("fp64", skx.FP64), ("mixed", skx.MIXED)):
        _say(f"case: 8x144x144 optimise {name}")
        c = skx.Context(0).setup(s, precision=prec)
        rho, res = c.optimize(gtol=1e-8)
        assert res["status"] == 0, (name, res)
        out[name] = (res["energy"]["free_energy"], rho.cpu().numpy())
    (e64, r64), (em, rm) = out["fp64"], out["mixed"]
    nion = len(s.zval)
    assert abs(em - e64) / nion <= 1e-6
    assert np.max(np.abs(rm - r64)) <= 1e-5 * np.max(np.abs(r64))
