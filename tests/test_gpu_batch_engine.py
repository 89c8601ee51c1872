"""Batched solves and the serving engine (through the C ABI).

A solve's arithmetic must not depend on which other solves share its
launches: batched and engine results are compared bit for bit with the same
solve run alone. Mixed-precision solves are compared with the FP64 oracle
at the stated accuracy (1e-6 Ha/atom in energy, 1e-5 relative in density).
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


def _c1(s):
    # densities near the ions of these dense systems reach r_s < 1: the
    # published PZ81 fit's jump at r_s = 1 would floor ||r||, so they take
    # the C1-joined branches (the oracle follows the same setting)
    s.xc = W.XC_PZ81_C1
    return s


def _systems():
    return [W.uniform_system(6, 1.0, 0.4, 2.0, 1.0, 12, seed=41),
            _c1(W.uniform_system(8, 1.0, 0.3, 1.5, 4.0, 16, seed=42)),
            _c1(W.uniform_system(3, 4.0, 0.5, 1.5, 4.0, 20, seed=43)),
            W.uniform_system(10, 1.0, 0.3, 3.0, 0.5, 16, seed=44, beta=0.5)]


def _alone(skx, s, precision, **kw):
    c = skx.Context(0).setup(s, precision=precision)
    rho, r = c.optimize(**kw)
    return rho.cpu().numpy(), r


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_run_batch_equals_alone(precision):
    skx, torch = _lib()
    prec = {"fp64": skx.FP64, "mixed": skx.MIXED}[precision]
    systems = _systems()
    _say(f"case: run_batch vs alone, {precision}, grids {[s.n[0] for s in systems]}")
    kw = dict(gtol=1e-9, max_iter=400, m=5, fp32_switch_gtol=1e-5)
    ctxs = [skx.Context(0).setup(s, precision=prec) for s in systems]
    rhos = [torch.empty(s.n, dtype=torch.float64, device="cuda") for s in systems]
    res = skx.run_batch(ctxs, rhos, **kw)
    for s, r, rho in zip(systems, res, rhos):
        n_a, r_a = _alone(skx, s, prec, **kw)
        assert r["status"] == skx.OK, r
        assert r["iters"] == r_a["iters"] and r["evals"] == r_a["evals"]
        assert r["energy"]["free_energy"] == r_a["energy"]["free_energy"]
        assert np.array_equal(rho.cpu().numpy(), n_a)


def test_mixed_matches_oracle():
    skx, torch = _lib()
    from oracle.functional import Problem
    from oracle.optimize import optimize
    for s in _systems()[:3]:
        _say(f"case: mixed vs oracle, n={s.n[0]}, N={len(s.zval)}")
        ref = optimize(Problem(s), gtol=1e-9, max_iter=600)
        n, r = _alone(skx, s, skx.MIXED, gtol=1e-9, max_iter=600, fp32_switch_gtol=1e-5)
        assert r["status"] == skx.OK, r
        assert r["fp32_iters"] > 0
        per_atom = abs(r["energy"]["free_energy"] - ref["energy"]["free_energy"]) / len(s.zval)
        assert per_atom < 1e-6
        assert np.sum(np.abs(n - ref["n"])) / np.sum(ref["n"]) < 1e-5


def test_fp32_phase_alone_within_single_precision():
    """An FP32-only solve already lands within the mixed-precision bar of the
    FP64 minimum for a moderate gtol."""
    skx, _ = _lib()
    s = _systems()[1]
    _say("case: fp32-only solve vs fp64 solve, n=16")
    n64, r64 = _alone(skx, s, skx.FP64, gtol=1e-9, max_iter=600)
    n32, r32 = _alone(skx, s, skx.FP32, gtol=1e-5, max_iter=600)
    assert r32["status"] in (skx.OK, skx.NOT_CONVERGED)
    assert abs(r32["energy"]["free_energy"] - r64["energy"]["free_energy"]) / len(s.zval) < 1e-6
    assert np.sum(np.abs(n32 - n64)) / np.sum(n64) < 1e-4


def test_engine_equals_alone_and_reports_latency():
    skx, _ = _lib()
    systems = _systems() + [W.uniform_system(5, 1.0, 0.3, 2.0, 2.0, 12, seed=45)]
    kw = dict(gtol=1e-9, max_iter=400, m=5, fp32_switch_gtol=1e-5)
    _say(f"case: engine, {len(systems)} requests, 2 slots")
    eng = skx.Engine(0, hbm_budget=1 << 30, max_slots=2)
    tickets = {}
    for i, s in enumerate(systems):
        prec = skx.FP64 if i == 2 else skx.MIXED
        tickets[eng.submit(s, precision=prec, **kw)] = (s, prec)
    done = []
    steps = 0
    while eng.pending() > 0 and steps < 5000:
        resident = eng.step()
        assert 0 <= resident <= 2
        done += eng.poll(want_density=True)
        steps += 1
    assert len(done) == len(systems)
    lat = []
    for d in done:
        s, prec = tickets[d["ticket"]]
        n_a, r_a = _alone(skx, s, prec, **kw)
        r = d["result"]
        assert r["status"] == skx.OK, r
        assert r["iters"] == r_a["iters"] and r["evals"] == r_a["evals"]
        assert r["energy"]["free_energy"] == r_a["energy"]["free_energy"]
        assert np.array_equal(d["rho"], n_a)
        assert 0.0 <= d["t_admit"] <= d["t_done"]
        lat.append(d["t_done"])
    p50, p99 = np.percentile(lat, [50, 99])
    assert 0 < p50 <= p99
    eng.close()


def test_engine_admission_limits():
    skx, _ = _lib()
    s = W.uniform_system(6, 1.0, 0.4, 2.0, 1.0, 32, seed=46)
    _say("case: engine budget")
    eng = skx.Engine(0, hbm_budget=1 << 20, max_slots=4)
    with pytest.raises(skx.SkxError):
        eng.submit(s)                       # 32^3 mixed needs far more than 1 MiB
    bad = W.uniform_system(6, 1.0, 0.4, 2.0, 1.0, 14, seed=46)
    with pytest.raises(skx.SkxError):
        eng.submit(bad)                     # 14 is not 5-smooth
    assert eng.pending() == 0
    eng.close()


def test_graph_replay_equals_eager():
    """The driver replays one captured graph per chunk of step sequences, with
    host polling and synchronisation between replays; every solve must end in
    the state of the eager launches, on repeated calls."""
    skx, torch = _lib()
    systems = _systems()
    kw = dict(gtol=1e-9, max_iter=400, m=5, fp32_switch_gtol=1e-5)
    out = {}
    old = skx.set_graphs(False)
    for graphs in (False, True, True):
        _say(f"case: run_batch mixed, graphs={graphs}")
        skx.set_graphs(graphs)
        ctxs = [skx.Context(0).setup(s, precision=skx.MIXED) for s in systems]
        rhos = [torch.empty(s.n, dtype=torch.float64, device="cuda") for s in systems]
        res = skx.run_batch(ctxs, rhos, **kw)
        key = [(r["iters"], r["evals"], r["energy"]["free_energy"]) for r in res]
        dens = [r.cpu().numpy() for r in rhos]
        if "eager" not in out:
            out["eager"] = (key, dens)
        else:
            assert key == out["eager"][0]
            for a, b in zip(dens, out["eager"][1]):
                assert np.array_equal(a, b)
    skx.set_graphs(old)


def test_mixed_precision_96cubed_beryllium_like():
    """128 Z=4 ions (rc 0.5 bohr), rs 1.5, T 4 Ha on 96^3: FP32 iterations then
    FP64 refinement. Against the plain FP64 GPU solve: 1e-6 Ha/atom and 1e-5
    relative density. Against the oracle, evaluated once at the mixed
    solution (a full oracle solve at this size takes hours): the energy to
    1e-10 relative, and the oracle's own constrained residual at that point
    is at the convergence threshold."""
    skx, _ = _lib()
    from oracle.functional import Problem
    s = _c1(W.config_mixed())
    _say("case: mixed precision 96^3, 128 Z=4 ions")
    gtol = 1e-8
    n_mx, r_mx = _alone(skx, s, skx.MIXED, gtol=gtol, max_iter=2000, fp32_switch_gtol=1e-5)
    assert r_mx["status"] == skx.OK, r_mx
    assert r_mx["fp32_iters"] > 0
    n_64, r_64 = _alone(skx, s, skx.FP64, gtol=gtol, max_iter=2000)
    assert r_64["status"] == skx.OK, r_64
    nat = len(s.zval)
    d_e = abs(r_mx["energy"]["free_energy"] - r_64["energy"]["free_energy"]) / nat
    d_n = np.sum(np.abs(n_mx - n_64)) / np.sum(n_64)
    _say(f"  mixed vs fp64: {d_e:.3e} Ha/atom, density {d_n:.3e}; "
         f"iters {r_mx['fp32_iters']}+{r_mx['iters'] - r_mx['fp32_iters']} vs {r_64['iters']}")
    assert d_e < 1e-6 and d_n < 1e-5
    p = Problem(s)
    phi = np.sqrt(n_mx)
    e, g = p.evaluate(phi)
    rel = abs(e["free_energy"] - r_mx["energy"]["free_energy"]) / abs(e["free_energy"])
    mu = p.dot(phi, g) / (2.0 * p.ne)
    res = g - 2.0 * mu * phi
    rn = np.sqrt(p.dot(res, res))
    _say(f"  oracle at the mixed solution: energy rel {rel:.3e}, |r| {rn:.3e}")
    assert rel < 1e-10
    assert rn < 2.0 * gtol


def test_thermal_ensemble_batch():
    """Uneven thermal-like snapshots (Z=1 and Z=4, 16..256 ions, grids from
    h = 0.25 bohr clamped to 16..48 here) solved in one batch; each equals
    its solve alone."""
    skx, torch = _lib()
    systems = [_c1(x) for x in W.config_ensemble(count=12, nmin=16, nmax=48)]
    _say(f"case: ensemble batch, grids {[s.n[0] for s in systems]}")
    kw = dict(gtol=1e-8, max_iter=1000, m=5, fp32_switch_gtol=1e-5)
    ctxs = [skx.Context(0).setup(s, precision=skx.MIXED) for s in systems]
    rhos = [torch.empty(s.n, dtype=torch.float64, device="cuda") for s in systems]
    res = skx.run_batch(ctxs, rhos, **kw)
    for i in (0, 5, 11):
        n_a, r_a = _alone(skx, systems[i], skx.MIXED, **kw)
        assert res[i]["status"] == skx.OK, res[i]
        assert res[i]["energy"]["free_energy"] == r_a["energy"]["free_energy"]
        assert np.array_equal(rhos[i].cpu().numpy(), n_a)
    assert all(r["status"] == skx.OK for r in res)


def test_engine_reused_contexts_equal_alone():
    """Requests of one grid through 2 slots: later requests run on the
    contexts of finished ones (kept by the engine); every result must still
    be bitwise the result of solving alone, including a request with a longer
    history (no reusable context) and one in FP64."""
    skx, _ = _lib()
    kw = dict(gtol=1e-9, max_iter=400, fp32_switch_gtol=1e-5)
    reqs = [(W.uniform_system(4, 1.0, 0.4, 2.0, T, 16, seed=70 + i), skx.MIXED, 5)
            for i, T in enumerate((0.5, 1.0, 2.0, 4.0))]
    reqs.append((W.uniform_system(4, 1.0, 0.4, 2.0, 1.5, 16, seed=75), skx.MIXED, 7))
    reqs.append((W.uniform_system(4, 1.0, 0.4, 2.0, 1.5, 16, seed=76), skx.FP64, 5))
    _say(f"case: engine context reuse, {len(reqs)} requests on 16^3, 2 slots")
    eng = skx.Engine(0, hbm_budget=1 << 30, max_slots=2)
    tickets = {}
    for s, prec, m in reqs:
        tickets[eng.submit(s, precision=prec, m=m, **kw)] = (s, prec, m)
    done = []
    steps = 0
    while eng.pending() > 0 and steps < 5000:
        eng.step()
        done += eng.poll(want_density=True)
        steps += 1
    assert len(done) == len(reqs)
    for d in done:
        s, prec, m = tickets[d["ticket"]]
        n_a, r_a = _alone(skx, s, prec, m=m, **kw)
        r = d["result"]
        assert r["status"] == skx.OK, r
        assert r["iters"] == r_a["iters"] and r["evals"] == r_a["evals"]
        assert r["energy"]["free_energy"] == r_a["energy"]["free_energy"]
        assert np.array_equal(d["rho"], n_a)
    eng.close()


def test_engine_cancel_frees_the_slot_and_leaves_others_alone():
    skx, _ = _lib()
    kw = dict(gtol=1e-9, max_iter=400, fp32_switch_gtol=1e-5)
    reqs = [W.uniform_system(4, 1.0, 0.4, 2.0, T, 16, seed=80 + i)
            for i, T in enumerate((0.5, 1.0, 2.0, 4.0))]
    _say("case: engine cancel, 4 requests on 16^3, 2 slots")
    eng = skx.Engine(0, hbm_budget=1 << 30, max_slots=2)
    t = [eng.submit(s, precision=skx.MIXED, **kw) for s in reqs]
    assert eng.step() == 2                  # two resident, two queued
    eng.cancel(t[0])                        # resident
    eng.cancel(t[3])                        # queued
    with pytest.raises(skx.SkxError) as e:
        eng.cancel(t[0])                    # no longer queued or resident
    assert e.value.code == skx.E_INVALID
    done = []
    steps = 0
    while eng.pending() > 0 and steps < 5000:
        eng.step()
        done += eng.poll(want_density=True)
        steps += 1
    by = {d["ticket"]: d for d in done}
    assert sorted(by) == sorted(t)
    for k in (0, 3):
        assert by[t[k]]["result"]["status"] == skx.CANCELLED and "rho" not in by[t[k]]
    for k in (1, 2):
        n_a, r_a = _alone(skx, reqs[k], skx.MIXED, **kw)
        r = by[t[k]]["result"]
        assert r["status"] == skx.OK
        assert r["iters"] == r_a["iters"] and r["energy"]["free_energy"] == r_a["energy"]["free_energy"]
        assert np.array_equal(by[t[k]]["rho"], n_a)
    eng.close()
