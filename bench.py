#!/usr/bin/env python3
"""Throughput of the batched mixed-precision OFDFT solve on one MI355X.

One step = one batched solve, through the C-ABI library, of the scan
workload: 9 independent systems of 64 Z=1 ions (erf pseudopotential,
rc = 0.3 bohr) at rs in {1,2,4} bohr x T in {0.5,2,8} Ha on 64^3 grids,
uniform random positions (seeds 2..10). Every step runs every hot-path row:
structure factor and kernel tables (set-up of each solve), then the
optimiser with its fused FFT/functional evaluations, FP32 until
||r|| < 1e-5 and FP64 refinement to ||r|| < 1e-8.

Metric: grid-point functional evaluations per second,
sum over solves of (evaluations x grid points) / wall time of the step.
The plain FP64 GPU path is timed on the same workload for the speedup,
and the mixed results are checked against it per solve (Ha/atom).

The headline timed region records a HIP-event pair around every pass launch
(the library then launches eagerly); the per-pass times and the roofline come
from those events. The same steps are then timed again replayed from captured
HIP graphs without events (value_graphs).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--gtol", type=float, default=1e-8)
    ap.add_argument("--fp64-max-iter", type=int, default=500,
                    help="iteration cap of the plain FP64 comparison solves")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run one device-to-device copy of MIB MiB (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters against known bytes)")
    return ap.parse_args()


def pass_bytes(sys_, prec_bytes, nf, with_loc, phase_trial):
    """Algorithmic HBM bytes of one evaluation of passes A, B, C for one solve."""
    n1, n2, n3 = sys_.n
    M = n1 * n2 * n3
    Hh = n1 * n2 * (n3 // 2 + 1)          # half-spectrum complex entries
    b = prec_bytes
    spec = 2 * b * Hh                     # one half spectrum
    # A: phi (+ d) in; phi_t, local potential, n^a and nf half spectra out
    a = (2 if phase_trial else 1) * b * M + 3 * b * M + nf * spec
    bb = 2 * nf * spec + (spec if with_loc else 0)
    # C: nf half spectra, phi_t, local potential, n^a in; dE/dphi out
    c = nf * spec + 4 * b * M
    return a, bb, c


PASS_SOURCES = ("paper_2601_23002_amd/csrc/skx_passes.hip", "paper_2601_23002_amd/csrc/skx_device.hpp",
                 "paper_2601_23002_amd/csrc/skx_internal.hpp")
TRAFFIC_FILE = "profiles/traffic_scan64_mixed.md"


def measured_traffic():
    """Pass A HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE summary,
    or None when the pass sources changed since those counters were taken."""
    import hashlib
    h = hashlib.sha256()
    for f in PASS_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    try:
        with open(os.path.join(ROOT, TRAFFIC_FILE)) as fh:
            kv = dict(l.strip().split(": ", 1) for l in fh if l.startswith("    pass"))
    except OSError:
        return None
    if kv.get("pass_sources_sha256_16") != h.hexdigest()[:16]:
        return None
    return float(kv["passA_traffic_bytes_per_launch"])


def fields_count(sys_):
    nf = 1                                # density always
    if sys_.terms & 2:
        nf += 1
    if sys_.terms & (4 | 8):
        nf += 1
    if (sys_.terms & 8) and sys_.beta != 0:
        nf += 1
    return nf


def cpu_baseline(sys_, seed=5):
    """The oracle as it stands, one FP64 evaluation of one 64^3 system."""
    from threadpoolctl import threadpool_limits
    from paper_2601_23002_amd import workloads as W
    from oracle.functional import Problem
    with threadpool_limits(limits=1):
        p = Problem(sys_)
        phi = W.random_phi(sys_, seed)
        t0 = time.perf_counter()
        p.evaluate(phi)
        dt = time.perf_counter() - t0
    return dict(value=sys_.M / dt, unit="grid-pt evals/s", cores=1, kind="oracle",
                sample=f"one FP64 evaluation (all terms, energy + dE/dphi) of one {sys_.n[0]}^3 "
                       f"scan system, single thread, {dt:.1f} s")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n}))
        return
    from paper_2601_23002_amd import skx
    from paper_2601_23002_amd import workloads as W

    systems = W.config_scan(64)
    dev = torch.device("cuda:0")

    def make(prec):
        ctxs = [skx.Context(0).setup(s, precision=prec) for s in systems]
        rhos = [torch.empty(s.n, dtype=torch.float64, device=dev) for s in systems]
        return ctxs, rhos

    def step(ctxs, rhos, max_iter=3000):
        return skx.run_batch(ctxs, rhos, gtol=args.gtol, max_iter=max_iter, m=5,
                             fp32_switch_gtol=1e-5)

    def work(res):
        return sum(r["evals"] * s.M for r, s in zip(res, systems))

    # ---- plain FP64 GPU path (speedup denominator and accuracy reference)
    fp64 = None
    if not args.no_fp64:
        print("fp64 reference solves", file=sys.stderr, flush=True)
        c64, r64 = make(skx.FP64)
        step(c64, r64, args.fp64_max_iter)        # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res64 = step(c64, r64, args.fp64_max_iter)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        fp64 = dict(value=work(res64) / t64, seconds=t64,
                    E=[r["energy"]["free_energy"] for r in res64],
                    rho=[r.cpu().numpy() for r in r64],
                    iters=[r["iters"] for r in res64])
        for c in c64:
            c.close()

    # ---- batched mixed precision (the headline)
    ctxs, rhos = make(skx.MIXED)
    for _ in range(args.warmup):
        step(ctxs, rhos)
    torch.cuda.synchronize()
    skx.profile_reset()
    skx.profile_enable(True)
    total_work = 0
    evals = {"fp32": 0, "fp64": 0}
    bytes_pass = {"passA": 0.0, "passB": 0.0, "passC": 0.0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = None
    for it in range(args.steps):
        results = step(ctxs, rhos)
        print(f"step {it}: {time.perf_counter() - t0:.3f} s", file=sys.stderr, flush=True)
        total_work += work(results)
        for r, s in zip(results, systems):
            nf = fields_count(s)
            e32, e64 = r["fp32_evals"], r["evals"] - r["fp32_evals"]
            evals["fp32"] += e32
            evals["fp64"] += e64
            for (ne, b) in ((e32, 4), (e64, 8)):
                if ne <= 0:
                    continue
                a1, b1, c1 = pass_bytes(s, b, nf, True, False)    # first evaluation
                aT, bT, cT = pass_bytes(s, b, nf, True, True)     # trial evaluations
                bytes_pass["passA"] += a1 + (ne - 1) * aT
                bytes_pass["passB"] += b1 + (ne - 1) * bT
                bytes_pass["passC"] += c1 + (ne - 1) * cT
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    skx.profile_enable(False)
    prof = skx.profile_read()
    value = total_work / wall

    # the same steps replayed from captured HIP graphs (no per-launch events)
    graph_work = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(args.steps):
        graph_work += work(step(ctxs, rhos))
    torch.cuda.synchronize()
    wall_graph = time.perf_counter() - t0
    print(f"graph steps: {wall_graph:.3f} s", file=sys.stderr, flush=True)

    # roofline of the dominant evaluation kernel
    dom = max(("passA", "passB", "passC"), key=lambda k: prof[k][0])
    ms, launches = prof[dom]
    avg_s = ms / 1e3 / max(1, launches)
    achieved = bytes_pass[dom] / max(1, launches) / avg_s / 1e9
    traffic = measured_traffic() if dom == "passA" else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic),
            "kernel": dom, "avg_launch_us": round(avg_s * 1e6, 2), "launches": launches,
            "bytes_per_launch": round(bytes_pass[dom] / max(1, launches))}

    out = {
        "metric": "grid-pt functional evals/s, batched+mixed vs plain FP64 @1e-6 Ha/atom; p99 lat",
        "value": value,
        "unit": "grid-pt evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "scan: 9 solves, 64 Z=1 ions, rs in {1,2,4} x T in {0.5,2,8} Ha, "
                               "64^3, batched, FP32 to |r|<1e-5 then FP64 to |r|<%g" % args.gtol,
                   "global_batch": len(systems), "grid": 64, "parallelism": "batch"},
        "roofline": roof,
        "passes_ms": {k: round(v[0], 3) for k, v in prof.items()},
        "value_graphs": graph_work / wall_graph,
        "ms_per_step_graphs": wall_graph / args.steps * 1e3,
        "evals": evals,
    }
    if fp64 is not None:
        err = []
        rerr = []
        for i, (r, s) in enumerate(zip(results, systems)):
            err.append(abs(r["energy"]["free_energy"] - fp64["E"][i]) / len(s.zval))
            n_m = rhos[i].cpu().numpy()
            rerr.append(float(np.sum(np.abs(n_m - fp64["rho"][i])) / np.sum(fp64["rho"][i])))
        out["fp64_value"] = fp64["value"]
        out["speedup_vs_fp64"] = value / fp64["value"]
        out["max_err_ha_per_atom"] = max(err)
        out["max_rel_density_err"] = max(rerr)
        out["iters_fp64"] = fp64["iters"]
        out["fp64_max_iter"] = args.fp64_max_iter
    out["iters_mixed"] = [r["iters"] for r in results]
    out["status"] = [r["status"] for r in results]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(systems[0])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
