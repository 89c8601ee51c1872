"""Write converged oracle minima for the solve-parity tests.

Calls only the CPU oracle (oracle/) and the seeded input recipes
(paper_2601_23002_amd/workloads.py, which hold no method arithmetic). For
each case it minimises the free energy from the uniform density to
||r|| < gtol and stores, in tests/golden/minima_<case>.npz:

  n        the minimising density (float32: its rounding, ~6e-8 relative,
           is far below the 1e-6 density gate of the tests)
  energy   the energy terms at the minimum, FP64, in the order of KEYS
  info     [gnorm, iterations, evaluations, status, xc variant]

Cases (the single small solve and one 64^3 scan system per rs, seeds 2, 5
and 8 of the scan recipe):

  c1      16 H, rs = 2, T = 1 Ha, 32^3, seed 1
  scan2   64 H, rs = 1, T = 0.5 Ha, 64^3, seed 2
  scan5   64 H, rs = 2, T = 0.5 Ha, 64^3, seed 5
  scan8   64 H, rs = 4, T = 0.5 Ha, 64^3, seed 8

Usage: python tests/golden/make_minima.py CASE [XC]   (XC: 1 published
PZ81 fit, 2 the C1-joined variant; default 1). A run at 64^3 takes
10-20 minutes on one core.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.functional import Problem, ENERGY_KEYS  # noqa: E402
from oracle.optimize import optimize  # noqa: E402
from paper_2601_23002_amd import workloads as W  # noqa: E402

KEYS = ENERGY_KEYS + ("free_energy", "mu", "nelec")


def case_system(name: str):
    if name == "c1":
        return W.config_single_small(32)
    if name.startswith("scan"):
        seed = int(name[4:])
        return W.config_scan(64)[seed - 2]
    raise ValueError(f"unknown case {name}")


def main():
    name = sys.argv[1]
    variant = int(sys.argv[2]) if len(sys.argv) > 2 else W.XC_PZ81
    gtol = 1e-8
    s = case_system(name)
    s.xc = variant
    t0 = time.time()
    p = Problem(s)
    res = optimize(p, gtol=gtol, max_iter=600, verbose=True)
    e = res["energy"]
    energy = np.array([e[k] for k in KEYS], dtype=np.float64)
    info = np.array([res["gnorm"], res["iters"], res["evals"], res["status"], variant],
                    dtype=np.float64)
    out = os.path.join(HERE, f"minima_{name}.npz")
    np.savez_compressed(out, n=res["n"].astype(np.float32), energy=energy, info=info,
                        keys=np.array(KEYS))
    rs_min = (3.0 / (4.0 * np.pi * res["n"].max())) ** (1.0 / 3.0)
    print(f"{name}: F = {e['free_energy']:.14f} |r| = {res['gnorm']:.3e} iters {res['iters']} "
          f"status {res['status']} xc {variant} rs_min {rs_min:.4f} ({time.time() - t0:.0f} s) -> {out}",
          flush=True)


if __name__ == "__main__":
    main()
