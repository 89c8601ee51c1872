"""Seeded synthetic inputs shared by the tests, the benchmark and the serving demo.

This module holds no arithmetic of the orbital-free method: it only draws
ionic positions and picks cell and grid sizes. Both the HIP path and the
CPU oracle consume what it returns, so neither depends on the other.

Stand-ins for the paper's workloads (warm dense hydrogen, and beryllium-like
Z=4 ions; Methods section, "Numerical calculations"): the paper's
Heine-Abarenkov and fhi98PP pseudopotentials are not printed, so a local
erf pseudopotential -Z erf(r/rc)/r of stated width replaces them.

Cell recipe: the Wigner-Seitz radius rs is defined by the electron density
(Results section, definition of r_s), so for N ions of valence Z the cube
volume is V = N*Z*(4*pi/3)*rs**3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

def _five_smooth_even(lo: int = 8, hi: int = 512):
    out = []
    for n in range(lo, hi + 1):
        if n % 2:
            continue
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return tuple(out)


# Even 5-smooth sizes the FFTs accept (both sides support every one of them).
ALLOWED_N = _five_smooth_even()


def smallest_allowed(n_min: float, lo: int = 8, hi: int = 512) -> int:
    for n in ALLOWED_N:
        if n >= n_min and lo <= n <= hi:
            return n
    return max(x for x in ALLOWED_N if x <= hi)


@dataclass
class System:
    """One OFDFT problem: cubic cell, grid, ions and functional settings."""
    L: float                       # cube side, bohr
    n: tuple                       # (n1, n2, n3)
    pos: np.ndarray                # (N, 3) cartesian bohr
    zval: np.ndarray               # (N,) valence charge per ion
    rc: np.ndarray                 # (N,) erf width per ion, bohr
    T: float                       # electron temperature, Ha
    beta: float = 1.0              # weight of the first-order kernel correction
    alpha: float = 5.0 / 6.0       # exponent a of f = n**a in the nonlocal term
    terms: int = 0x7F              # bitmask, see TERM_* below
    xc: int = 1                    # XC_PZ81 (published fit) or XC_PZ81_C1 (joined), see below
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nelec(self) -> float:
        return float(np.sum(self.zval))

    @property
    def volume(self) -> float:
        return self.L ** 3

    @property
    def M(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])


TERM_TF, TERM_VW, TERM_NL0, TERM_NL1, TERM_HARTREE, TERM_LOCPP, TERM_XC = (
    1, 2, 4, 8, 16, 32, 64)
TERM_ALL = 0x7F
# exchange-correlation variant codes (the same numbers as the library's)
XC_NONE, XC_PZ81, XC_PZ81_C1 = 0, 1, 2


def cell_side(nelec: float, rs: float) -> float:
    return (nelec * 4.0 * math.pi / 3.0 * rs ** 3) ** (1.0 / 3.0)


def uniform_system(nions: int, Z: float, rc: float, rs: float, T: float, n: int,
                   seed: int, beta: float = 1.0, alpha: float = 5.0 / 6.0,
                   terms: int = TERM_ALL, name: str = "") -> System:
    """Ions placed uniformly at random in the cube (PCG64 stream of `seed`)."""
    L = cell_side(nions * Z, rs)
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, L, size=(nions, 3))
    return System(L=L, n=(n, n, n), pos=pos, zval=np.full(nions, float(Z)),
                  rc=np.full(nions, float(rc)), T=float(T), beta=beta,
                  alpha=alpha, terms=terms, name=name,
                  meta=dict(rs=rs, Z=Z, seed=seed))


def thermal_system(nions: int, Z: float, rc: float, rs: float, T: float,
                   h_target: float, nmin: int, nmax: int, seed: int,
                   rng: np.random.Generator | None = None, name: str = "") -> System:
    """Random sites (no pair closer than half a Wigner-Seitz radius) plus
    Gaussian displacements of 0.1 a_ws, the thermal-like snapshot recipe."""
    rng = rng if rng is not None else np.random.default_rng(seed)
    L = cell_side(nions * Z, rs)
    a_ws = (3.0 * L ** 3 / (4.0 * math.pi * nions)) ** (1.0 / 3.0)
    dmin = 0.5 * a_ws
    sites = []
    tries = 0
    while len(sites) < nions:
        p = rng.uniform(0.0, L, size=3)
        ok = True
        for q in sites:
            d = p - q
            d -= L * np.round(d / L)
            if float(d @ d) < dmin * dmin:
                ok = False
                break
        tries += 1
        if ok or tries > 200 * nions:
            sites.append(p)
    pos = np.array(sites) + rng.normal(0.0, 0.1 * a_ws, size=(nions, 3))
    pos = np.mod(pos, L)
    n = smallest_allowed(L / h_target, lo=nmin, hi=nmax)
    n = min(max(n, nmin), nmax)
    return System(L=L, n=(n, n, n), pos=pos, zval=np.full(nions, float(Z)),
                  rc=np.full(nions, float(rc)), T=float(T), name=name,
                  meta=dict(rs=rs, Z=Z, seed=seed))


# ----------------------------------------------------------------------------
# The five workload recipes
# ----------------------------------------------------------------------------

def config_single_small(n: int = 32) -> System:
    """16 Z=1 ions (rc=0.3), rs=2, T=1 Ha, 32^3, seed 1."""
    return uniform_system(16, 1.0, 0.3, 2.0, 1.0, n, seed=1, name="h16_rs2_T1_32")


def config_scan(n: int = 64):
    """64 Z=1 ions at rs in {1,2,4} x T in {0.5,2,8} Ha on 64^3, seeds 2..10."""
    out = []
    seed = 2
    for rs in (1.0, 2.0, 4.0):
        for T in (0.5, 2.0, 8.0):
            out.append(uniform_system(64, 1.0, 0.3, rs, T, n, seed=seed,
                                      name=f"h64_rs{rs:g}_T{T:g}_{n}"))
            seed += 1
    return out


def config_mixed(n: int = 96) -> System:
    """128 Z=4 ions (rc=0.5), rs=1.5, T=4 Ha, 96^3, seed 11."""
    return uniform_system(128, 4.0, 0.5, 1.5, 4.0, n, seed=11, name="be128_rs1.5_T4_96")


def config_ensemble(count: int = 256, seed: int = 12, nmin: int = 32, nmax: int = 80):
    """Uneven snapshots: N log-uniform in [16,256], Z in {1,4}; grid for h=0.25 bohr."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        N = int(round(math.exp(rng.uniform(math.log(16), math.log(256)))))
        if rng.uniform() < 0.5:
            Z, rs, T, rc = 1.0, 2.0, 1.0, 0.3
        else:
            Z, rs, T, rc = 4.0, 1.5, 4.0, 0.5
        out.append(thermal_system(N, Z, rc, rs, T, 0.25, nmin, nmax, seed, rng=rng,
                                  name=f"snap{i}_N{N}_Z{int(Z)}"))
    return out


def config_stream(count: int = 2200, rate: float = 200.0, seed: int = 13,
                  nmin: int = 32, nmax: int = 192, nions_max: int = 1024):
    """Poisson request stream: arrival times plus one System per request."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        N = int(round(math.exp(rng.uniform(math.log(16), math.log(nions_max)))))
        Z = 1.0 if rng.uniform() < 0.5 else 4.0
        rc = 0.3 if Z == 1.0 else 0.5
        rs = rng.uniform(1.0, 4.0)
        T = math.exp(rng.uniform(math.log(0.5), math.log(10.0)))
        h = rng.uniform(0.15, 0.35)
        L = cell_side(N * Z, rs)
        n = smallest_allowed(L / h, lo=nmin, hi=nmax)
        pos = rng.uniform(0.0, L, size=(N, 3))
        reqs.append((t, System(L=L, n=(n, n, n), pos=pos, zval=np.full(N, Z),
                               rc=np.full(N, rc), T=T, name=f"req{i}",
                               meta=dict(rs=rs, Z=Z))))
    return reqs


def random_phi(sys: System, seed: int, amp: float = 0.3) -> np.ndarray:
    """A smooth positive random sqrt-density normalised to the electron count,
    built from a few random plane waves (no method arithmetic involved)."""
    rng = np.random.default_rng(seed)
    n1, n2, n3 = sys.n
    x = np.arange(n1)[:, None, None] / n1
    y = np.arange(n2)[None, :, None] / n2
    z = np.arange(n3)[None, None, :] / n3
    f = np.ones(sys.n)
    for _ in range(6):
        g = rng.integers(-3, 4, size=3)
        ph = rng.uniform(0, 2 * math.pi)
        f = f + amp * rng.uniform(0.2, 1.0) * np.cos(2 * math.pi * (g[0] * x + g[1] * y + g[2] * z) + ph)
    f = np.abs(f) + 0.05
    dv = sys.volume / sys.M
    f *= math.sqrt(sys.nelec / (dv * np.sum(f * f)))
    return f
