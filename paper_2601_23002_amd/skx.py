"""Thin Python binding of libskx (include/skx.h) over ctypes.

Argument marshalling only: every step of the evaluation and of the
optimisation runs in the library's HIP kernels. PyTorch supplies device
memory and the stream. If the shared library is missing, importing this
module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
# torch first: its HIP runtime must be the one the library binds to (both
# carry the soname libamdhip64.so.7), so device pointers and streams are
# shared between the two
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libskx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libskx.so not built ({LIB_PATH}); run paper_2601_23002_amd/build.py")
_lib = C.CDLL(LIB_PATH)

OK, NOT_CONVERGED, CANCELLED = 0, 1, 2
E_INVALID, E_STATE, E_NOMEM, E_DEVICE, E_NUMERIC = -1, -2, -3, -4, -5
TERM_TF, TERM_VW, TERM_NL0, TERM_NL1, TERM_HARTREE, TERM_LOCPP, TERM_XC = 1, 2, 4, 8, 16, 32, 64
TERM_ALL = 127
XC_NONE, XC_PZ81, XC_PZ81_C1 = 0, 1, 2
FP64, FP32, MIXED = 0, 1, 2
RHO, SQRT_RHO = 0, 1


class SkxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"skx error {code}: {msg}")
        self.code = code


class Functional(C.Structure):
    _fields_ = [("T", C.c_double), ("beta", C.c_double), ("alpha", C.c_double),
                ("terms", C.c_uint), ("xc", C.c_int), ("precision", C.c_int)]


class Energy(C.Structure):
    _fields_ = [(k, C.c_double) for k in (
        "f_tf", "e_vw", "f_nl0", "f_nl1", "e_h", "e_loc", "e_xc", "e_ii",
        "free_energy", "total", "mu", "nelec")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class OptParams(C.Structure):
    _fields_ = [("gtol", C.c_double), ("max_iter", C.c_int), ("lbfgs_m", C.c_int),
                ("fp32_switch_gtol", C.c_double), ("warm_start", C.c_int)]


class OptResult(C.Structure):
    _fields_ = [("e", Energy), ("iters", C.c_int), ("evals", C.c_int),
                ("fp32_iters", C.c_int), ("fp32_evals", C.c_int), ("gnorm", C.c_double),
                ("status", C.c_int), ("resets", C.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "e"}
        d["energy"] = self.e.as_dict()
        return d


class NoseHoover(C.Structure):
    """Thermostat state of md_step_nvt (xi and eta are updated in place)."""
    _fields_ = [("T_ion", C.c_double), ("Q", C.c_double), ("xi", C.c_double), ("eta", C.c_double)]


class Request(C.Structure):
    _fields_ = [("lattice", C.c_double * 9), ("n1", C.c_int), ("n2", C.c_int), ("n3", C.c_int),
                ("nions", C.c_int), ("pos", C.POINTER(C.c_double)),
                ("species", C.POINTER(C.c_int)), ("nspecies", C.c_int),
                ("zval", C.POINTER(C.c_double)), ("rc", C.POINTER(C.c_double)),
                ("fn", Functional), ("opt", OptParams), ("t_arrival", C.c_double)]


class Result(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("r", OptResult), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("npoints", C.c_longlong)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_VP = C.c_void_p
_sig("skx_create", C.c_int, [C.POINTER(_VP), C.c_int, _VP])
_sig("skx_destroy", None, [_VP])
_sig("skx_last_error", C.c_char_p, [_VP])
_sig("skx_set_cell", C.c_int, [_VP, C.POINTER(C.c_double), C.c_int, C.c_int, C.c_int])
_sig("skx_set_ions", C.c_int, [_VP, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_int,
                               C.POINTER(C.c_double), C.POINTER(C.c_double)])
_sig("skx_set_functional", C.c_int, [_VP, C.POINTER(Functional)])
_sig("skx_evaluate_energy_potential", C.c_int, [_VP, _VP, C.c_int, _VP, C.POINTER(Energy)])
_sig("skx_optimize_density", C.c_int, [_VP, _VP, C.POINTER(OptParams), C.POINTER(OptResult)])
_sig("skx_run_batch", C.c_int, [C.POINTER(_VP), C.c_int, C.POINTER(_VP), C.POINTER(OptParams),
                                C.POINTER(OptResult)])
_sig("skx_ion_forces", C.c_int, [_VP, _VP, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)])
_sig("skx_md_step", C.c_int, [_VP, _VP, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double,
                              C.POINTER(OptParams), C.POINTER(OptResult)])
_sig("skx_structure_factors", C.c_int, [_VP, _VP, C.c_int, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_int), C.c_int])
_sig("skx_density_deviation", C.c_int, [_VP, _VP, _VP, C.POINTER(C.c_double)])
_sig("skx_density_deviation_noalloc", C.c_int, [_VP, _VP, _VP, C.POINTER(C.c_double)])
_sig("skx_fit_beta", C.c_int, [_VP, _VP, _VP, C.c_double, C.c_double, C.c_double,
                               C.POINTER(OptParams), C.POINTER(C.c_double),
                               C.POINTER(C.c_double), C.POINTER(C.c_int)])
_sig("skx_md_step_nvt", C.c_int, [_VP, _VP, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double,
                                  C.POINTER(NoseHoover), C.POINTER(OptParams),
                                  C.POINTER(OptResult)])
_sig("skx_pressure", C.c_int, [_VP, _VP, C.c_double, C.POINTER(OptParams), C.POINTER(C.c_double),
                               C.POINTER(C.c_double), C.POINTER(C.c_double)])
_sig("skx_get_kernel_tables", C.c_int, [_VP, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int])
_sig("skx_get_vloc", C.c_int, [_VP, C.POINTER(C.c_double)])
_sig("skx_num_shells", C.c_int, [_VP])
_sig("skx_fd_eval", C.c_int, [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.POINTER(C.c_double), C.c_longlong])
_sig("skx_fft_check", C.c_int, [_VP, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.POINTER(C.c_double)])
_sig("skx_profile_enable", C.c_int, [C.c_int])
_sig("skx_set_graphs", C.c_int, [C.c_int])
_sig("skx_profile_mask", C.c_uint, [C.c_uint])
_sig("skx_set_autotune", C.c_int, [C.c_int])
_sig("skx_set_shape_kernels", C.c_int, [C.c_int])
_sig("skx_set_plane_chunking", C.c_int, [C.c_int])
_sig("skx_get_radix_order", C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int), C.c_int])
_sig("skx_profile_reset", C.c_int, [])
_sig("skx_profile_read", C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_longlong), C.c_int])
_sig("skx_bench_eval", C.c_int, [C.POINTER(_VP), C.c_int, C.c_int, C.POINTER(C.c_double)])
_sig("skx_engine_create", C.c_int, [C.POINTER(_VP), C.c_int, C.c_size_t, C.c_int])
_sig("skx_engine_submit", C.c_int, [_VP, C.POINTER(Request), C.POINTER(C.c_uint64)])
_sig("skx_engine_step", C.c_int, [_VP])
_sig("skx_engine_poll", C.c_int, [_VP, C.POINTER(Result), C.POINTER(C.POINTER(C.c_double)),
                                  C.c_int, C.POINTER(C.c_int)])
_sig("skx_engine_pending", C.c_int, [_VP])
_sig("skx_engine_cancel", C.c_int, [_VP, C.c_uint64])
_sig("skx_engine_destroy", None, [_VP])
_sig("skx_engine_clock", C.c_double, [_VP])
_sig("skx_engine_last_error", C.c_char_p, [_VP])


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _torch():
    import torch
    return torch


def _stream_handle(device):
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


def _ion_arrays(pos, zval, rc, species=None):
    """Positions [N][3], species index per ion and per-species (Z, rc) arrays."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    zval = np.asarray(zval, dtype=np.float64).reshape(-1)
    rc = np.asarray(rc, dtype=np.float64).reshape(-1)
    if species is None:
        # one species per distinct (Z, rc) pair
        keys = list(zip(zval.tolist(), rc.tolist())) if zval.size == len(pos) else None
        if keys is None:
            raise ValueError("give species, or per-ion zval and rc")
        uniq = sorted(set(keys))
        species = np.array([uniq.index(k) for k in keys], dtype=np.int32)
        zsp = np.array([u[0] for u in uniq])
        rsp = np.array([u[1] for u in uniq])
    else:
        species = np.asarray(species, dtype=np.int32)
        zsp, rsp = zval, rc
    return (pos, np.ascontiguousarray(species, dtype=np.int32),
            np.ascontiguousarray(zsp, dtype=np.float64), np.ascontiguousarray(rsp, dtype=np.float64))


class Context:
    """One solve: cell, ions, functional and its device state."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("libskx needs a GPU")
        self.device = device
        h = _VP()
        s = stream if stream is not None else _stream_handle(device)
        rc = _lib.skx_create(C.byref(h), device, _VP(s))
        if rc != OK:
            raise SkxError(rc, "skx_create failed")
        self._h = h
        self.n = None
        self.L = None
        self.precision = FP64

    def close(self):
        if getattr(self, "_h", None):
            _lib.skx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc < 0:
            raise SkxError(rc, _lib.skx_last_error(self._h).decode())
        return rc

    def set_cell(self, L: float, n):
        n = tuple(int(x) for x in (n if hasattr(n, "__len__") else (n, n, n)))
        lat = (C.c_double * 9)(L, 0, 0, 0, L, 0, 0, 0, L)
        self._check(_lib.skx_set_cell(self._h, lat, *n))
        self.n, self.L = n, float(L)

    def set_ions(self, pos, zval, rc, species=None):
        pos, species, zsp, rsp = _ion_arrays(pos, zval, rc, species)
        self._check(_lib.skx_set_ions(self._h, len(pos), _dptr(pos),
                                      species.ctypes.data_as(C.POINTER(C.c_int)), len(zsp),
                                      _dptr(zsp), _dptr(rsp)))
        self.nions = len(pos)
        self.nspecies = len(zsp)
        self.species_zrc = list(zip(zsp.tolist(), rsp.tolist()))   # (Z, rc) per species index

    def set_functional(self, T, beta=1.0, alpha=5.0 / 6.0, terms=TERM_ALL, xc=XC_PZ81,
                       precision=FP64):
        fn = Functional(T, beta, alpha, terms, xc, precision)
        self._check(_lib.skx_set_functional(self._h, C.byref(fn)))
        self.precision = precision

    def setup(self, sys, precision=FP64):
        """Configure from a workloads.System."""
        self.set_cell(sys.L, sys.n)
        self.set_ions(sys.pos, sys.zval, sys.rc)
        self.set_functional(sys.T, sys.beta, sys.alpha, sys.terms, getattr(sys, "xc", XC_PZ81),
                            precision)
        return self

    def evaluate(self, field, kind=SQRT_RHO, want_grad=True):
        """Energies (dict) and dE/dphi (tensor or None) for a device field."""
        torch = _torch()
        dt = torch.float32 if self.precision == FP32 else torch.float64
        if field.dtype != dt or not field.is_cuda or not field.is_contiguous():
            raise ValueError(f"field must be a contiguous {dt} CUDA tensor")
        out = torch.empty_like(field) if want_grad else None
        e = Energy()
        self._check(_lib.skx_evaluate_energy_potential(
            self._h, _VP(field.data_ptr()), kind, _VP(out.data_ptr()) if out is not None else None,
            C.byref(e)))
        return e.as_dict(), out

    def optimize(self, gtol=1e-8, max_iter=1000, m=5, fp32_switch_gtol=1e-5, rho0=None):
        torch = _torch()
        if rho0 is not None:
            rho = rho0.to(dtype=torch.float64).contiguous().clone()
            warm = 1
        else:
            rho = torch.empty(self.n, dtype=torch.float64, device=f"cuda:{self.device}")
            warm = 0
        p = OptParams(gtol, max_iter, m, fp32_switch_gtol, warm)
        r = OptResult()
        rc = _lib.skx_optimize_density(self._h, _VP(rho.data_ptr()), C.byref(p), C.byref(r))
        self._check(rc)
        return rho, r.as_dict()

    def ion_forces(self, field=None, kind=SQRT_RHO, local=True, ewald=True):
        """Forces on the ions (Hartree/bohr): (f_loc, f_ii), each [nions][3]
        or None when not asked for. field: contiguous FP64 CUDA tensor on
        the cell's grid, the density (RHO) or its square root (SQRT_RHO)."""
        torch = _torch()
        if local and (field is None or field.dtype != torch.float64 or not field.is_cuda
                      or not field.is_contiguous()):
            raise ValueError("field must be a contiguous float64 CUDA tensor")
        fl = np.zeros((self.nions, 3)) if local else None
        fi = np.zeros((self.nions, 3)) if ewald else None
        self._check(_lib.skx_ion_forces(
            self._h, _VP(field.data_ptr()) if local else None, kind,
            _dptr(fl) if local else None, _dptr(fi) if ewald else None))
        return fl, fi

    def structure_factors(self, field, kind=RHO):
        """Shell-averaged S_ei, S_ee, S_ii (numpy arrays over shells
        s = g1^2 + g2^2 + g3^2) and the number of grid wave vectors per shell,
        for one density snapshot (contiguous FP64 CUDA tensor)."""
        torch = _torch()
        if field.dtype != torch.float64 or not field.is_cuda or not field.is_contiguous():
            raise ValueError("field must be a contiguous float64 CUDA tensor")
        ns = _lib.skx_num_shells(self._h)
        ei, ee, ii = np.zeros(ns), np.zeros(ns), np.zeros(ns)
        cnt = np.zeros(ns, dtype=np.int32)
        self._check(_lib.skx_structure_factors(self._h, _VP(field.data_ptr()), kind, _dptr(ei),
                                               _dptr(ee), _dptr(ii),
                                               cnt.ctypes.data_as(C.POINTER(C.c_int)), ns))
        return ei, ee, ii, cnt

    def density_deviation(self, a, b):
        """integral |a - b| dr of two contiguous FP64 CUDA densities."""
        torch = _torch()
        for t in (a, b):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("densities must be contiguous float64 CUDA tensors")
        out = C.c_double()
        self._check(_lib.skx_density_deviation(self._h, _VP(a.data_ptr()), _VP(b.data_ptr()),
                                               C.byref(out)))
        return out.value

    def density_deviation_noalloc(self, a, b):
        """density_deviation with the library's fixed device scratch (the call
        allocates nothing; calls on one device must not overlap)."""
        torch = _torch()
        for t in (a, b):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("densities must be contiguous float64 CUDA tensors")
        out = C.c_double()
        self._check(_lib.skx_density_deviation_noalloc(self._h, _VP(a.data_ptr()),
                                                       _VP(b.data_ptr()), C.byref(out)))
        return out.value

    def fit_beta(self, rho_ref, lo=0.0, hi=2.0, xtol=1e-4, gtol=1e-8, max_iter=1000, m=5,
                 fp32_switch_gtol=1e-5, rho0=None):
        """beta minimising integral |n[beta] - rho_ref| (Eq. (3)) for this
        configuration; returns (beta, deviation, solves, density at beta)."""
        torch = _torch()
        if rho_ref.dtype != torch.float64 or not rho_ref.is_cuda or not rho_ref.is_contiguous():
            raise ValueError("rho_ref must be a contiguous float64 CUDA tensor")
        if rho0 is not None:
            rho = rho0.to(dtype=torch.float64).contiguous().clone()
        else:
            rho = torch.empty_like(rho_ref)
        p = OptParams(gtol, max_iter, m, fp32_switch_gtol, 1 if rho0 is not None else 0)
        beta, dev, ns = C.c_double(), C.c_double(), C.c_int()
        self._check(_lib.skx_fit_beta(self._h, _VP(rho_ref.data_ptr()), _VP(rho.data_ptr()),
                                      lo, hi, xtol, C.byref(p), C.byref(beta), C.byref(dev),
                                      C.byref(ns)))
        return beta.value, dev.value, ns.value, rho

    def pressure(self, rho, eps=1e-4, gtol=1e-9, max_iter=2000, m=5, fp32_switch_gtol=1e-5):
        """-dF/dV (Hartree/bohr^3) at fixed fractional ion positions by a
        central difference of minimised free energies; returns
        (P, F(V(1-eps)), F(V(1+eps))). self.last_status holds the call's
        status: OK, or NOT_CONVERGED when either solve stopped short."""
        torch = _torch()
        if rho.dtype != torch.float64 or not rho.is_cuda or not rho.is_contiguous():
            raise ValueError("rho must be a contiguous float64 CUDA tensor")
        p = OptParams(gtol, max_iter, m, fp32_switch_gtol, 1)
        P, Flo, Fhi = C.c_double(), C.c_double(), C.c_double()
        rc = self._check(_lib.skx_pressure(self._h, _VP(rho.data_ptr()), eps, C.byref(p),
                                           C.byref(P), C.byref(Flo), C.byref(Fhi)))
        self.last_status = rc
        return P.value, Flo.value, Fhi.value

    def md_step(self, rho, pos, vel, force, mass, dt, gtol=1e-8, max_iter=1000, m=5,
                fp32_switch_gtol=1e-5, thermostat=None):
        """One velocity-Verlet step; pos, vel, force (float64 [nions][3]
        arrays) are updated in place, rho (FP64 CUDA density) too. mass per
        species in electron masses. thermostat: a NoseHoover state for an NVT
        step (updated in place), None for NVE. Returns the solve's result
        dict."""
        for a in (pos, vel, force):
            if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous
                    and a.shape == (self.nions, 3)):
                raise ValueError("pos, vel and force must be C-contiguous float64 [nions][3] arrays")
        mass = np.ascontiguousarray(mass, dtype=np.float64).reshape(-1)
        if mass.size != self.nspecies:
            raise ValueError("one mass per species")
        p = OptParams(gtol, max_iter, m, fp32_switch_gtol, 1)
        r = OptResult()
        if thermostat is None:
            rc = _lib.skx_md_step(self._h, _VP(rho.data_ptr()), _dptr(pos), _dptr(vel),
                                  _dptr(force), _dptr(mass), dt, C.byref(p), C.byref(r))
        else:
            rc = _lib.skx_md_step_nvt(self._h, _VP(rho.data_ptr()), _dptr(pos), _dptr(vel),
                                      _dptr(force), _dptr(mass), dt, C.byref(thermostat),
                                      C.byref(p), C.byref(r))
        self._check(rc)
        return r.as_dict()

    def kernel_tables(self):
        ns = _lib.skx_num_shells(self._h)
        w = np.zeros(ns)
        wp = np.zeros(ns)
        self._check(_lib.skx_get_kernel_tables(self._h, _dptr(w), _dptr(wp), ns))
        return w, wp

    def vloc(self):
        n1, n2, n3 = self.n
        out = np.zeros((n1, n2, n3 // 2 + 1, 2))
        self._check(_lib.skx_get_vloc(self._h, _dptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def fft_check(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros_like(x)
        n1, n2, n3 = x.shape
        spec = np.zeros((n1, n2, n3 // 2 + 1, 2))
        self._check(_lib.skx_fft_check(self._h, _dptr(x), _dptr(out), _dptr(spec)))
        return out, spec[..., 0] + 1j * spec[..., 1]


def fd_eval(u, device=0):
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    eta = np.zeros_like(u)
    psi = np.zeros_like(u)
    rc = _lib.skx_fd_eval(device, _dptr(u), _dptr(eta), _dptr(psi), u.size)
    if rc != OK:
        raise SkxError(rc, "skx_fd_eval failed")
    return eta, psi


def run_batch(ctxs, rhos, gtol=1e-8, max_iter=1000, m=5, fp32_switch_gtol=1e-5, warm=False):
    n = len(ctxs)
    hs = (_VP * n)(*[c._h for c in ctxs])
    ptrs = (_VP * n)(*[r.data_ptr() for r in rhos])
    p = OptParams(gtol, max_iter, m, fp32_switch_gtol, 1 if warm else 0)
    res = (OptResult * n)()
    rc = _lib.skx_run_batch(hs, n, ptrs, C.byref(p), res)
    if rc < 0:
        raise SkxError(rc, _lib.skx_last_error(ctxs[0]._h).decode())
    return [r.as_dict() for r in res]


PASS_NAMES = ("passA", "passB", "passC", "reduce", "update", "direction", "precond", "point",
              "force_loc", "force_ewald", "structure")


def profile_enable(on=True):
    _lib.skx_profile_enable(1 if on else 0)


def profile_mask(passes=None):
    """Time only the named passes (PASS_NAMES) while profiling; None: all.
    Returns the previous mask."""
    mask = 0xFFFFFFFF if passes is None else sum(1 << PASS_NAMES.index(p) for p in passes)
    return _lib.skx_profile_mask(mask)


def set_graphs(on=True):
    """Replay the driver's step sequences from a captured HIP graph, or
    launch them eagerly (the default); returns the previous setting."""
    return bool(_lib.skx_set_graphs(1 if on else 0))


def set_autotune(on=True):
    """Time candidate FFT radix orders at first set-up of each length and keep
    the fastest (process-wide); returns the previous setting."""
    return bool(_lib.skx_set_autotune(1 if on else 0))


def set_shape_kernels(mask=7):
    """Passes (bit mask: 1 A, 2 B, 4 C; True = all, False = none) that run
    their compile-time-shaped kernels on the cubic lengths that have them
    (all three passes at 36-80, pass B alone at twelve lengths 90-192;
    process-wide);
    returns the previous mask."""
    if mask is True:
        mask = 7
    elif mask is False:
        mask = 0
    return _lib.skx_set_shape_kernels(int(mask))


def set_plane_chunking(force=True):
    """Run passes A and C of every plane on the split kernels (row-pair and
    column chunks in separate launches; force) or only where they are chosen
    (planes beyond LDS and the sizes measured faster; default); returns the
    previous setting."""
    return bool(_lib.skx_set_plane_chunking(1 if force else 0))


def radix_order(n, precision=FP64):
    buf = (C.c_int * 16)()
    k = _lib.skx_get_radix_order(n, precision, buf, 16)
    if k < 0:
        raise SkxError(k, "skx_get_radix_order failed")
    return [buf[i] for i in range(k)]


def profile_reset():
    _lib.skx_profile_reset()


def profile_read():
    """{pass name: (total ms, launches)} from the library's HIP-event timers."""
    k = len(PASS_NAMES)
    ms = (C.c_double * k)()
    cnt = (C.c_longlong * k)()
    n = _lib.skx_profile_read(ms, cnt, k)
    return {PASS_NAMES[i]: (ms[i], cnt[i]) for i in range(min(n, len(PASS_NAMES)))}


def bench_eval(ctxs, reps=20):
    """Mean per-launch milliseconds of passes A, B, C over a batch."""
    n = len(ctxs)
    hs = (_VP * n)(*[c._h for c in ctxs])
    ms = (C.c_double * 3)()
    rc = _lib.skx_bench_eval(hs, n, reps, ms)
    if rc < 0:
        raise SkxError(rc, _lib.skx_last_error(ctxs[0]._h).decode())
    return {"passA": ms[0], "passB": ms[1], "passC": ms[2]}


class Engine:
    """Serving engine (skx_engine_*): continuous batching of optimisations."""

    def __init__(self, device: int = 0, hbm_budget: int = 64 << 30, max_slots: int = 64):
        self._h = _VP()
        rc = _lib.skx_engine_create(C.byref(self._h), device, hbm_budget, max_slots)
        if rc != OK:
            raise SkxError(rc, "skx_engine_create failed")
        self._npts = {}

    def close(self):
        if self._h:
            _lib.skx_engine_destroy(self._h)
            self._h = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clock(self) -> float:
        return _lib.skx_engine_clock(self._h)

    def submit(self, sys, precision=MIXED, gtol=1e-8, max_iter=1000, m=5,
               fp32_switch_gtol=1e-5, t_arrival=None) -> int:
        """Queue one workloads.System; returns its ticket."""
        pos, species, zsp, rsp = _ion_arrays(sys.pos, sys.zval, sys.rc)
        req = Request()
        L = float(sys.L)
        for i, v in enumerate((L, 0, 0, 0, L, 0, 0, 0, L)):
            req.lattice[i] = v
        req.n1, req.n2, req.n3 = sys.n
        req.nions = len(pos)
        req.pos = _dptr(pos)
        req.species = species.ctypes.data_as(C.POINTER(C.c_int))
        req.nspecies = len(zsp)
        req.zval = _dptr(zsp)
        req.rc = _dptr(rsp)
        req.fn = Functional(sys.T, sys.beta, sys.alpha, sys.terms, getattr(sys, "xc", XC_PZ81),
                            precision)
        req.opt = OptParams(gtol, max_iter, m, fp32_switch_gtol, 0)
        req.t_arrival = self.clock() if t_arrival is None else t_arrival
        t = C.c_uint64()
        rc = _lib.skx_engine_submit(self._h, C.byref(req), C.byref(t))
        if rc != OK:
            raise SkxError(rc, _lib.skx_engine_last_error(self._h).decode())
        self._npts[t.value] = tuple(sys.n)
        return t.value

    def step(self) -> int:
        rc = _lib.skx_engine_step(self._h)
        if rc < 0:
            raise SkxError(rc, _lib.skx_engine_last_error(self._h).decode())
        return rc

    def pending(self) -> int:
        return _lib.skx_engine_pending(self._h)

    def cancel(self, ticket: int):
        """Cancel a queued or resident request (reported by poll as CANCELLED)."""
        rc = _lib.skx_engine_cancel(self._h, ticket)
        if rc != OK:
            raise SkxError(rc, _lib.skx_engine_last_error(self._h).decode())

    def poll(self, want_density=False, max_results=256):
        """Finished results: dicts with ticket, result, t_admit, t_done (engine clock)
        and the density (numpy, FP64) when want_density."""
        res = []
        while len(res) < max_results:
            k = 1 if want_density else max_results - len(res)
            out = (Result * k)()
            bufs, buf = None, None
            if want_density:
                biggest = max((int(np.prod(v)) for v in self._npts.values()), default=1)
                buf = np.empty(biggest)
                bufs = (C.POINTER(C.c_double) * 1)(_dptr(buf))
            n = C.c_int()
            rc = _lib.skx_engine_poll(self._h, out, bufs, k, C.byref(n))
            if rc != OK:
                raise SkxError(rc, _lib.skx_engine_last_error(self._h).decode())
            for i in range(n.value):
                r = out[i]
                shape = self._npts.pop(r.ticket, None)
                d = {"ticket": r.ticket, "result": r.r.as_dict(), "t_admit": r.t_admit,
                     "t_done": r.t_done, "npoints": r.npoints}
                if want_density and shape is not None and r.npoints > 0:
                    d["rho"] = buf[:r.npoints].reshape(shape).copy()
                res.append(d)
            if n.value < k:
                break
        return res


def exported_symbols():
    """Names of the functions this binding expects the library to export."""
    return [n for n in dir(_lib) if n.startswith("skx_")]
