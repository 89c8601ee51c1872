"""Free energy and dE/dphi of the finite-temperature orbital-free functional
on a periodic grid (test infrastructure only).

Paper: F_s = F_TF + F_vW + F_NL (Eq. (1)), F_NL = F0 + beta F1 (Eq. (2)),
plus Perdew-Zunger LDA exchange-correlation and a local pseudopotential
(Methods). The total electronic free energy here is

  F[n] = F_TF + F_vW + F0 + beta F1 + E_H + E_loc + E_xc,   n = phi^2,

with the ion-ion Ewald energy E_ii reported beside it.

Readings (the paper prints no formula for these terms):
  vW     F_vW = 1/2 int |grad phi|^2 = (V/2) sum_G G^2 |phi~(G)|^2
         (temperature independent, coefficient one)
  F0     V sum_G w(G) |f~(G)|^2 with f = n^a, a = 5/6 by default
  F1     (1/3) int dF dn (w' * dF), dF = n^a - n0^a, dn = n - n0,
         = (V/3) sum_G Re(w'(G) f~(G) h~*(G)),  h = dF dn
  E_H    (V/2) sum_{G != 0} 4 pi |n~(G)|^2 / G^2
  E_loc  V sum_G Re(n~(G) V_loc*(G))

The gradient with respect to phi, under no constraint, is
  dE/dphi = sum_G G^2 phi~ e^{iGr}
          + 2 phi (T eta + v_H + V_loc + v_xc)
          + 2 phi a n^{a-1} (2 w*f + (beta/3) w'*h + dn (beta/3) w'*f)
          + 2 phi dF (beta/3) w'*f
where 2 phi a n^{a-1} is evaluated as 2 a sign(phi) |phi|^{2a-1} so that
every term stays finite as phi -> 0. Transforms are the full complex
3D DFT of `oracle.fft` (no real-to-complex shortcut).

Pins (tests): uniform-gas free energy from the Fermi-Dirac integrals,
vW closed forms (cosine, Gaussian orbital), Hartree energy of a Gaussian
charge, F0 and F1 closed forms at a = 1, finite-difference checks of every
potential term against its energy, gauge and symmetry invariances.
"""
from __future__ import annotations

import math

import numpy as np

from . import fermi, kernel, xc, ions
from .fft import fft3, ifft3

TERM_TF, TERM_VW, TERM_NL0, TERM_NL1, TERM_HARTREE, TERM_LOCPP, TERM_XC = (
    1, 2, 4, 8, 16, 32, 64)

ENERGY_KEYS = ("f_tf", "e_vw", "f_nl0", "f_nl1", "e_h", "e_loc", "e_xc")


class Problem:
    """All per-system data the evaluation needs (tables, V_loc, Ewald)."""

    def __init__(self, sys, with_ewald: bool = True, tables=None):
        self.sys = sys
        self.L = float(sys.L)
        self.n = tuple(int(x) for x in sys.n)
        self.V = self.L ** 3
        self.M = self.n[0] * self.n[1] * self.n[2]
        self.dV = self.V / self.M
        self.ne = float(np.sum(sys.zval))
        self.n0 = self.ne / self.V
        self.T = float(sys.T)
        self.beta = float(sys.beta)
        self.a = float(sys.alpha)
        self.terms = int(sys.terms)
        # XC_PZ81 (published fit) unless the system names the C1-joined variant
        self.xc = int(getattr(sys, "xc", xc.XC_PZ81))
        if self.xc == xc.XC_NONE:
            self.terms &= ~TERM_XC
        _, self.G2 = ions.gvectors(self.L, self.n)
        self.shell = ions.shells(self.n)
        nl = self.terms & (TERM_NL0 | TERM_NL1)
        need_wp = bool(self.terms & TERM_NL1) and self.beta != 0.0
        if tables is not None:
            self.w_shell, self.wp_shell = tables
        elif nl:
            self.w_shell, self.wp_shell = kernel.shell_tables(
                self.L, self.n, self.n0, self.T, self.a, need_wprime=need_wp)
        else:
            self.w_shell = self.wp_shell = np.zeros(int(self.shell.max()) + 1)
        self.wG = self.w_shell[self.shell]
        self.wpG = self.wp_shell[self.shell]
        if self.terms & TERM_LOCPP:
            self.vloc = ions.vloc_spectrum(self.L, self.n, sys.pos, sys.zval, sys.rc)
        else:
            self.vloc = np.zeros(self.n, dtype=np.complex128)
        self.e_ii = ions.ewald(self.L, sys.pos, sys.zval) if with_ewald else 0.0

    # ------------------------------------------------------------------
    def evaluate(self, phi: np.ndarray, need_grad: bool = True):
        phi = np.asarray(phi, dtype=np.float64)
        if phi.shape != self.n:
            raise ValueError("phi has the wrong shape")
        if not np.all(np.isfinite(phi)):
            raise FloatingPointError("non-finite input")
        T, a, beta, V, dV = self.T, self.a, self.beta, self.V, self.dV
        n = phi * phi
        e = {k: 0.0 for k in ENERGY_KEYS}
        vmult = np.zeros(self.n)          # multiplies 2 phi in the gradient
        grad = np.zeros(self.n)
        if self.terms & TERM_TF:
            eta, ftf, vtf = fermi.tf_terms(n, T)
            e["f_tf"] = dV * np.sum(ftf)
            vmult += np.where(n > 0, vtf, 0.0)
        if self.terms & TERM_XC:
            eps, vxc = xc.pz81(n, self.xc)
            e["e_xc"] = dV * np.sum(n * eps)
            vmult += vxc
        nt = fft3(n)
        pos = self.G2 > 0
        if self.terms & TERM_HARTREE:
            vh = np.zeros(self.n, dtype=np.complex128)
            vh[pos] = 4.0 * math.pi * nt[pos] / self.G2[pos]
            e["e_h"] = 0.5 * V * np.sum(np.real(vh * np.conj(nt)))
            if need_grad:
                vmult += np.real(ifft3(vh))
        if self.terms & TERM_LOCPP:
            e["e_loc"] = V * np.sum(np.real(nt * np.conj(self.vloc)))
            if need_grad:
                vmult += np.real(ifft3(self.vloc))
        if self.terms & TERM_VW:
            pt = fft3(phi)
            e["e_vw"] = 0.5 * V * np.sum(self.G2 * np.abs(pt) ** 2)
            if need_grad:
                grad += np.real(ifft3(self.G2 * pt))
        if self.terms & (TERM_NL0 | TERM_NL1):
            aphi = np.abs(phi)
            f = aphi ** (2.0 * a)
            dF = f - self.n0 ** a
            dn = n - self.n0
            ft = fft3(f)
            P = np.zeros(self.n)
            Q = np.zeros(self.n)
            if self.terms & TERM_NL0:
                e["f_nl0"] = V * np.sum(self.wG * np.abs(ft) ** 2)
                if need_grad:
                    P += 2.0 * np.real(ifft3(self.wG * ft))
            if (self.terms & TERM_NL1) and beta != 0.0:
                ht = fft3(dF * dn)
                F1 = V / 3.0 * np.sum(np.real(self.wpG * ft * np.conj(ht)))
                e["f_nl1"] = beta * F1
                if need_grad:
                    P += beta / 3.0 * np.real(ifft3(self.wpG * ht))
                    Q = beta / 3.0 * np.real(ifft3(self.wpG * ft))
            if need_grad:
                cP = 2.0 * a * np.sign(phi) * aphi ** (2.0 * a - 1.0)
                grad += cP * (P + dn * Q) + 2.0 * phi * dF * Q
        if need_grad:
            grad += 2.0 * phi * vmult
        F = sum(e[k] for k in ENERGY_KEYS)
        e["free_energy"] = F
        e["e_ii"] = self.e_ii
        e["total"] = F + self.e_ii
        e["nelec"] = dV * np.sum(n)
        if need_grad:
            e["mu"] = dV * np.sum(phi * grad) / (2.0 * self.ne)
            return e, grad
        return e, None

    def dot(self, x, y) -> float:
        return self.dV * float(np.sum(x * y))
