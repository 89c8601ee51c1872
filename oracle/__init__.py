"""CPU oracle for the finite-temperature orbital-free DFT hot path.

TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The product path
(the HIP library and its Python binding) never imports, links or calls it.

Plain, slow, FP64 numpy code written from the paper's statement of the
method (Eq. (1) decomposition F_s = F_TF + F_vW + F_NL, Eq. (2)
F_NL = F0 + beta*F1, the Perdew-Zunger LDA of the Methods section) and
from the readings listed under "Readings" in each module's docstring where
the paper gives no formula. Nothing here shares code with the HIP path; the
only common module is the seeded input generator, which holds none of the
method's arithmetic.

Modules:
  fft        naive recursive mixed-radix complex DFT (factors 2, 3, 5)
  fermi      Fermi-Dirac integrals by composite Gauss-Legendre, inversion
  kernel     finite-T Lindhard response, kernel w(q) and dw/dn0
  xc         Perdew-Zunger 1981 LDA (unpolarised)
  ions       local pseudopotential via the structure factor, Ewald sum
  functional energy terms and dE/dphi on the periodic grid
  optimize   L-BFGS on sqrt(n) with the electron-count constraint
  forces     forces on the ions: local pseudopotential and Ewald
  structure  static structure factors S_ei, S_ee, S_ii of one snapshot
  fit        the beta fit of Eq. (3) against a reference density
  pressure   closed-form pressures (uniform gas, Ewald) for the equation of state

Parity status per function is stated in each module header. The only
functions without an independent pin ("parity unpinned") are the PZ81
correlation constants (the 1981 paper is not available here) and the F1
normalisation relative to the paper's XWMF/SKANEX (the paper prints no
functional values).
"""
