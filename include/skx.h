/*
 * skx.h -- C ABI of libskx, a GPU (gfx950) implementation of the repeated
 * evaluation of the finite-temperature orbital-free free energy and its
 * potential on a periodic grid, and of the constrained density optimisation
 * that drives it.
 *
 * Method (arXiv 2601.23002, "Unlocking the Power of Orbital-Free Density
 * Functional Theory to Explore the Electronic Structure Under Extreme
 * Conditions"):
 *   F_s[n;T] = F_TF + F_vW + F_NL                       (Eq. (1))
 *   F_NL     = F0 + beta F1, beta = 1 is XWMF           (Eq. (2) and text)
 *   exchange-correlation: Perdew-Zunger LDA, adiabatic  (Methods)
 *   local pseudopotential per ion                       (Methods)
 * The paper prints no formula for the individual terms. This library uses
 * the following readings (each is a choice where the paper is silent):
 *   TF   exact uniform-gas free energy at T: f = n T eta - (2/3) n_T T I_3/2(eta),
 *        n = n_T I_1/2(eta), n_T = sqrt(2)/pi^2 T^(3/2)
 *   vW   (1/2) int |grad sqrt(n)|^2, temperature independent
 *   F0   V sum_G w(G) |f~(G)|^2, f = n^a; w chosen so that TF + vW + F0
 *        reproduce the finite-T Lindhard response at the mean density n0
 *        (the kernel is the second functional derivative at the mean
 *        valence density, Results section)
 *   F1   (1/3) int dF dn (w' * dF), dF = n^a - n0^a, dn = n - n0,
 *        w' = dw/dn0 at fixed T (first-order density dependence of the
 *        kernel along n0 + t(n - n0), the "line integral" correction)
 *   E_H  Hartree with the G = 0 term removed
 *   V_loc erf-smeared Coulomb -Z erf(r/rc)/r per ion through the structure
 *        factor, with its G = 0 (non-Coulomb) term; the real part of the
 *        plane-wave sum on even grids
 *   E_xc Perdew-Zunger 1981, unpolarised, temperature independent; the
 *        published fit (SKX_XC_PZ81) or the same branches joined C1 over
 *        0.99 <= rs <= 1.01 (SKX_XC_PZ81_C1, see the enum)
 *
 * Units: Hartree atomic units. Energies are totals over the cell.
 *
 * Conventions for every entry point:
 *   - Return codes only (no exceptions, no abort). SKX_OK = 0; a positive
 *     value is a completed call with a warning; a negative value is an
 *     error, described by skx_last_error(ctx) until the next call on ctx.
 *   - The caller owns every pointer it passes; the library keeps no caller
 *     pointer after a call returns (the serving engine copies its inputs).
 *   - Device pointers must be on the context's device. Real grid fields are
 *     C-order [n1][n2][n3] with n3 fastest, FP64 unless stated otherwise.
 *   - Work is queued on the context's stream; calls that return host
 *     scalars synchronise that stream. Calls on one context must not
 *     overlap; distinct contexts are independent.
 *   - State order: set_cell -> set_ions -> set_functional -> evaluate /
 *     optimise. set_cell invalidates ions and kernel tables.
 */
#ifndef SKX_H
#define SKX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SKX_OK = 0,
  SKX_NOT_CONVERGED = 1,   /* optimisation stopped at max_iter, in the line search, or after
                              150 iterations without a 10% gain in ||r|| (best state kept) */
  SKX_E_INVALID = -1,      /* bad size, lattice, parameter or pointer */
  SKX_E_STATE = -2,        /* call out of order */
  SKX_E_NOMEM = -3,        /* device allocation failed */
  SKX_E_DEVICE = -4,       /* HIP runtime error */
  SKX_E_NUMERIC = -5,      /* non-finite input or numerical blow-up */
  SKX_CANCELLED = 2        /* engine request cancelled before it finished (no density) */
};

/* term mask bits of skx_functional.terms */
enum {
  SKX_TERM_TF = 1, SKX_TERM_VW = 2, SKX_TERM_NL0 = 4, SKX_TERM_NL1 = 8,
  SKX_TERM_HARTREE = 16, SKX_TERM_LOCPP = 32, SKX_TERM_XC = 64, SKX_TERM_ALL = 127
};

/* Exchange-correlation (Methods: Perdew-Zunger LDA, adiabatic approximation).
 *   SKX_XC_PZ81     the published 1981 fit: correlation from the dilute
 *                   branch gamma / (1 + beta1 sqrt(rs) + beta2 rs) for rs >= 1,
 *                   the dense branch A ln rs + B + C rs ln rs + D rs below.
 *                   With the printed constants the branches jump by ~3e-5 Ha
 *                   in e_c and v_c at rs = 1, which floors a minimisation's
 *                   ||r|| (about 1e-5..1e-4) when the density straddles rs = 1.
 *   SKX_XC_PZ81_C1  the same branches joined over 0.99 <= rs <= 1.01 with the
 *                   weight w = 3t^2 - 2t^3, t = (rs - 0.99) / 0.02,
 *                   e_c = (1 - w) e_dense + w e_dilute, v_c the exact potential
 *                   of that e_c; equal to SKX_XC_PZ81 outside the window. */
enum { SKX_XC_NONE = 0, SKX_XC_PZ81 = 1, SKX_XC_PZ81_C1 = 2 };
/* Precision of the fields and transforms (sums and the optimiser's scalar
 * work are FP64 throughout).
 *   SKX_FP64   every field FP64.
 *   SKX_FP32   every field FP32.
 *   SKX_MIXED  FP32 until ||r|| < fp32_switch_gtol or stalls, then FP64 from
 *              that point to gtol (the precision policy of the batched path);
 *              the FP64 phase keeps its L-BFGS pairs (s, P y) in FP32, every
 *              inner product taken with the stored values. */
enum { SKX_FP64 = 0, SKX_FP32 = 1, SKX_MIXED = 2 };
enum { SKX_RHO = 0, SKX_SQRT_RHO = 1 };

typedef struct skx_ctx skx_ctx;

/* Create a context on HIP device `device`. `hip_stream` is a hipStream_t to
 * queue work on, or NULL for a library-owned stream. Errors: SKX_E_DEVICE. */
int skx_create(skx_ctx **out, int device, void *hip_stream);
void skx_destroy(skx_ctx *ctx);
/* Text of the last error on ctx (valid until the next call on ctx). */
const char *skx_last_error(const skx_ctx *ctx);

/* Periodic cell and grid of the problem (Methods, "Numerical calculations
 * for OFDFT and KSDFT": the OFDFT fields live on a uniform grid of stated
 * spacing in the periodic cell; the cell volume fixes the mean density
 * n0 = N_e / V and so r_s, Results). lattice: 9
 * doubles, rows a1, a2, a3 in bohr; this version accepts cubic cells only
 * (a1 = L x, a2 = L y, a3 = L z). n1, n2, n3: even and 5-smooth, 8..512.
 * The x axis is transformed as whole pencils in LDS: n1 <= 300 for FP64
 * work and n1 <= 310 for FP32 (the check is made when a solve is prepared,
 * SKX_E_INVALID); y-z planes beyond LDS run in row-pair and column chunks
 * (separate launches), so n2 and n3 may take any allowed size. Invalidates
 * ions and tables. Errors: SKX_E_INVALID. */
int skx_set_cell(skx_ctx *ctx, const double lattice[9], int n1, int n2, int n3);

/* Ions and their local pseudopotentials (Methods, "Numerical calculations
 * for OFDFT and KSDFT": the ion-electron interaction is a local
 * pseudopotential per species; its parameters are not printed, so here the
 * erf-smeared Coulomb -Z erf(r/rc)/r stands in, whose Fourier transform
 * -4 pi Z exp(-G^2 rc^2/4)/G^2 enters through the ionic structure factor).
 * nions host positions [nions][3] (cartesian bohr, any image, wrapped into
 * the cell), a species index per ion, and per species the valence zval and
 * erf width rc (bohr, > 0); N_e = sum of zval over ions. Builds V_loc(G) on
 * the device and the Ewald ion-ion energy. The arrays are copied; the
 * caller keeps ownership. Errors: SKX_E_INVALID (no ion, bad species
 * index, non-finite position, zval or rc <= 0), SKX_E_STATE (no cell),
 * SKX_E_NOMEM / SKX_E_DEVICE. */
int skx_set_ions(skx_ctx *ctx, int nions, const double *pos, const int *species, int nspecies,
                 const double *zval, const double *rc);

typedef struct {
  double T;          /* electron temperature, Ha, > 0 */
  double beta;       /* weight of F1 (Eq. (2)); 1 reproduces XWMF */
  double alpha;      /* exponent a of f = n^a in F0/F1, in (0.5, 1.5]; default 5/6 */
  unsigned terms;    /* SKX_TERM_* mask */
  int xc;            /* SKX_XC_PZ81, SKX_XC_PZ81_C1 or SKX_XC_NONE (clears SKX_TERM_XC) */
  int precision;     /* SKX_FP64, SKX_FP32 or SKX_MIXED */
} skx_functional;

/* Store the functional; kernel tables are rebuilt lazily. Errors:
 * SKX_E_INVALID, SKX_E_STATE. */
int skx_set_functional(skx_ctx *ctx, const skx_functional *fn);

typedef struct {
  double f_tf, e_vw, f_nl0, f_nl1;  /* f_nl1 already carries the factor beta */
  double e_h, e_loc, e_xc, e_ii;
  double free_energy;               /* electronic: f_tf + ... + e_xc */
  double total;                     /* free_energy + e_ii */
  double mu;                        /* int phi dE/dphi / (2 N_e) */
  double nelec;                     /* int n */
} skx_energy;

/* One evaluation of the free energy F[n;T] = F_TF + F_vW + F0 + beta F1
 * + E_H + E_loc + E_xc (Eq. (1), Eq. (2) and the Methods' XC and
 * pseudopotential) and of its potential, as dE/dphi with phi = sqrt(n).
 * in_dev: device field, n (SKX_RHO, phi = sqrt(n) is formed internally) or
 *   phi = sqrt(n) (SKX_SQRT_RHO). FP64 for SKX_FP64/SKX_MIXED, FP32 for SKX_FP32.
 * out_dev: NULL, or a device field of the same type receiving dE/dphi
 *   (the unconstrained gradient with respect to phi).
 * e: host struct receiving the energies. Synchronises the stream.
 * Errors: SKX_E_STATE, SKX_E_INVALID, SKX_E_NUMERIC (non-finite field or a
 * density beyond the Fermi-Dirac table). */
int skx_evaluate_energy_potential(skx_ctx *ctx, const void *in_dev, int in_kind, void *out_dev,
                                  skx_energy *e);

typedef struct {
  double gtol;              /* stop when ||r|| = (int r^2)^(1/2) < gtol, r = dE/dphi - 2 mu phi */
  int max_iter;             /* iteration cap */
  int lbfgs_m;              /* history length, 1..8 (5 by default) */
  double fp32_switch_gtol;  /* SKX_MIXED: FP32 phase stops below this ||r|| */
  int warm_start;           /* 1: rho_dev holds the starting density */
} skx_opt_params;

typedef struct {
  skx_energy e;
  int iters, evals, fp32_iters, fp32_evals;
  double gnorm;
  int status;               /* SKX_OK or SKX_NOT_CONVERGED (or a negative error) */
  int resets;
} skx_opt_result;

/* Minimise the free energy over n = phi^2 at fixed electron number with
 * limited-memory BFGS on phi (the minimisation the paper calls its SCF
 * iterations). rho_dev: FP64 device field; input guess if warm_start,
 * output density always. Returns SKX_OK, SKX_NOT_CONVERGED (best state
 * returned) or an error. SKX_MIXED: a numerical failure of the FP32 phase
 * ends the solve with that phase's status (no FP64 refinement from it);
 * skx_run_batch and the serving engine apply the same rule. Synchronises
 * the stream. */
int skx_optimize_density(skx_ctx *ctx, void *rho_dev, const skx_opt_params *p,
                         skx_opt_result *res);

/* Solve nctx independent problems together: every kernel of the step
 * sequence is one launch over all solves (uneven grids allowed, same
 * precision mode required). rho_devs[i] as in skx_optimize_density.
 * Each result equals that of solving alone (per-solve reductions are in a
 * fixed order). Errors as skx_optimize_density; res[i].status per solve. */
int skx_run_batch(skx_ctx **ctxs, int nctx, void **rho_devs, const skx_opt_params *p,
                  skx_opt_result *res);

/* Forces on the ions for molecular dynamics (Methods, molecular dynamics in
 * the NVT ensemble; the paper gives no force formula). At the minimising
 * density the energy is stationary in n at fixed N_e, so the force on ion I
 * is f_loc[I] + f_ii[I] (Hellmann-Feynman), in Hartree/bohr:
 *   f_loc: the local pseudopotential's force -dE_loc/dR_I from the density,
 *     sum over the grid's G of G v_I(G) Im[exp(i G.R_I) n~(G)];
 *   f_ii:  the Ewald ion-ion force -dE_ii/dR_I (same split as the energy).
 * in_dev: FP64 device field on the cell's grid, n (SKX_RHO) or phi = sqrt(n)
 *   (SKX_SQRT_RHO); read only; may be NULL when f_loc is NULL.
 * f_loc, f_ii: host arrays [nions][3] (ion order of skx_set_ions), either
 *   may be NULL, not both. Works in FP64 whatever the functional's precision.
 * Needs set_cell and set_ions (not set_functional). Allocates and frees a
 * scratch buffer of about nions (24 max(n1 n2 n3 / 4096, 16) + 16 (n1 + n2
 * + n3 / 2)) bytes on the ctx stream; synchronises it.
 * Errors: SKX_E_STATE (no cell or ions), SKX_E_INVALID (no output, missing
 * field, bad in_kind, a grid the FP64 plane kernels cannot take),
 * SKX_E_NOMEM / SKX_E_DEVICE. */
int skx_ion_forces(skx_ctx *ctx, const void *in_dev, int in_kind, double *f_loc, double *f_ii);

/* Static structure factors of one snapshot (Methods, static structure
 * factors): S_ab(q) = <n_a(q) n_b*(q)> / sqrt(N_a N_b) averaged over the
 * grid's wave vectors of equal |q|; the average over MD steps is the
 * caller's mean of these per-snapshot values. Readings:
 *   n_e(q) = integral n(r) exp(-i q.r) dr (N_e = sum of the ionic charges),
 *   n_i(q) = sum_I exp(-i q.R_I) over all ions as one species (N_i ions);
 *   shell s = g1^2 + g2^2 + g3^2 (|q| = 2 pi sqrt(s) / L), every grid index
 *   (index map, Nyquist -> -n/2) counted once; real parts of the products.
 * in_dev: FP64 device field, n (SKX_RHO) or sqrt(n) (SKX_SQRT_RHO).
 * s_ei, s_ee, s_ii: host arrays of len >= skx_num_shells(ctx) receiving the
 *   shell averages (0 for shells without grid vectors); count: host ints,
 *   grid wave vectors per shell. Any may be NULL, not all.
 * Needs set_cell and set_ions. Allocates and frees about
 * 24 n1 n2 (n3/2+1) + 16 nions (n1 + n2 + n3/2) bytes of device scratch;
 * the first call on a grid also builds the list of half-spectrum indices by
 * shell (4 n1 n2 (n3/2+1) bytes), kept by the ctx until the grid changes or
 * the ctx is destroyed. Synchronises the ctx stream.
 * Errors: SKX_E_STATE, SKX_E_INVALID (null field, bad in_kind, short len,
 * no output, a grid the FP64 plane kernels cannot take), SKX_E_DEVICE. */
int skx_structure_factors(skx_ctx *ctx, const void *in_dev, int in_kind, double *s_ei,
                          double *s_ee, double *s_ii, int *count, int len);

/* The integrated absolute deviation of two FP64 device densities on the
 * cell's grid, D = integral |a - b| dr = dV sum |a - b| (Eq. (3)), into
 * *out (host). Fixed-order reduction. Synchronises the ctx stream.
 * Errors: SKX_E_INVALID (null argument), SKX_E_STATE (no cell). */
int skx_density_deviation(skx_ctx *ctx, const void *a_dev, const void *b_dev, double *out);

/* skx_density_deviation for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and the same value, bit for bit, with the
 * partial sums and the result in a fixed device array of the library
 * (1025 doubles, 8200 bytes per device, held until the process ends), so
 * the call allocates and frees nothing. Every call on a device shares that
 * device's array: calls that overlap on one device (other contexts or
 * streams) race and must be serialised by the caller. Nothing needs
 * clearing between calls (each call writes every value it reads). Arguments
 * and errors as skx_density_deviation; SKX_E_INVALID also if the grid would
 * need more partial sums than the array holds (no grid of the accepted
 * sizes does: the partial sums are capped at 1024). */
int skx_density_deviation_noalloc(skx_ctx *ctx, const void *a_dev, const void *b_dev,
                                  double *out);

/* Kohn-Sham-assisted fit of beta for one configuration (Eq. (3); Methods,
 * optimisation of the beta parameter): the beta in [beta_lo, beta_hi]
 * minimising D(beta) = integral |n[beta] - n_ref| dr, n[beta] the minimising
 * density of the ctx's functional with beta replaced (skx_optimize_density
 * with p; warm-started from the previous solve after the first one). The
 * line minimisation is Brent's method (the one-parameter case of the
 * paper's Powell search), to an absolute tolerance xtol in beta. The
 * paper's beta over several configurations is the mean of the results.
 * rho_ref_dev: FP64 reference density (KSDFT in the paper). rho_dev: FP64
 *   device work density; a start guess if p->warm_start, on return the
 *   minimising density at *beta_out.
 * beta_out, dev_out (may be NULL), nsolves (may be NULL): host results.
 * The ctx's functional is left as it was. Synchronises the ctx stream.
 * Errors: SKX_E_INVALID (null arguments, empty interval, xtol <= 0),
 * SKX_E_STATE, or an error of the solves. */
int skx_fit_beta(skx_ctx *ctx, const void *rho_ref_dev, void *rho_dev, double beta_lo,
                 double beta_hi, double xtol, const skx_opt_params *p, double *beta_out,
                 double *dev_out, int *nsolves);

/* One velocity-Verlet step of the ions on the free-energy surface of the
 * functional (the paper's molecular dynamics, Methods; NVE here,
 * skx_md_step_nvt adds the thermostat), the density warm-started from the
 * previous minimum:
 *   v += (dt/2) F/m;  R += dt v (wrapped into the cell);  minimise the
 *   density (skx_optimize_density, warm_start forced) from rho_dev, or from
 *   max(2 n(t) - n(t - dt), n(t) / 10) once the ctx holds the density of the
 *   step before (kept by the ctx, an M-double buffer; only a start guess);
 *   F = f_loc + f_ii at the new minimum (skx_ion_forces);  v += (dt/2) F/m.
 * pos, vel, force: host [nions][3] in bohr, bohr per atomic time unit and
 *   Hartree/bohr, updated in place; force must hold the forces at pos on
 *   entry (skx_ion_forces at the current minimum).
 * mass: host [nspecies], electron masses. dt in atomic time units.
 * rho_dev: FP64 device density, the current minimum on entry, the new one
 *   on exit. p, res: as skx_optimize_density.
 * Returns SKX_OK or SKX_NOT_CONVERGED (the step is completed with the best
 * density) or an error of the calls above; SKX_E_INVALID for null
 * arguments, dt <= 0 or a non-positive mass (checked before anything
 * moves). After an error of the solve or the forces, pos and vel hold the
 * drifted values and force the old forces. */
int skx_md_step(skx_ctx *ctx, void *rho_dev, double *pos, double *vel, double *force,
                const double *mass, double dt, const skx_opt_params *p, skx_opt_result *res);

/* Nose-Hoover thermostat state for skx_md_step_nvt (the paper's MD runs in
 * the NVT ensemble with a Nose-Hoover thermostat, Methods). */
typedef struct {
  double T_ion;   /* target ionic temperature, Ha */
  double Q;       /* thermostat mass, Ha (atomic time)^2, > 0 */
  double xi;      /* thermostat velocity, 1 / atomic time; in/out */
  double eta;     /* thermostat position (for the conserved quantity); in/out */
} skx_nose_hoover;

/* skx_md_step in the NVT ensemble: the velocity-Verlet step wrapped in two
 * half steps of a single Nose-Hoover thermostat, each symmetric:
 *   xi += (h/2) G;  v *= exp(-xi h);  eta += xi h;  xi += (h/2) G,
 * h = dt/2, G = (2 K - g T_ion) / Q, K the ionic kinetic energy, g = 3 N_ion.
 * F[n_min(R)] + K + Q xi^2 / 2 + g T_ion eta is conserved. Arguments and
 * errors as skx_md_step; SKX_E_INVALID also for a NULL nh, Q <= 0,
 * T_ion < 0 or a non-finite xi. */
int skx_md_step_nvt(skx_ctx *ctx, void *rho_dev, double *pos, double *vel, double *force,
                    const double *mass, double dt, skx_nose_hoover *nh, const skx_opt_params *p,
                    skx_opt_result *res);

/* Pressure of the configuration for the equation of state (Table 1,
 * Fig. 3; the paper prints no stress formula): P = -dF/dV of the minimised
 * total free energy (electronic free energy + Ewald energy) at fixed ion
 * fractional positions, as the central difference between cells of volume
 * V (1 -+ eps) on the same grid, each minimised warm-started from rho_dev.
 * The ionic ideal-gas term N_i T_i / V is the caller's. Hartree/bohr^3.
 * rho_dev: FP64 density at the current minimum (read only). eps in (0, 0.1);
 * 1e-4 .. 1e-3 keeps the O(eps^2) error below 1e-6 of P. P (host) receives
 * the pressure, F_lo / F_hi (may be NULL) the two free energies. The ctx's
 * cell and ions are restored (V_loc and tables are rebuilt on next use).
 * Returns SKX_OK or SKX_NOT_CONVERGED (a solve hit max_iter) or an error. */
int skx_pressure(skx_ctx *ctx, const void *rho_dev, double eps, const skx_opt_params *p, double *P,
                 double *F_lo, double *F_hi);

/* ---- introspection (tests and tools) ---- */

/* Copy the shell tables w[s], w'[s], s = g1^2+g2^2+g3^2 = 0..len-1, to host. */
int skx_get_kernel_tables(skx_ctx *ctx, double *w_host, double *wp_host, int len);
/* Copy V_loc(G) (half spectrum [n1][n2][n3/2+1] complex, FP64 pairs) to host. */
int skx_get_vloc(skx_ctx *ctx, double *host);
/* Number of shells (3 (n/2)^2 + 1 for cubic grids) of the current cell. */
int skx_num_shells(const skx_ctx *ctx);
/* Universal Fermi-Dirac table on `device`: for host ratios u = n / n_T > 0
 * return eta with I_1/2(eta) = u and psi = eta - (2/3) I_3/2(eta) / u. */
int skx_fd_eval(int device, const double *u_host, double *eta_host, double *psi_host, long long n);
/* Forward then inverse transform of a host real field through the GPU FFT
 * passes (spectral multipliers off); returns the round trip in out_host and
 * the half spectrum [n1][n2][n3/2+1] complex (FP64 pairs, normalised 1/M)
 * in spec_host (may be NULL). Cell must be set; SKX_E_INVALID for grids
 * whose FP64 planes exceed LDS. */
int skx_fft_check(skx_ctx *ctx, const double *in_host, double *out_host, double *spec_host);

/* ---- instrumentation ---- */
/* Process-wide per-pass timing with HIP events recorded on the launch stream
 * around every launch of: 0 pass A's transform kernel, 1 pass B, 2 pass C,
 * 3 evaluation reductions, 4 optimiser update pass (+ its reduction),
 * 5 direction pass (+ its reduction), 6 preconditioner passes, 7 the
 * pointwise kernel that precedes pass A's transform, 8 the local force
 * kernel and 9 the Ewald force kernels of skx_ion_forces, 10 the structure
 * factor kernel of skx_structure_factors. skx_profile_read fills
 * up to n entries of total milliseconds and launch counts and returns the
 * number of passes. */
int skx_profile_enable(int on);
/* Passes timed while profiling is on: bit i for pass i of the list above
 * (all by default); the other passes launch without events. Returns the
 * previous mask. */
unsigned skx_profile_mask(unsigned mask);
int skx_profile_reset(void);
int skx_profile_read(double *ms, long long *launches, int n);

/* Process-wide: capture the optimisation driver's fixed chunk of step
 * sequences once per batch into a HIP graph and replay it (on = 1), or
 * launch every kernel eagerly (on = 0, the default: faster on the 64^3
 * scan, equal on larger grids). Results are identical either way. While
 * per-pass profiling is enabled the driver launches eagerly. Returns the
 * previous setting. */
int skx_set_graphs(int on);

/* Process-wide FFT autotuner (off by default). When on, the first set-up of
 * an instance of a given transform length and precision times whole
 * evaluations with each candidate radix order (radix 8 first; no radix 8;
 * odd radices first; small radices first) and keeps the fastest for the rest
 * of the process. Different orders round differently, so results are
 * reproducible bit for bit only with the same choices. Returns the previous
 * setting. */
int skx_set_autotune(int on);
/* Process-wide choice of the compile-time-shaped pass kernels, a bit mask
 * of the passes that use them: 1 pass A, 2 pass B, 4 pass C (default 7,
 * all). A batch whose solves all have a 64 x 64 x 64 grid runs the selected
 * passes with kernels built for that shape in place of the runtime-shaped
 * ones; passes A and C fold the real DC and Nyquist columns of each plane
 * into one complex y transform, so results differ from the runtime-shaped
 * kernels by rounding only. Applies to batches built after the call.
 * Returns the previous mask. */
int skx_set_shape_kernels(int mask);

/* Planes (y-z slices) whose half spectrum does not fit in LDS (FP64
 * beyond 128 x 128, FP32 beyond 192 x 192) run passes A and C in chunks of
 * row pairs and columns, the half spectrum staying in HBM between the z and
 * y transforms. force = 1 makes every plane take that path (for checking it
 * against the in-LDS kernels on small grids); 0 (default) uses it only where
 * needed. Results differ from the in-LDS kernels by rounding only. Applies
 * to batches built after the call. Returns the previous setting. */
int skx_set_plane_chunking(int force);

/* Radix order in use for length n in `precision` (SKX_FP64 / SKX_FP32):
 * writes up to max radices, returns their count or SKX_E_INVALID. */
int skx_get_radix_order(int n, int precision, int *radices, int max);

/* Time the three evaluation passes over a batch of nctx configured contexts
 * (uniform starting density, all in the precision of ctxs[0]): reps timed
 * repetitions after one warm-up; ms_out[0..2] receive the mean milliseconds
 * of passes A, B and C per launch. */
int skx_bench_eval(skx_ctx **ctxs, int nctx, int reps, double *ms_out);

/* ---- serving engine (continuous batching over requests) ---- */
typedef struct {
  double lattice[9];
  int n1, n2, n3;
  int nions;
  const double *pos;         /* host [nions][3] */
  const int *species;
  int nspecies;
  const double *zval, *rc;
  skx_functional fn;
  skx_opt_params opt;
  double t_arrival;          /* seconds; callers use skx_engine_clock's clock */
} skx_request;

typedef struct {
  uint64_t ticket;
  skx_opt_result r;
  double t_admit, t_done;    /* engine clock, seconds since engine creation */
  long long npoints;         /* n1*n2*n3 */
} skx_result;

typedef struct skx_engine skx_engine;
/* hbm_budget_bytes bounds the device memory of resident solves;
 * max_slots bounds how many solves are resident at once. The contexts of
 * up to max_slots finished solves are kept (their memory counted against
 * the budget) and reused by requests of the same grid, precision mode and
 * history length; they are freed when an admission needs the memory and at
 * skx_engine_destroy. */
int skx_engine_create(skx_engine **out, int device, size_t hbm_budget_bytes, int max_slots);
/* Copies the request; SKX_E_INVALID if it can never fit the budget. */
int skx_engine_submit(skx_engine *eng, const skx_request *req, uint64_t *ticket);
/* Admit queued requests (in arrival order) into free slots while their
 * device footprint fits the budget, then advance every resident solve by
 * two fused step sequences (one launch per kernel over all resident solves
 * of a precision; a step sequence is one trial evaluation of the line search
 * plus the history update when the trial is accepted). Mixed-precision
 * solves move from the FP32 to the FP64 group at the switch; finished solves
 * leave and free their slot. Returns the number of resident solves (>= 0) or
 * an error. A request that fails set-up is reported by poll with its
 * negative status. Results equal those of solving each request alone. */
int skx_engine_step(skx_engine *eng);
/* Collect finished results (up to max); the density of each is copied to
 * rho_host[i] when rho_host is non-NULL and rho_host[i] is non-NULL. */
int skx_engine_poll(skx_engine *eng, skx_result *out, double **rho_host, int max, int *n_out);
/* Cancel a queued or resident request: it leaves the engine at once (a
 * resident one frees its slot and budget share) and poll reports it with
 * status SKX_CANCELLED, no density (npoints 0). Other solves are unaffected: their
 * results stay those of solving alone. SKX_E_INVALID for an unknown ticket
 * or one already finished. */
int skx_engine_cancel(skx_engine *eng, uint64_t ticket);
/* Queued + resident + finished-but-unpolled requests. */
int skx_engine_pending(const skx_engine *eng);
/* Seconds since engine creation (the clock of t_admit / t_done). */
double skx_engine_clock(const skx_engine *eng);
/* Text of the engine's last error. */
const char *skx_engine_last_error(const skx_engine *eng);
void skx_engine_destroy(skx_engine *eng);

#ifdef __cplusplus
}
#endif
#endif
