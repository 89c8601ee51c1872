// Internal declarations shared by the HIP translation units of libskx.
// Not part of the public C ABI (include/skx.h).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstdint>
#include <cstddef>

namespace skx {

constexpr int MMAX = 8;            // largest L-BFGS memory supported
constexpr int NFIELD = 4;          // transformed fields: phi, n, f, h
constexpr int MAX_STAGES = 8;      // FFT stages per axis
constexpr int PART_A = 4;          // pointwise-pass partial sums: f_tf, e_xc, nelec, nonfinite
constexpr int PART_B = 6;          // pass B: e_vw, e_h, f0, f1, e_loc, nonfinite
constexpr int PART_C = 2;          // pass C: int phi dE/dphi, nonfinite
constexpr int NDOT = 6 * MMAX + 10; // update-pass dot products
constexpr int CHUNK = 1024;        // grid points per workgroup in the vector passes
// Pass B column-block width on the runtime-shaped path and for the large
// cubic lengths whose pass B alone is compile-time shaped: 8 in FP64 and 16
// in FP32, halved (to 4 at least) while the x tile of n1 x (NFIELD tk)
// complex values exceeds 40 KB in FP64 or 80 KB in FP32, so that several
// workgroups share a CU.
__host__ __device__ constexpr int passb_width(int n1, int prec) {
  return prec == 0 ? (16 * n1 * (NFIELD * 8 + 1) > 40 * 1024 ? 4 : 8)
                   : (8 * n1 * (NFIELD * 16 + 1) <= 80 * 1024 ? 16
                      : (8 * n1 * (NFIELD * 8 + 1) <= 80 * 1024 ? 8 : 4));
}
// Larger cubic lengths of the serving mix whose pass B alone runs on the
// compile-time-shaped kernel (passes A and C on the runtime-shaped in-LDS
// or the split kernels).
__host__ __device__ constexpr bool shaped_b_only(int n) {
  return n == 90 || n == 96 || n == 100 || n == 108 || n == 120 || n == 128 || n == 144 ||
         n == 150 || n == 160 || n == 162 || n == 180 || n == 192;
}

constexpr int SPLIT_NT = 256;      // threads of the split plane kernels (planes beyond LDS)
constexpr int SPLIT_RPMAX = 16;    // row pairs per chunk at most
// Row pairs per chunk of the split plane kernels: every field's rows of the
// chunk (pitch n3 + 2) take at most 52 KB of LDS in FP64 and 26 KB in FP32
// (measured on MI355X against 36 KB and 26 KB in FP64, 52 KB in FP32:
// 192^3 FP64 passes A + C 1138 us against 1154 and 1154 for two solves,
// FP32 584 us against 630); and columns per column chunk (128-byte row
// segments in both precisions; 64- and 256-byte segments measured 5-12%
// slower at 192^3).
__host__ __device__ constexpr int split_rp(int n3) {
  return 832 / (n3 + 2) < 1 ? 1 : (832 / (n3 + 2) > SPLIT_RPMAX ? SPLIT_RPMAX : 832 / (n3 + 2));
}
__host__ __device__ constexpr int split_cc(int prec) { return prec == 0 ? 8 : 16; }
constexpr int UCHUNK = 4096;       // grid points per workgroup of the optimiser update on
                                   // large grids (fewer rows of its 58 partial sums)
constexpr int NPREFIX = 5;         // batch prefix-sum arrays: A, B, C, vector, update

// Which transformed fields are present (slot order phi, n, f, h).
enum FieldBits { F_PHI = 1, F_N = 2, F_F = 4, F_H = 8 };

// Optimiser phases of one solve; every kernel of the fixed step sequence
// checks the phase and skips solves it has nothing to do for.
enum Phase { PH_IDLE = 0, PH_EVAL_INIT = 1, PH_TRIAL = 2, PH_UPDATE = 3,
             PH_NEED_DIR = 4, PH_DONE = 5, PH_FAILED = 6, PH_EVAL_ONLY = 7 };

struct Plan {                      // 1D FFT plan for one axis length
  int n;
  int nst;
  unsigned rad;                    // radix of stage s in bits [4s, 4s+4)
  int tw;                          // offset of exp(-2 pi i k / n) in the twiddle bank
  // per stage s (Ns = product of the radices before s, RAD its radix):
  // ceil(2^32 / (n / RAD)) and ceil(2^32 / Ns) for division by
  // multiplication, and the twiddle stride n / (Ns RAD)
  unsigned long long m_nb[MAX_STAGES], m_ns[MAX_STAGES];
  int twstep[MAX_STAGES];
};

// Control state of one solve (device resident, FP64).
// The current point lives in buffer `par` of each pair (phi, r, P r); the
// trial point is written to buffer 1 - par and accepted by flipping par.
struct OptState {
  int phase, iters, evals, trials, k, head, status, resets;
  int m, max_iter, max_trials, reset_pending;
  int pair_ok, par, stall, stall_limit;
  double gtol, c1, theta_max, tolE_rel;
  double stall_factor;             // best ||r|| must drop below this fraction of itself
  double E, Et, mu, mut, rnorm, theta, g0, dnorm, rd, best_r;
  double gamma, cr, cphi;
  double cS[MMAX], cY[MMAX];
  double SY[MMAX][MMAX], YPY[MMAX][MMAX];   // s_i.y_j (upper), y_i.P y_j
  double Sr[MMAX], YPr[MMAX], Sphi[MMAX], PYphi[MMAX];
  double rr, rphi, rPr, phiPr;
  double e_acc[12];                // energy terms at the accepted point
  double e_trial[12];              // energy terms at the last evaluation
};

// Energy slots used in e_acc / e_trial
enum ESlot { E_TF = 0, E_VW, E_NL0, E_NL1, E_H, E_LOC, E_XC, E_NELEC, E_FREE, E_MU, E_NONFINITE, E_SPARE };

// Per-solve descriptor (device resident, POD).
struct SolveDev {
  int n1, n2, n3, nh, pitch;
  int fields, nf;                  // FieldBits mask and count
  int slot[NFIELD];                // spectrum slot of phi, n, f, h (-1 if absent)
  int nkb, tk;                     // pass-B column blocks and their width
  int nwg_vec;                     // workgroups of the vector passes
  int nwg_upd, uchunk;             // workgroups of the optimiser update and their points
  int mh;                          // history slots allocated (>= the solve's m)
  int debug;                       // 0 normal; FFT check: 1 forward x only, 2 inverse x only
  int big;                         // passes on the split plane kernels: 1 A, 2 C
  int rp, nrc;                     // split plane kernels: row pairs per chunk, chunks per plane
  int nrcp;                        // chunks per plane of the preconditioner (NFIELD rp row pairs)
  int rowsC;                       // rows of pass C partial sums (n1, n1 * nrc when split)
  unsigned terms;
  int xc;                          // 1 published PZ81 fit, 2 its C1-joined branches
  int hist32;                      // FP64 fields with the history S, P Y stored in FP32
  long long M, H;                  // H = n1*n2*pitch complex entries per spectrum
  double L, V, dV, ne, n0, n0a, T, beta, a, kscale, lnnT, inv_sqrt_ne, sqrt_ne;
  Plan p1, p2, p3;
  double kappa;                    // preconditioner P(G) = 1 / (G^2 + kappa)
  void *phi2[2], *r2[2], *pr2[2];  // current / trial point pairs (see OptState::par)
  void *grad, *d, *S, *Y;          // real fields (fp64 or fp32; S, Y fp32 if hist32); Y holds P y
  void *vpt;                       // w0 = 2 phi_t (T eta + v_xc) at the trial point (pass A -> C)
  void *fpt, *qpt;                 // coefficients c_P, c_Q of the fields P, Q (pass A -> C)
  void *npa;                       // n^a at the trial point (pointwise kernel -> pass A)
  void *spec, *vloc;                         // complex spectra
  const double *w, *wp;                      // shell tables
  double *partA, *partB, *partC, *partU, *partD;
  OptState *st;
};

struct FDTable {                   // nodes of eta(y), psi(y) on y = y0 + k h, y = ln(n/n_T)
  double y0, inv_h, h;
  int n;                           // intervals; n + 1 nodes
  const double *node;              // [n+1][4]: eta, d eta/dy, d2 eta/dy2, psi
};

// ---- launch wrappers (defined in the .hip files) ----
hipError_t build_twiddles(double *bank_dev, const int *sizes, const int *offsets, int nsizes,
                          hipStream_t s);
hipError_t build_fd_table(double *node_dev, double y0, double h, int n, hipStream_t s);
hipError_t build_kernel_tables(double *w, double *wp, int smax, double L, double n0, double T,
                               double a, const FDTable &fd, double *gas_out /* eta0, I_-1/2, dI_-1/2 */,
                               hipStream_t s);
hipError_t build_vloc(void *vloc, int prec, int n1, int n2, int n3, int pitch, double L,
                      int nions, const double *pos_dev, const int *species_dev,
                      int nspecies, const double *zval_dev, const double *rc_dev,
                      double2 *phase_scratch, hipStream_t s);
hipError_t ewald_energy(double L, int nions, const double *pos_dev, const double *charge_dev,
                        double *scratch_dev, int scratch_len, double *out_dev, hipStream_t s);
hipError_t debug_fd_eval(const double *u_dev, double *eta_dev, double *psi_dev, long long n,
                         const FDTable &fd, hipStream_t s);
hipError_t ion_phase_tables(double2 *ph, int nions, const double *pos_dev, int n1, int n2, int n3,
                            double L, hipStream_t s);
// forces on the ions (skx_forces.hip)
int force_row_blocks(int n1, int n2, int n3);   // partial sums per ion of the force kernels
hipError_t local_forces(const double2 *spec, int n1, int n2, int n3, int pitch, double L,
                        const double2 *ph, const int *order_dev, int nions, const int *species_dev,
                        const double *zval_dev, const double *rc_dev, double *part_dev,
                        double *out_dev, hipStream_t s);
int ewald_force_terms(double L);
// integrated absolute density deviation of the beta fit (skx_fit.hip);
// part_dev holds deviation_blocks(n) doubles
int deviation_blocks(long long n);
// Per-device set-up of the fixed scratch of skx_density_deviation_noalloc
// (call with `dev` current).
hipError_t init_noalloc_scratch(int dev);
hipError_t density_deviation(const double *a, const double *b, long long n, double dV,
                             double *part_dev, double *out_dev, hipStream_t s);
// static structure factors (skx_structure.hip)
hipError_t structure_items(const double2 *spec, int n1, int n2, int n3, int pitch, double V,
                           const double2 *ph, int nions, double *val, hipStream_t s);
hipError_t structure_shells(const double *val, const int *off, const int *idx, int nshell, int n3,
                            double norm_ei, double norm_ee, double norm_ii, double *out,
                            hipStream_t s);
hipError_t ewald_forces(double L, int nions, const double *pos_dev, const double *charge_dev,
                        double2 *sf_dev, double *part_dev, double *out_dev, hipStream_t s);

// The fixed step sequence over a batch of solves (defined in skx_passes.hip)
constexpr int MAX_GROUPS = 24;     // pass launch groups: runtime-shaped (by block width) + 21 lengths

// The solves of a batch whose evaluation passes run on one kernel family:
// the compile-time-shaped kernels of one cubic length, or the
// runtime-shaped (and split) kernels. Each group has its own copies of
// its solves' descriptors and prefix sums of its pass work items, so every
// launch covers only the solves it computes.
struct PassGroup {
  SolveDev *dev;                   // device array of the group's descriptors
  int nsolve;
  int shapeN;                      // 0: runtime-shaped; else the compile-time length
  int shape;                       // passes (1 A, 2 B, 4 C) on the compile-time-shaped kernels
  int tk;                          // pass B column-block width of every solve of the group
  int gridA, gridB, gridC;         // work items (workgroups) of the runtime-shaped passes
  const int *firstA, *firstB, *firstC;  // device prefix sums (nsolve+1)
  size_t ldsA, ldsB, ldsC;
  size_t ldsBp;                    // pass B of the preconditioner (one field)
  int accC_lds;                    // pass C accumulates in LDS (else in the output)
  int bigA, smallA, bigC, smallC;  // solves on the split / in-LDS kernels of passes A, C
  int krow, kcol, krowp;           // split kernels: most row-pair and column chunks per plane
  size_t ldsRow, ldsCol;           // and their LDS
};

struct BatchLaunch {
  SolveDev *dev;                   // device array of descriptors (every solve)
  int nsolve;
  int prec;                        // 0 fp64, 1 fp32
  const double *twbank;
  FDTable fd;
  int gridV, gridU;                // workgroups of the vector and update kernels
  const int *firstV, *firstU;      // device prefix sums (nsolve+1)
  int mh;                          // largest history length of the batch (1..MMAX)
  int ngroup;
  PassGroup grp[MAX_GROUPS];
};
// Device descriptors and prefix-sum ints a batch of n solves needs (the
// full batch plus the copies of its pass groups).
inline size_t batch_desc_count(int n) { return 2 * (size_t)n; }
inline size_t batch_first_count(int n) { return (size_t)(NPREFIX + 3) * (size_t)(n + MAX_GROUPS + 1); }
// Start/stop events for the next kernel launch while its pass is being timed
// (defined with the profiler), else false.
bool kernel_events(hipEvent_t *start, hipEvent_t *stop);
// A kernel launch that carries start/stop events of its own while its pass
// is being timed, so the time covers the kernel's execution only.
#define SKX_TIMED_LAUNCH(K, G, B, SH, S, ...)                             \
  do {                                                                  \
    hipEvent_t e0_, e1_;                                                \
    if (::skx::kernel_events(&e0_, &e1_))                               \
      hipExtLaunchKernelGGL(K, G, B, SH, S, e0_, e1_, 0, __VA_ARGS__);  \
    else                                                                \
      hipLaunchKernelGGL(K, G, B, SH, S, __VA_ARGS__);                  \
  } while (0)
// mask: 1 pass A (pointwise kernel + transform), 2 pass B, 4 pass C,
// 8 pointwise kernel only, 16 pass A transform only
hipError_t launch_eval(const BatchLaunch &b, hipStream_t s, int mask = 7);
hipError_t launch_finalize_eval(const BatchLaunch &b, hipStream_t s);
hipError_t launch_prec(const BatchLaunch &b, hipStream_t s, int mask = 7);  // P r_t, passes A|B|C
hipError_t launch_opt_update(const BatchLaunch &b, hipStream_t s);
hipError_t launch_opt_dir(const BatchLaunch &b, hipStream_t s);
hipError_t launch_normalize(const BatchLaunch &b, hipStream_t s);     // scale phi to N_e

}  // namespace skx
