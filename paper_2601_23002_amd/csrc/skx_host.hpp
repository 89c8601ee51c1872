// Host-side internals shared by the C ABI and the serving engine: the
// per-precision solve instance, the context, and the batch driver pieces.
#pragma once
#include "skx_internal.hpp"
#include "../../include/skx.h"

#include <string>
#include <vector>

namespace skx {
namespace host {

// One solve instance in one precision: device buffers + descriptor.
struct Instance {
  int prec = -1;                 // 0 fp64, 1 fp32
  size_t rsz = 0;
  void *mem = nullptr;           // one arena for every field of the solve
  size_t bytes = 0;
  SolveDev h{};                  // host mirror of the descriptor
  SolveDev *dptr = nullptr;      // device copy (batch of one)
  OptState *st = nullptr;        // device
  int *first = nullptr;          // device prefix sums for the batch of one [4][2]
  BatchLaunch bl{};
  bool vloc_ok = false;
  int m_alloc = 0;
  bool own_hist = true;          // false: S, P Y live in the FP32 instance (mixed)
};

}  // namespace host
}  // namespace skx

struct skx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  bool has_cell = false, has_ions = false, has_fn = false;
  double L = 0;
  int n1 = 0, n2 = 0, n3 = 0;
  std::vector<double> pos, zsp, rcsp;
  std::vector<int> species;
  int nspecies = 0;
  double ne = 0;
  skx_functional fn{};
  double *w = nullptr, *wp = nullptr;
  int smax = 0;
  int w_cap = 0;                   // shells the w / wp buffers hold
  bool tables_ok = false;
  double kappa = 1.0;              // preconditioner shift (uniform-gas TF curvature)
  double e_ii = 0;
  skx::host::Instance inst[2];
  double *ion_pos = nullptr, *ion_z = nullptr, *sp_z = nullptr, *sp_rc = nullptr;
  int *ion_sp = nullptr;
  int ion_cap = 0, sp_cap = 0;     // capacities of the device ion arrays
  double *md_prev = nullptr;       // density before the last MD step
  long long md_prev_n = 0;
  // half-spectrum indices listed by shell (structure factors), for grid sf_n
  int *sf_off = nullptr, *sf_idx = nullptr;
  int sf_n[3] = {0, 0, 0};
};

namespace skx {
namespace host {

int fail(skx_ctx *c, int code, const std::string &msg);
void free_instance(Instance &I);
int hip_fail(skx_ctx *c, hipError_t e, const char *what);
// Buffers, kernel tables and V_loc of precision instance `prec` (0 FP64, 1 FP32).
int prepare(skx_ctx *c, int prec, int m);
// Device bytes of one instance (the arena of ensure_instance plus
// descriptors); own_hist false for the FP64 instance of a mixed solve.
size_t instance_bytes(int n1, int n2, int n3, int prec, int m, bool own_hist);
void init_state(OptState &st, const skx_opt_params &p, double gtol, int from_rho, int prec);
int build_batch(skx_ctx *c, const std::vector<SolveDev> &hs, int prec, SolveDev *ddev,
                int *dfirst, BatchLaunch &bl, hipStream_t s);
hipError_t step_sequence(const BatchLaunch &bl, hipStream_t s);
void energy_from(const double *e, double e_ii, skx_energy *out);
// phi of instance I (buffer 0) := sqrt(n0) everywhere.
hipError_t start_uniform(skx_ctx *c, Instance &I, hipStream_t s);
// FP64 phi (buffer 0) of the FP64 instance from the FP32 phi of parity `par`.
hipError_t promote_phi(const Instance &I32, int par, Instance &I64, hipStream_t s);
// rho = phi^2 of parity `par` into an FP64 device field.
hipError_t square_out(const Instance &I, int par, double *rho, hipStream_t s);
// True when step sequences may be captured into HIP graphs (graphs on and
// per-pass event timing off).
bool graphs_enabled();
// Gather states[i]->phase of a batch into out[i] (device).
hipError_t gather_phases(const SolveDev *dev, int n, int *out, hipStream_t s);

}  // namespace host
}  // namespace skx
