// The integrated absolute density deviation of the beta fit (Eq. (3)):
// D = dV sum_r |a(r) - b(r)|, FP64. Per-workgroup partial sums over a fixed
// grid-stride assignment, then one workgroup adds the partials in order, so
// the value does not depend on scheduling.
#include "skx_internal.hpp"
#include "skx_host.hpp"

#include <algorithm>
#include <cmath>

namespace skx {

namespace {

constexpr int DEV_BLOCKS = 1024;       // workgroups (partial sums) of the deviation at most

__device__ __forceinline__ double block_sum(double v, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void k_absdiff_part(const double *a, const double *b, long long n,
                                                      double *part) {
  __shared__ double red[4];
  double v = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += 256LL * gridDim.x)
    v += fabs(a[i] - b[i]);
  const double t = block_sum(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_partials_sum(const double *part, int n, double scale,
                                                      double *out) {
  __shared__ double red[4];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += part[i];
  const double t = block_sum(v, red);
  if (threadIdx.x == 0) *out = scale * t;
}

}  // namespace

}  // namespace skx

// ---------------------------------------------------------------------------
// Fixed device scratch of skx_density_deviation_noalloc: the per-workgroup
// partial sums (at most DEV_BLOCKS of them) and the result, 8200 bytes, held
// by every device the library runs on until the process ends. Host code
// never uses the array's name (a host-side stand-in, not a device address):
// it uses the per-device address taken at set-up (init_noalloc_scratch).
// ---------------------------------------------------------------------------
static constexpr int NOALLOC_DOUBLES = skx::DEV_BLOCKS + 1;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace skx {

namespace {
double *g_scratch_ptr[64] = {nullptr};
}  // namespace

// With `dev` current (the library's per-device set-up): the device address
// of this device's copy of the fixed scratch.
hipError_t init_noalloc_scratch(int dev) {
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = static_cast<double *>(p);
  return hipSuccess;
}

int deviation_blocks(long long n) {
  return (int)std::min<long long>(DEV_BLOCKS, std::max<long long>(1, (n + 255) / 256));
}

hipError_t density_deviation(const double *a, const double *b, long long n, double dV,
                             double *part_dev, double *out_dev, hipStream_t s) {
  const int nb = deviation_blocks(n);
  hipLaunchKernelGGL(k_absdiff_part, dim3(nb), dim3(256), 0, s, a, b, n, part_dev);
  hipLaunchKernelGGL(k_partials_sum, dim3(1), dim3(256), 0, s, part_dev, nb, dV, out_dev);
  return hipGetLastError();
}

}  // namespace skx

// ---------------------------------------------------------------------------
// C ABI: the deviation with the fixed scratch above (no allocation or free).
// ---------------------------------------------------------------------------
extern "C" int skx_density_deviation_noalloc(skx_ctx *c, const void *a_dev, const void *b_dev,
                                             double *out) {
  using namespace skx;
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!a_dev || !b_dev || !out) return host::fail(c, SKX_E_INVALID, "null argument");
  if (!c->has_cell) return host::fail(c, SKX_E_STATE, "set_cell first");
  const long long M = (long long)c->n1 * c->n2 * c->n3;
  const int nb = deviation_blocks(M);
  if (nb + 1 > NOALLOC_DOUBLES)
    return host::fail(c, SKX_E_INVALID, "grid needs more partial sums than the fixed scratch holds");
  if (c->device < 0 || c->device >= 64 || !g_scratch_ptr[c->device])
    return host::fail(c, SKX_E_STATE, "fixed scratch not set up on this device");
  (void)hipSetDevice(c->device);
  hipStream_t s = c->stream;
  double *part = g_scratch_ptr[c->device];
  const double dV = c->L * c->L * c->L / (double)M;
  // every partial the second kernel reads is written by the first, and the
  // result by the second: nothing needs clearing between calls
  hipError_t e = density_deviation((const double *)a_dev, (const double *)b_dev, M, dV, part,
                                   part + nb, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, part + nb, sizeof(double), hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipStreamSynchronize(s);
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) return host::hip_fail(c, e, "deviation kernels");
  return SKX_OK;
}
