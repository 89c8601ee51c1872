// The integrated absolute density deviation of the beta fit (Eq. (3)):
// D = dV sum_r |a(r) - b(r)|, FP64. Per-workgroup partial sums over a fixed
// grid-stride assignment, then one workgroup adds the partials in order, so
// the value does not depend on scheduling.
#include "skx_internal.hpp"

#include <algorithm>

namespace skx {

namespace {

constexpr int DEV_BLOCKS = 1024;

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
