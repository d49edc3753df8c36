// Fixed-order reduction kernel.
#include "pf_kernels.h"
#include "pf_launch.h"

namespace pf {

__global__ void __launch_bounds__(256) reduce_kernel(const double* __restrict__ partials, int n,
                                                     int width, double* __restrict__ out,
                                                     double s0, double s1, double s2, double s3,
                                                     int accumulate) {
  __shared__ double red[4 * 4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i < width) acc[i] += partials[(long long)r * width + i];
  }
  block_sum<4>(acc, red);
  if (threadIdx.x == 0) {
    const double sc[4] = {s0, s1, s2, s3};
    for (int i = 0; i < width; ++i) out[i] = (accumulate ? out[i] : 0.0) + acc[i] * sc[i];
  }
}

int reduce_launch(const double* partials, int n, int width, double* out, const double* scale4,
                  int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, s, partials, n, width, out, scale4[0],
                     scale4[1], scale4[2], scale4[3], accumulate);
  return 1;
}

}  // namespace pf
