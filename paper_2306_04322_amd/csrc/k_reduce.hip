// Fixed-order reduction kernel.
#include "pf_kernels.h"
#include "pf_launch.h"

namespace pf {

// One work-group of 256 lanes sums n records of W doubles.  Lane t adds the
// records t, t + 256, t + 512, ... in that order, then the work-group sum
// runs in a fixed order, so the result does not change from run to run.
// Eight records per lane are loaded before any of them is added, so eight
// loads are in flight rather than one; past the last record a lane loads
// the last record again and does not add it.
template <int W>
__global__ void __launch_bounds__(256) reduce_kernel(const double* __restrict__ partials, int n,
                                                     double* __restrict__ out, double s0, double s1,
                                                     double s2, double s3, int accumulate) {
  constexpr int B = 256, U = 8;
  __shared__ double red[4 * 4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = threadIdx.x; r0 < n; r0 += U * B) {
    double v[U][W];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = min(r0 + u * B, n - 1);
#pragma unroll
      for (int i = 0; i < W; ++i) v[u][i] = partials[(long long)r * W + i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (r0 + u * B < n) {
#pragma unroll
        for (int i = 0; i < W; ++i) acc[i] += v[u][i];
      }
  }
  block_sum<4>(acc, red);
  if (threadIdx.x == 0) {
    const double sc[4] = {s0, s1, s2, s3};
#pragma unroll
    for (int i = 0; i < W; ++i) out[i] = (accumulate ? out[i] : 0.0) + acc[i] * sc[i];
  }
}

int reduce_launch(const double* partials, int n, int width, double* out, const double* scale4,
                  int accumulate, hipStream_t s) {
  if (width == 2)
    hipLaunchKernelGGL(reduce_kernel<2>, dim3(1), dim3(256), 0, s, partials, n, out, scale4[0],
                       scale4[1], scale4[2], scale4[3], accumulate);
  else if (width == 4)
    hipLaunchKernelGGL(reduce_kernel<4>, dim3(1), dim3(256), 0, s, partials, n, out, scale4[0],
                       scale4[1], scale4[2], scale4[3], accumulate);
  else
    return -1;
  return 1;
}

}  // namespace pf
