// Column-pass launcher instantiations (both precisions) and the fixed-order
// reduction kernel.
#include "pf_kernels.h"
#include "pf_launch.h"

namespace pf {

// Returns the number of logical work items (= partial-sum records written
// in energy mode).
template <typename T, int N>
static int claunch(int nouter, const ColArgs<T>& a, hipStream_t s) {
  using G = ColGeom<T, N>;
  const int tiles = (a.ncols + G::C - 1) / G::C;
  const int ngroups = a.F;
  const long long W = (long long)tiles * nouter * ngroups;
  const int nslots = int((W + 7) / 8);
  hipLaunchKernelGGL((col_kernel<T, N>), dim3(8 * nslots), dim3(G::WG), 0, s, a, tiles, nouter,
                     ngroups, nslots);
  return int(W);
}

template <typename T>
static int cdispatch(int n, int nouter, const ColArgs<T>& a, hipStream_t s) {
  switch (n) {
    case 8: return claunch<T, 8>(nouter, a, s);
    case 16: return claunch<T, 16>(nouter, a, s);
    case 32: return claunch<T, 32>(nouter, a, s);
    case 64: return claunch<T, 64>(nouter, a, s);
    case 128: return claunch<T, 128>(nouter, a, s);
    case 256: return claunch<T, 256>(nouter, a, s);
    case 512: return claunch<T, 512>(nouter, a, s);
    case 1024: return claunch<T, 1024>(nouter, a, s);
    case 2048: return claunch<T, 2048>(nouter, a, s);
    case 4096: return claunch<T, 4096>(nouter, a, s);
    default: return -1;
  }
}

template <>
int col_launch<float>(int n, int nouter, const ColArgs<float>& a, hipStream_t s) {
  return cdispatch<float>(n, nouter, a, s);
}
template <>
int col_launch<double>(int n, int nouter, const ColArgs<double>& a, hipStream_t s) {
  return cdispatch<double>(n, nouter, a, s);
}

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
