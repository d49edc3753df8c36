// Explicit finite-difference comparison step (forward Euler, 5-point /
// 7-point periodic Laplacian, every right-hand side at time t) and the
// forward-difference free-energy sums.
//
// One thread per grid point, x fastest, so the centre and x-neighbour loads
// of a wavefront are contiguous and the y/z neighbours are the same rows
// shifted (served from cache).  Periodic wrap uses power-of-two masks
// instead of ghost layers.
#include "pf_kernels.h"
#include "pf_launch.h"

namespace pf {


struct Nb {
  long long xm, xp, ym, yp, zm, zp;
};

template <typename T>
__device__ __forceinline__ Nb neighbours(const FdArgs<T>& a, long long i) {
  const int x = int(i & (a.nx - 1));
  const int y = int((i >> a.lx) & (a.ny - 1));
  const int z = int(i >> (a.lx + a.ly));
  const long long row = i - x;
  const long long plane = (long long)a.nx * a.ny;
  Nb n;
  n.xm = row + ((x - 1) & (a.nx - 1));
  n.xp = row + ((x + 1) & (a.nx - 1));
  const long long zoff = (long long)z * plane;
  n.ym = zoff + (long long)((y - 1) & (a.ny - 1)) * a.nx + x;
  n.yp = zoff + (long long)((y + 1) & (a.ny - 1)) * a.nx + x;
  if (a.ndim == 3) {
    const long long rest = (long long)y * a.nx + x;
    n.zm = (long long)((z - 1) & (a.nz - 1)) * plane + rest;
    n.zp = (long long)((z + 1) & (a.nz - 1)) * plane + rest;
  } else {
    n.zm = n.zp = i;
  }
  return n;
}

template <typename T>
__device__ __forceinline__ T lap(const T* __restrict__ v, long long i, const Nb& n,
                                 const FdArgs<T>& a) {
  const T c = v[i];
  T r = (v[n.xp] - T(2) * c + v[n.xm]) * a.ix2 + (v[n.yp] - T(2) * c + v[n.ym]) * a.iy2;
  if (a.ndim == 3) r += (v[n.zp] - T(2) * c + v[n.zm]) * a.iz2;
  return r;
}

// mu = df/dc - kappa_c lap(c);  eta_i' = eta_i - dt L (df/deta_i - kappa_eta lap(eta_i))
template <typename T, int PMAX>
__global__ void __launch_bounds__(256) fd_mu_kernel(FdArgs<T> a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.P) return;
  const Nb n = neighbours(a, i);
  const int p = a.F - 1;
  T eta[PMAX], ge[PMAX];
#pragma unroll
  for (int j = 0; j < PMAX; ++j) {
    eta[j] = (j < p) ? a.in[(j + 1) * a.P + i] : T(0);
    ge[j] = T(0);
  }
  const T c = a.in[i];
  T gc;
  fe_grad<T, PMAX>(a.fe, p, c, eta, gc, ge);
  a.mu[i] = gc - a.kc * lap(a.in, i, n, a);
#pragma unroll
  for (int j = 0; j < PMAX; ++j)
    if (j < p) {
      const T* e = a.in + (j + 1) * a.P;
      a.out[(j + 1) * a.P + i] = eta[j] - a.dtL * (ge[j] - a.ke * lap(e, i, n, a));
    }
}

// c' = c + dt M lap(mu)
template <typename T>
__global__ void __launch_bounds__(256) fd_c_kernel(FdArgs<T> a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.P) return;
  const Nb n = neighbours(a, i);
  a.out[i] = a.in[i] + a.dtM * lap(a.mu, i, n, a);
}

// partials[block] = {sum f(u), sum_d (dc/dx_d)^2, sum_i sum_d (deta_i/dx_d)^2, sum c}
// with forward differences, accumulated in double.
template <typename T, int PMAX>
__global__ void __launch_bounds__(256) fd_energy_kernel(FdArgs<T> a) {
  __shared__ double red[4 * 4];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < a.P) {
    const Nb n = neighbours(a, i);
    const int p = a.F - 1;
    T eta[PMAX];
#pragma unroll
    for (int j = 0; j < PMAX; ++j) eta[j] = (j < p) ? a.in[(j + 1) * a.P + i] : T(0);
    const T c = a.in[i];
    acc[0] = fe_density<T, PMAX>(a.fe, p, c, eta);
    acc[3] = double(c);
    for (int f = 0; f < a.F; ++f) {
      const T* v = a.in + f * a.P;
      const double vc = double(v[i]);
      double dx = (double(v[n.xp]) - vc) * a.ix;
      double dy = (double(v[n.yp]) - vc) * a.iy;
      double s = dx * dx + dy * dy;
      if (a.ndim == 3) {
        const double dz = (double(v[n.zp]) - vc) * a.iz;
        s += dz * dz;
      }
      acc[f == 0 ? 1 : 2] += s;
    }
  }
  block_sum<4>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) a.partials[4 * blockIdx.x + k] = acc[k];
  }
}

template <typename T, int PMAX>
static int fd_go(int which, const FdArgs<T>& a, hipStream_t s) {
  const int grid = int((a.P + 255) / 256);
  if (which == 0) hipLaunchKernelGGL((fd_mu_kernel<T, PMAX>), dim3(grid), dim3(256), 0, s, a);
  else if (which == 1) hipLaunchKernelGGL((fd_c_kernel<T>), dim3(grid), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((fd_energy_kernel<T, PMAX>), dim3(grid), dim3(256), 0, s, a);
  return grid;
}

template <typename T>
static int fd_dispatch(int which, int p, const FdArgs<T>& a, hipStream_t s) {
  if (p <= 2) return fd_go<T, 2>(which, a, s);
  if (p <= 4) return fd_go<T, 4>(which, a, s);
  if (p <= 8) return fd_go<T, 8>(which, a, s);
  return -1;
}

template <>
int fd_launch<float>(int which, int p, const FdArgs<float>& a, hipStream_t s) {
  return fd_dispatch<float>(which, p, a, s);
}
template <>
int fd_launch<double>(int which, int p, const FdArgs<double>& a, hipStream_t s) {
  return fd_dispatch<double>(which, p, a, s);
}

}  // namespace pf
