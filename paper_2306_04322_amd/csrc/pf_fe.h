// Pointwise chemical free energy: density, gradient and Hessian-vector
// product, for the paper's f_chem (Sec. 2.1) and the Landau polynomial.
// The order-parameter count p is a runtime value <= PMAX; every loop over
// eta is unrolled to PMAX with a uniform guard, so the eta values stay in
// registers.
#pragma once

#include <hip/hip_runtime.h>

namespace pf {

enum { FE_POLY = 0, FE_PAPER = 1 };

template <typename T>
struct FeParams {
  int kind;
  T k[12];  // PAPER: rho2, c_alpha, c_beta, w, alpha
            // POLY:  c_alpha, c_beta, c_m, A, B, D, gamma, delta, eps
};

// df/dc and df/deta_i at one point.  PX > 0 fixes p = PX and FEK >= 0 the
// free-energy kind at compile time (the steady-state kernels); otherwise
// both come from the arguments.
template <typename T, int PMAX, int FEK = -1, int PX = 0>
__device__ __forceinline__ void fe_grad(const FeParams<T>& P, int p_rt, T c, const T* eta,
                                        T& gc, T* ge) {
  const int p = PX > 0 ? PX : p_rt;
  const int kind = FEK >= 0 ? FEK : P.kind;
  T s2 = T(0);
#pragma unroll
  for (int i = 0; i < PMAX; ++i)
    if (i < p) s2 += eta[i] * eta[i];
  if (kind == FE_PAPER) {
    // f_chem = rho2 (c-ca)^2 (1-H) + rho2 (cb-c)^2 H + w g, H = sum h(eta_i):
    //   df/dc      = 2 rho2 (c - ca) - 2 rho2 (cb - ca) H
    //   df/deta_i  = J h'(e) + w [2 e (1-e)(1-2e) + 4 alpha e (s2 - e^2)]
    // with J = rho2 [(cb-c)^2 - (c-ca)^2] = rho2 (cb-ca)(cb+ca-2c),
    // h(e) = e^3 (6e^2 - 15e + 10), h'(e) = 30 e^2 (1-e)^2.  Factored as
    //   df/deta_i = e { (1-e) [30 J e (1-e) + 2w - 4w e] + 4 w alpha (s2 - e^2) }
    // so every term keeps its factors of e and 1 - e (no cancellation near
    // e = 0 or 1) with about half the operations of the expanded form.
    const T rho2 = P.k[0], ca = P.k[1], cb = P.k[2], w = P.k[3], al = P.k[4];
    const T dcb = cb - ca;
    T H = T(0);
#pragma unroll
    for (int i = 0; i < PMAX; ++i)
      if (i < p) {
        const T e = eta[i];
        H += (e * e * e) * ((T(6) * e - T(15)) * e + T(10));
      }
    gc = T(2) * rho2 * ((c - ca) - dcb * H);
    const T A = T(30) * rho2 * dcb * ((cb + ca) - T(2) * c);  // 30 J
    const T w2 = T(2) * w, w4 = T(4) * w, wa4 = T(4) * w * al;
#pragma unroll
    for (int i = 0; i < PMAX; ++i)
      if (i < p) {
        const T e = eta[i];
        const T om = T(1) - e;
        const T inner = (A * e) * om + (w2 - w4 * e);
        ge[i] = e * (om * inner + wa4 * (s2 - e * e));
      }
  } else {
    const T ca = P.k[0], cb = P.k[1], cm = P.k[2], A = P.k[3], B = P.k[4], D = P.k[5];
    const T gam = P.k[6], dl = P.k[7], ep = P.k[8];
    const T dm = c - cm, da = c - ca, db = c - cb;
    gc = -A * dm + B * dm * dm * dm + D * da * da * da + D * db * db * db - gam * da * s2;
#pragma unroll
    for (int i = 0; i < PMAX; ++i)
      if (i < p) {
        const T e = eta[i];
        ge[i] = -gam * da * da * e + dl * e * e * e + T(2) * ep * e * (s2 - e * e);
      }
  }
}

// Free-energy density at one point, accumulated in double.
template <typename T, int PMAX>
__device__ __forceinline__ double fe_density(const FeParams<T>& P, int p, T cT, const T* etaT) {
  const double c = double(cT);
  double s2 = 0.0, pair = 0.0;
#pragma unroll
  for (int i = 0; i < PMAX; ++i)
    if (i < p) s2 += double(etaT[i]) * double(etaT[i]);
#pragma unroll
  for (int i = 0; i < PMAX; ++i)
    if (i < p) {
      const double e2 = double(etaT[i]) * double(etaT[i]);
      pair += e2 * (s2 - e2);
    }
  if (P.kind == FE_PAPER) {
    const double rho2 = P.k[0], ca = P.k[1], cb = P.k[2], w = P.k[3], al = P.k[4];
    double h = 0.0, g = 0.0;
#pragma unroll
    for (int i = 0; i < PMAX; ++i)
      if (i < p) {
        const double e = double(etaT[i]);
        h += e * e * e * (6.0 * e * e - 15.0 * e + 10.0);
        g += e * e * (1.0 - e) * (1.0 - e);
      }
    g += al * pair;
    return rho2 * (c - ca) * (c - ca) * (1.0 - h) + rho2 * (cb - c) * (cb - c) * h + w * g;
  } else {
    const double ca = P.k[0], cb = P.k[1], cm = P.k[2], A = P.k[3], B = P.k[4], D = P.k[5];
    const double gam = P.k[6], dl = P.k[7], ep = P.k[8];
    double q4 = 0.0;
#pragma unroll
    for (int i = 0; i < PMAX; ++i)
      if (i < p) {
        const double e2 = double(etaT[i]) * double(etaT[i]);
        q4 += e2 * e2;
      }
    const double dm = c - cm, da = c - ca, db = c - cb;
    return -A / 2 * dm * dm + B / 4 * dm * dm * dm * dm + D / 4 * da * da * da * da +
           D / 4 * db * db * db * db - gam / 2 * da * da * s2 + dl / 4 * q4 + ep / 2 * pair;
  }
}

// (H v) at one point, H = Hessian of f at (c, eta); v = (vc, ve[0..p-1]).
template <typename T, int PMAX>
__device__ __forceinline__ void fe_hvp(const FeParams<T>& P, int p, T c, const T* eta, T vc,
                                       const T* ve, T& oc, T* oe) {
  T s2 = T(0), dot = T(0);
#pragma unroll
  for (int i = 0; i < PMAX; ++i)
    if (i < p) {
      s2 += eta[i] * eta[i];
      dot += eta[i] * ve[i];
    }
  if (P.kind == FE_PAPER) {
    const T rho2 = P.k[0], ca = P.k[1], cb = P.k[2], w = P.k[3], al = P.k[4];
    const T jump = rho2 * ((cb - c) * (cb - c) - (c - ca) * (c - ca));
    T accc = T(2) * rho2 * vc;
#pragma unroll
    for (int i = 0; i < PMAX; ++i)
      if (i < p) {
        const T e = eta[i];
        const T om = T(1) - e;
        const T h1 = T(30) * e * e * om * om;
        const T h2 = T(60) * e * om * (T(1) - T(2) * e);
        const T hci = -T(2) * rho2 * (cb - ca) * h1;
        const T hii = jump * h2 + w * (T(2) * (T(1) - T(6) * e + T(6) * e * e) +
                                       T(4) * al * (s2 - e * e));
        accc += hci * ve[i];
        oe[i] = hci * vc + hii * ve[i] + T(8) * w * al * e * (dot - e * ve[i]);
      }
    oc = accc;
  } else {
    const T ca = P.k[0], cb = P.k[1], cm = P.k[2], A = P.k[3], B = P.k[4], D = P.k[5];
    const T gam = P.k[6], dl = P.k[7], ep = P.k[8];
    const T dm = c - cm, da = c - ca, db = c - cb;
    const T hcc = -A + T(3) * B * dm * dm + T(3) * D * da * da + T(3) * D * db * db - gam * s2;
    T accc = hcc * vc;
#pragma unroll
    for (int i = 0; i < PMAX; ++i)
      if (i < p) {
        const T e = eta[i];
        const T hci = -T(2) * gam * da * e;
        const T hii = -gam * da * da + T(3) * dl * e * e + T(2) * ep * (s2 - e * e);
        accc += hci * ve[i];
        oe[i] = hci * vc + hii * ve[i] + T(4) * ep * e * (dot - e * ve[i]);
      }
    oc = accc;
  }
}

// Work-group sum of NV doubles per lane, fixed reduction order (so the
// result is reproducible run to run).  `scratch` holds at least
// NV * (blockDim.x / 64) doubles.  The result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double* v, double* scratch) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwave = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_down(v[i], off, 64);
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) scratch[wave * NV + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < nwave; ++w) s += scratch[w * NV + i];
      v[i] = s;
    }
  }
}

}  // namespace pf
