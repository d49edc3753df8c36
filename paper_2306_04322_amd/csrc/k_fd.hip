// Explicit finite-difference comparison step (forward Euler, 5-point /
// 7-point periodic Laplacian, every right-hand side at time t) and the
// forward-difference free-energy sums.
//
// The two step kernels give each thread V consecutive points along x, read
// as one vector of up to 16 bytes (V = 4 float or 2 double on large grids,
// fewer on small ones): each field's centre values and its y / z neighbours
// arrive as one vector load each, the x neighbours inside the vector come
// from registers and only the two at its ends are extra scalar loads, so a
// field costs 5 (2D) or 7 (3D) loads per V points instead of per point.
// The y and z neighbours are rows that neighbouring work-groups also read;
// on grids whose neighbour rows or planes fit in L2, each XCD takes a
// contiguous band of the grid so those re-reads stay in its own L2.  On
// larger 3D grids each thread instead marches along z over a few planes and
// keeps its neighbour planes in registers, and a work-group stages the
// current plane of its rows (plus one halo row on each side) in LDS for the
// y and x neighbours.  The energy kernel keeps one thread per point.
// Periodic wrap uses power-of-two masks instead of ghost layers.
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

// V consecutive points of one row, loaded and stored as one aligned vector
// (V * sizeof(T) <= 16 bytes).
template <typename T, int V>
struct alignas(sizeof(T) * V) FdVec {
  T v[V];
};

template <typename T, int V>
__device__ __forceinline__ FdVec<T, V> ld_vec(const T* __restrict__ p) {
  return *reinterpret_cast<const FdVec<T, V>*>(p);
}

template <typename T, int V>
__device__ __forceinline__ void st_vec(T* p, const T* v) {
  FdVec<T, V> w;
#pragma unroll
  for (int k = 0; k < V; ++k) w.v[k] = v[k];
  *reinterpret_cast<FdVec<T, V>*>(p) = w;
}

// The same store with the non-temporal hint: the marching kernels write
// their outputs once and never read them back, so the stores should not
// displace the neighbour planes the kernel re-reads from L2.
template <typename T, int V>
__device__ __forceinline__ void st_vec_nt(T* p, const T* v) {
  if constexpr (V == 1) {
    __builtin_nontemporal_store(v[0], p);
  } else {
    typedef T vt __attribute__((ext_vector_type(V)));
    vt w;
#pragma unroll
    for (int k = 0; k < V; ++k) w[k] = v[k];
    __builtin_nontemporal_store(w, reinterpret_cast<vt*>(p));
  }
}

// Neighbour offsets of the vector starting at point i0 (x0 = i0 mod nx, a
// multiple of V): the y and z neighbour vectors and the two x neighbours
// just outside the vector.
struct NbV {
  long long ym, yp, zm, zp, xl, xr;
};

template <typename T, int V>
__device__ __forceinline__ NbV neighbours_vec(const FdArgs<T>& a, long long i0) {
  const int x0 = int(i0 & (a.nx - 1));
  const int y = int((i0 >> a.lx) & (a.ny - 1));
  const int z = int(i0 >> (a.lx + a.ly));
  const long long row = i0 - x0;
  const long long plane = (long long)a.nx * a.ny;
  const long long zoff = (long long)z * plane;
  NbV n;
  n.xl = row + ((x0 - 1) & (a.nx - 1));
  n.xr = row + ((x0 + V) & (a.nx - 1));
  n.ym = zoff + (long long)((y - 1) & (a.ny - 1)) * a.nx + x0;
  n.yp = zoff + (long long)((y + 1) & (a.ny - 1)) * a.nx + x0;
  if (a.ndim == 3) {
    const long long rest = (long long)y * a.nx + x0;
    n.zm = (long long)((z - 1) & (a.nz - 1)) * plane + rest;
    n.zp = (long long)((z + 1) & (a.nz - 1)) * plane + rest;
  } else {
    n.zm = n.zp = i0;
  }
  return n;
}

// Laplacian of field v at the V points of the vector (centre values cv),
// in the same operation order as the per-point form.
template <typename T, int V>
__device__ __forceinline__ void lap_vec(const T* __restrict__ v, const FdVec<T, V>& cv, const NbV& n,
                                        const FdArgs<T>& a, T* out) {
  const FdVec<T, V> ym = ld_vec<T, V>(v + n.ym), yp = ld_vec<T, V>(v + n.yp);
  const T xl = v[n.xl], xr = v[n.xr];
  FdVec<T, V> zm, zp;
  if (a.ndim == 3) {
    zm = ld_vec<T, V>(v + n.zm);
    zp = ld_vec<T, V>(v + n.zp);
  }
#pragma unroll
  for (int k = 0; k < V; ++k) {
    const T c = cv.v[k];
    const T left = k == 0 ? xl : cv.v[k - 1];
    const T right = k == V - 1 ? xr : cv.v[k + 1];
    T r = (right - T(2) * c + left) * a.ix2 + (yp.v[k] - T(2) * c + ym.v[k]) * a.iy2;
    if (a.ndim == 3) r += (zp.v[k] - T(2) * c + zm.v[k]) * a.iz2;
    out[k] = r;
  }
}

// First point of this thread's vector.  Work-groups are dealt to the eight
// XCDs round-robin.  With `bands` set (the launch then rounds the group count
// up to a multiple of 8) XCD x instead takes the x-th contiguous eighth of
// the grid, so the neighbour rows or planes a group reads were mostly
// brought into that XCD's L2 by its neighbouring groups.
template <int V>
__device__ __forceinline__ long long fd_first_point(int bands) {
  unsigned b = blockIdx.x;
  if (bands) b = (b & 7u) * (gridDim.x >> 3) + (b >> 3);
  return ((long long)b * blockDim.x + threadIdx.x) * V;
}

// mu = df/dc - kappa_c lap(c);  eta_i' = eta_i - dt L (df/deta_i - kappa_eta lap(eta_i))
// FIXF: all PMAX order parameters in use (p fixed at compile time), as in
// the mu kernels below.
template <typename T, int PMAX, int V, bool FIXF = false>
__global__ void __launch_bounds__(256) fd_mu_kernel(FdArgs<T> a, int bands) {
  const long long i0 = fd_first_point<V>(bands);
  if (i0 >= a.P) return;
  const NbV n = neighbours_vec<T, V>(a, i0);
  const int p = FIXF ? PMAX : a.F - 1;
  const FdVec<T, V> cc = ld_vec<T, V>(a.in + i0);
  FdVec<T, V> ce[PMAX];
#pragma unroll
  for (int j = 0; j < PMAX; ++j)
    if (j < p) ce[j] = ld_vec<T, V>(a.in + (j + 1) * a.P + i0);
  T gc[V], ge[PMAX][V];
#pragma unroll
  for (int k = 0; k < V; ++k) {
    T eta[PMAX], g[PMAX];
#pragma unroll
    for (int j = 0; j < PMAX; ++j) {
      eta[j] = (j < p) ? ce[j].v[k] : T(0);
      g[j] = T(0);
    }
    fe_grad<T, PMAX>(a.fe, p, cc.v[k], eta, gc[k], g);
#pragma unroll
    for (int j = 0; j < PMAX; ++j) ge[j][k] = g[j];
  }
  T l[V], o[V];
  lap_vec<T, V>(a.in, cc, n, a, l);
#pragma unroll
  for (int k = 0; k < V; ++k) o[k] = gc[k] - a.kc * l[k];
  st_vec<T, V>(a.mu + i0, o);
#pragma unroll
  for (int j = 0; j < PMAX; ++j)
    if (j < p) {
      const T* e = a.in + (j + 1) * a.P;
      lap_vec<T, V>(e, ce[j], n, a, l);
#pragma unroll
      for (int k = 0; k < V; ++k) o[k] = ce[j].v[k] - a.dtL * (ge[j][k] - a.ke * l[k]);
      st_vec<T, V>(a.out + (j + 1) * a.P + i0, o);
    }
}

// c' = c + dt M lap(mu)
template <typename T, int V>
__global__ void __launch_bounds__(256) fd_c_kernel(FdArgs<T> a, int bands) {
  const long long i0 = fd_first_point<V>(bands);
  if (i0 >= a.P) return;
  const NbV n = neighbours_vec<T, V>(a, i0);
  const FdVec<T, V> cm = ld_vec<T, V>(a.mu + i0);
  const FdVec<T, V> c = ld_vec<T, V>(a.in + i0);
  T l[V], o[V];
  lap_vec<T, V>(a.mu, cm, n, a, l);
#pragma unroll
  for (int k = 0; k < V; ++k) o[k] = c.v[k] + a.dtM * l[k];
  st_vec<T, V>(a.out + i0, o);
}

// 3D grids whose neighbour planes do not fit in L2: each thread takes V
// consecutive x points of one (y, x) column and marches over ZB consecutive
// planes, keeping the planes z - 1, z and z + 1 of every field it reads in
// registers, so a thread loads each of its planes once per block of ZB
// planes instead of three times.  Same arithmetic, in the same order, as
// the one-plane kernels.
template <typename T, int V>
__device__ __forceinline__ void lap_vec_z(const T* __restrict__ v, const FdVec<T, V>& zm,
                                          const FdVec<T, V>& cv, const FdVec<T, V>& zp,
                                          long long row, int x0, long long ym, long long yp,
                                          const FdArgs<T>& a, T* out) {
  const FdVec<T, V> vm = ld_vec<T, V>(v + ym), vp = ld_vec<T, V>(v + yp);
  const T xl = v[row + ((x0 - 1) & (a.nx - 1))], xr = v[row + ((x0 + V) & (a.nx - 1))];
#pragma unroll
  for (int k = 0; k < V; ++k) {
    const T c = cv.v[k];
    const T left = k == 0 ? xl : cv.v[k - 1];
    const T right = k == V - 1 ? xr : cv.v[k + 1];
    T r = (right - T(2) * c + left) * a.ix2 + (vp.v[k] - T(2) * c + vm.v[k]) * a.iy2;
    r += (zp.v[k] - T(2) * c + zm.v[k]) * a.iz2;
    out[k] = r;
  }
}

struct ZCol {
  long long plane, rest, ymr, ypr;  // plane size; (y, x0) offset in a plane; y -/+ 1 rows
  int x0, z0;
};

// Work-groups are dealt to the eight XCDs round-robin; block b is mapped to
// the logical block of XCD b % 8's contiguous eighth of the grid (the launch
// rounds the group count up to a multiple of 8), so the groups of one z
// block that hold y-adjacent rows run on one XCD and find each other's rows
// (their y neighbours) in that XCD's L2.
template <typename T, int V>
__device__ __forceinline__ bool zcol(const FdArgs<T>& a, int zb, ZCol& q) {
  const long long nxv = a.nx / V;
  const long long per = nxv * a.ny;  // vectors per plane
  const unsigned b = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  const long long t = (long long)b * blockDim.x + threadIdx.x;
  if (t >= per * (a.nz / zb)) return false;
  const long long vin = t % per;
  q.z0 = int(t / per) * zb;
  q.x0 = int(vin % nxv) * V;
  const int y = int(vin / nxv);
  q.plane = (long long)a.nx * a.ny;
  q.rest = (long long)y * a.nx + q.x0;
  q.ymr = (long long)((y - 1) & (a.ny - 1)) * a.nx + q.x0;
  q.ypr = (long long)((y + 1) & (a.ny - 1)) * a.nx + q.x0;
  return true;
}

template <typename T, int PMAX, int V, bool FIXF = false>
__global__ void __launch_bounds__(256) fd_mu_z_kernel(FdArgs<T> a, int zb) {
  ZCol q;
  if (!zcol<T, V>(a, zb, q)) return;
  const int p = FIXF ? PMAX : a.F - 1;
  FdVec<T, V> m[PMAX + 1], c[PMAX + 1], n[PMAX + 1];
  const long long zm0 = (long long)((q.z0 - 1) & (a.nz - 1)) * q.plane + q.rest;
  const long long zc0 = (long long)q.z0 * q.plane + q.rest;
#pragma unroll
  for (int f = 0; f <= PMAX; ++f)
    if (f <= p) {
      m[f] = ld_vec<T, V>(a.in + f * a.P + zm0);
      c[f] = ld_vec<T, V>(a.in + f * a.P + zc0);
    }
  for (int k = 0; k < zb; ++k) {
    const int z = q.z0 + k;
    const long long zoff = (long long)z * q.plane;
    const long long i0 = zoff + q.rest;
    const long long zn = (long long)((z + 1) & (a.nz - 1)) * q.plane + q.rest;
#pragma unroll
    for (int f = 0; f <= PMAX; ++f)
      if (f <= p) n[f] = ld_vec<T, V>(a.in + f * a.P + zn);
    T gc[V], ge[PMAX][V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      T eta[PMAX], g[PMAX];
#pragma unroll
      for (int j = 0; j < PMAX; ++j) {
        eta[j] = (j < p) ? c[j + 1].v[e] : T(0);
        g[j] = T(0);
      }
      fe_grad<T, PMAX>(a.fe, p, c[0].v[e], eta, gc[e], g);
#pragma unroll
      for (int j = 0; j < PMAX; ++j) ge[j][e] = g[j];
    }
    const long long row = zoff + (q.rest - q.x0);
    T l[V], o[V];
    lap_vec_z<T, V>(a.in, m[0], c[0], n[0], row, q.x0, zoff + q.ymr, zoff + q.ypr, a, l);
#pragma unroll
    for (int e = 0; e < V; ++e) o[e] = gc[e] - a.kc * l[e];
    st_vec_nt<T, V>(a.mu + i0, o);
#pragma unroll
    for (int j = 0; j < PMAX; ++j)
      if (j < p) {
        const T* ev = a.in + (j + 1) * a.P;
        lap_vec_z<T, V>(ev, m[j + 1], c[j + 1], n[j + 1], row, q.x0, zoff + q.ymr, zoff + q.ypr, a, l);
#pragma unroll
        for (int e = 0; e < V; ++e) o[e] = c[j + 1].v[e] - a.dtL * (ge[j][e] - a.ke * l[e]);
        st_vec_nt<T, V>(a.out + (j + 1) * a.P + i0, o);
      }
#pragma unroll
    for (int f = 0; f <= PMAX; ++f) {
      m[f] = c[f];
      c[f] = n[f];
    }
  }
}

template <typename T, int V>
__global__ void __launch_bounds__(256) fd_c_z_kernel(FdArgs<T> a, int zb) {
  ZCol q;
  if (!zcol<T, V>(a, zb, q)) return;
  FdVec<T, V> m = ld_vec<T, V>(a.mu + (long long)((q.z0 - 1) & (a.nz - 1)) * q.plane + q.rest);
  FdVec<T, V> c = ld_vec<T, V>(a.mu + (long long)q.z0 * q.plane + q.rest);
  for (int k = 0; k < zb; ++k) {
    const int z = q.z0 + k;
    const long long zoff = (long long)z * q.plane;
    const long long i0 = zoff + q.rest;
    const FdVec<T, V> n = ld_vec<T, V>(a.mu + (long long)((z + 1) & (a.nz - 1)) * q.plane + q.rest);
    const FdVec<T, V> cu = ld_vec<T, V>(a.in + i0);
    T l[V], o[V];
    lap_vec_z<T, V>(a.mu, m, c, n, zoff + (q.rest - q.x0), q.x0, zoff + q.ymr, zoff + q.ypr, a, l);
#pragma unroll
    for (int e = 0; e < V; ++e) o[e] = cu.v[e] + a.dtM * l[e];
    st_vec_nt<T, V>(a.out + i0, o);
    m = c;
    c = n;
  }
}

// Marching kernels with the current plane staged in LDS.  A work-group of
// FD_ZL_WG threads owns a tile of R = FD_ZL_WG V / nx consecutive y rows
// (one vector per thread) of one block of planes; per plane it writes its
// centre vectors (kept in registers from the previous plane, as above) and
// the two halo rows y0 - 1 and y0 + R of every field it differentiates into
// LDS, and takes the y and x neighbours from there.  Each field is then
// read about (R + 2) / R times per step instead of once per neighbour row.
// Same arithmetic, in the same order, as the other FD step kernels.
constexpr int FD_ZL_WG = 512;

template <typename T, int V>
__device__ __forceinline__ void lap_lds(const T* __restrict__ tile, int r, int x0, int nx,
                                        const FdVec<T, V>& zm, const FdVec<T, V>& cv,
                                        const FdVec<T, V>& zp, const FdArgs<T>& a, T* out) {
  // tile rows: 0 = y0 - 1, 1..R = own rows, R + 1 = y0 + R
  const T* up = tile + (long long)r * nx;        // row y - 1
  const T* dn = tile + (long long)(r + 2) * nx;  // row y + 1
  const T* me = tile + (long long)(r + 1) * nx;
  const FdVec<T, V> vm = *reinterpret_cast<const FdVec<T, V>*>(up + x0);
  const FdVec<T, V> vp = *reinterpret_cast<const FdVec<T, V>*>(dn + x0);
  const T xl = me[(x0 - 1) & (nx - 1)], xr = me[(x0 + V) & (nx - 1)];
#pragma unroll
  for (int k = 0; k < V; ++k) {
    const T c = cv.v[k];
    const T left = k == 0 ? xl : cv.v[k - 1];
    const T right = k == V - 1 ? xr : cv.v[k + 1];
    T rr = (right - T(2) * c + left) * a.ix2 + (vp.v[k] - T(2) * c + vm.v[k]) * a.iy2;
    rr += (zp.v[k] - T(2) * c + zm.v[k]) * a.iz2;
    out[k] = rr;
  }
}

// Tile of this work-group: first row y0, first plane z0, and this thread's
// row r within the tile and x0.  Blocks are mapped to XCD-contiguous eighths
// of the grid as in zcol, so neighbouring tiles share an L2.
struct ZTile {
  long long plane;
  int y0, z0, r, x0, R;
};

template <typename T, int V>
__device__ __forceinline__ bool ztile(const FdArgs<T>& a, int zb, ZTile& q) {
  const int tpr = a.nx / V;  // threads per row
  q.R = FD_ZL_WG / tpr;
  const int tiles = a.ny / q.R;
  const unsigned b = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  if ((long long)b >= (long long)tiles * (a.nz / zb)) return false;
  q.y0 = int(b % tiles) * q.R;
  q.z0 = int(b / tiles) * zb;
  q.r = threadIdx.x / tpr;
  q.x0 = int(threadIdx.x - q.r * tpr) * V;
  q.plane = (long long)a.nx * a.ny;
  return true;
}

// Stage plane z of `nf` fields (field stride fs from base) into LDS: the
// centre vectors from registers, the halo rows from memory (threads of the
// first two rows of the tile load them).
template <typename T, int V, int NF>
__device__ __forceinline__ void stage_plane(T* lds, const T* __restrict__ base, long long fs,
                                            const FdVec<T, V>* cv, int nf, int z,
                                            const ZTile& q, const FdArgs<T>& a) {
  const int tsz = (q.R + 2) * a.nx;  // LDS values per field
#pragma unroll
  for (int f = 0; f < NF; ++f)
    if (f < nf)
      *reinterpret_cast<FdVec<T, V>*>(lds + f * tsz + (q.r + 1) * a.nx + q.x0) = cv[f];
  if (q.r < 2) {
    const int yh = q.r == 0 ? ((q.y0 - 1) & (a.ny - 1)) : ((q.y0 + q.R) & (a.ny - 1));
    const int lr = q.r == 0 ? 0 : q.R + 1;
    const long long off = (long long)z * q.plane + (long long)yh * a.nx + q.x0;
#pragma unroll
    for (int f = 0; f < NF; ++f)
      if (f < nf)
        *reinterpret_cast<FdVec<T, V>*>(lds + f * tsz + lr * a.nx + q.x0) =
            ld_vec<T, V>(base + f * fs + off);
  }
}

template <typename T, int PMAX, int V, bool FIXF = false>
__global__ void __launch_bounds__(FD_ZL_WG) fd_mu_zl_kernel(FdArgs<T> a, int zb) {
  extern __shared__ __align__(16) unsigned char fd_lds_raw[];
  T* lds = reinterpret_cast<T*>(fd_lds_raw);
  ZTile q;
  if (!ztile<T, V>(a, zb, q)) return;
  const int p = FIXF ? PMAX : a.F - 1;
  const int tsz = (q.R + 2) * a.nx;
  const long long rest = (long long)(q.y0 + q.r) * a.nx + q.x0;
  FdVec<T, V> m[PMAX + 1], c[PMAX + 1], n[PMAX + 1];
  const long long zm0 = (long long)((q.z0 - 1) & (a.nz - 1)) * q.plane + rest;
  const long long zc0 = (long long)q.z0 * q.plane + rest;
#pragma unroll
  for (int f = 0; f <= PMAX; ++f)
    if (f <= p) {
      m[f] = ld_vec<T, V>(a.in + f * a.P + zm0);
      c[f] = ld_vec<T, V>(a.in + f * a.P + zc0);
    }
  for (int k = 0; k < zb; ++k) {
    const int z = q.z0 + k;
    const long long i0 = (long long)z * q.plane + rest;
    const long long zn = (long long)((z + 1) & (a.nz - 1)) * q.plane + rest;
#pragma unroll
    for (int f = 0; f <= PMAX; ++f)
      if (f <= p) n[f] = ld_vec<T, V>(a.in + f * a.P + zn);
    stage_plane<T, V, PMAX + 1>(lds, a.in, a.P, c, p + 1, z, q, a);
    __syncthreads();
    T gc[V], ge[PMAX][V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      T eta[PMAX], g[PMAX];
#pragma unroll
      for (int j = 0; j < PMAX; ++j) {
        eta[j] = (j < p) ? c[j + 1].v[e] : T(0);
        g[j] = T(0);
      }
      fe_grad<T, PMAX>(a.fe, p, c[0].v[e], eta, gc[e], g);
#pragma unroll
      for (int j = 0; j < PMAX; ++j) ge[j][e] = g[j];
    }
    T l[V], o[V];
    lap_lds<T, V>(lds, q.r, q.x0, a.nx, m[0], c[0], n[0], a, l);
#pragma unroll
    for (int e = 0; e < V; ++e) o[e] = gc[e] - a.kc * l[e];
    st_vec_nt<T, V>(a.mu + i0, o);
#pragma unroll
    for (int j = 0; j < PMAX; ++j)
      if (j < p) {
        lap_lds<T, V>(lds + (j + 1) * tsz, q.r, q.x0, a.nx, m[j + 1], c[j + 1], n[j + 1], a, l);
#pragma unroll
        for (int e = 0; e < V; ++e) o[e] = c[j + 1].v[e] - a.dtL * (ge[j][e] - a.ke * l[e]);
        st_vec_nt<T, V>(a.out + (j + 1) * a.P + i0, o);
      }
    __syncthreads();
#pragma unroll
    for (int f = 0; f <= PMAX; ++f) {
      m[f] = c[f];
      c[f] = n[f];
    }
  }
}

template <typename T, int V>
__global__ void __launch_bounds__(FD_ZL_WG) fd_c_zl_kernel(FdArgs<T> a, int zb) {
  extern __shared__ __align__(16) unsigned char fd_lds_raw[];
  T* lds = reinterpret_cast<T*>(fd_lds_raw);
  ZTile q;
  if (!ztile<T, V>(a, zb, q)) return;
  const long long rest = (long long)(q.y0 + q.r) * a.nx + q.x0;
  FdVec<T, V> m = ld_vec<T, V>(a.mu + (long long)((q.z0 - 1) & (a.nz - 1)) * q.plane + rest);
  FdVec<T, V> c = ld_vec<T, V>(a.mu + (long long)q.z0 * q.plane + rest);
  for (int k = 0; k < zb; ++k) {
    const int z = q.z0 + k;
    const long long i0 = (long long)z * q.plane + rest;
    const FdVec<T, V> n = ld_vec<T, V>(a.mu + (long long)((z + 1) & (a.nz - 1)) * q.plane + rest);
    const FdVec<T, V> cu = ld_vec<T, V>(a.in + i0);
    stage_plane<T, V, 1>(lds, a.mu, 0, &c, 1, z, q, a);
    __syncthreads();
    T l[V], o[V];
    lap_lds<T, V>(lds, q.r, q.x0, a.nx, m, c, n, a, l);
#pragma unroll
    for (int e = 0; e < V; ++e) o[e] = cu.v[e] + a.dtM * l[e];
    st_vec_nt<T, V>(a.out + i0, o);
    __syncthreads();
    m = c;
    c = n;
  }
}

// partials[block] = {sum f(u), sum_d (dc/dx_d)^2, sum_i sum_d (deta_i/dx_d)^2, sum c}
// with forward differences, accumulated in double.  Each thread takes the V
// consecutive x points of one vector and adds them in increasing x.  Every
// value is loaded before any is used, so all loads are in flight together.
// Slots beyond F read field 0 again and are not used; in 2D the z neighbour
// vector is the centre one.
template <typename T, int PMAX, int V>
__global__ void __launch_bounds__(256) fd_energy_kernel(FdArgs<T> a) {
  __shared__ double red[4 * 4];
  const long long i0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * V;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (i0 < a.P) {
    const NbV n = neighbours_vec<T, V>(a, i0);
    const int p = a.F - 1;
    constexpr int FM = PMAX + 1;
    FdVec<T, V> vc[FM], vy[FM], vz[FM];
    T vr[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) {
      const T* v = a.in + (long long)(f < a.F ? f : 0) * a.P;
      vc[f] = ld_vec<T, V>(v + i0);
      vy[f] = ld_vec<T, V>(v + n.yp);
      vz[f] = ld_vec<T, V>(v + n.zp);
      vr[f] = v[n.xr];
    }
#pragma unroll
    for (int k = 0; k < V; ++k) {
      T eta[PMAX];
#pragma unroll
      for (int j = 0; j < PMAX; ++j) eta[j] = (j < p) ? vc[j + 1].v[k] : T(0);
      acc[0] += fe_density<T, PMAX>(a.fe, p, vc[0].v[k], eta);
      acc[3] += double(vc[0].v[k]);
    }
#pragma unroll
    for (int f = 0; f < FM; ++f) {
      if (f < a.F) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const double c = double(vc[f].v[k]);
          const double right = double(k == V - 1 ? vr[f] : vc[f].v[k + 1]);
          const double dx = (right - c) * a.ix;
          const double dy = (double(vy[f].v[k]) - c) * a.iy;
          double s = dx * dx + dy * dy;
          if (a.ndim == 3) {
            const double dz = (double(vz[f].v[k]) - c) * a.iz;
            s += dz * dz;
          }
          acc[f == 0 ? 1 : 2] += s;
        }
      }
    }
  }
  block_sum<4>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) a.partials[4 * blockIdx.x + k] = acc[k];
  }
}

// Points per thread of the two step kernels: the widest vector (16 bytes at
// most) that still leaves 512 work-groups of 256 threads, so small grids
// keep enough waves in flight to hide load latency.
template <typename T>
static int fd_vec_width(long long P) {
  for (int v = 16 / int(sizeof(T)); v > 1; v /= 2)
    if (P / (256LL * v) >= 512) return v;
  return 1;
}

#ifndef PF_FD_ZMARCH
#define PF_FD_ZMARCH 1  // 3D grids without bands: threads march along z
#endif
#ifndef PF_FD_ZLDS
#define PF_FD_ZLDS 1  // marching kernels with the current plane staged in LDS
#endif
#ifndef PF_FD_ZB
#define PF_FD_ZB 8  // planes per marching thread
#endif

// XCD bands pay while the three neighbour rows (2D) or planes (3D) of all F
// fields fit in half of one XCD's 4 MiB L2; beyond that (3D 256^3) the plain
// round-robin order, which sweeps the whole GPU through the grid together
// and shares the neighbour planes through the last-level cache, is faster.
template <typename T>
static int fd_bands(const FdArgs<T>& a) {
  const long long span = (a.ndim == 3 ? (long long)a.nx * a.ny : (long long)a.nx) * sizeof(T);
  return 3LL * a.F * span <= (2LL << 20) ? 1 : 0;
}

template <typename T, int PMAX, int V>
static int fd_go_v(int which, const FdArgs<T>& a, hipStream_t s) {
  const long long nv = a.P / V;  // nx >= 8 is a multiple of V
  const bool full = a.F == PMAX + 1;  // the mu kernel's p fixed at compile time
  const int bands = fd_bands(a);
  if (PF_FD_ZMARCH && a.ndim == 3 && !bands) {
    const int zb = a.nz < PF_FD_ZB ? a.nz : PF_FD_ZB;  // both powers of two
    // LDS-staged form: tiles of R >= 2 rows that divide Ny, with the plane
    // tiles of all F fields small enough for three work-groups per compute
    // unit (160 KiB of LDS); with fewer (FP64, F = 5, 256-point rows: two)
    // the register form was measured faster (3D 256^3 FD step 0.43 against
    // 0.39 ms)
    const int tpr = a.nx / V;
    const int R = tpr <= FD_ZL_WG ? FD_ZL_WG / tpr : 0;
    const size_t lds_mu = size_t(a.F) * (R + 2) * a.nx * sizeof(T);
    if (PF_FD_ZLDS && R >= 2 && R <= a.ny && lds_mu <= (160u << 10) / 3) {
      const long long nb = (long long)(a.ny / R) * (a.nz / zb);
      const int grid = int((nb + 7) / 8 * 8);
      if (which == 0 && full)
        hipLaunchKernelGGL((fd_mu_zl_kernel<T, PMAX, V, true>), dim3(grid), dim3(FD_ZL_WG), lds_mu, s, a, zb);
      else if (which == 0)
        hipLaunchKernelGGL((fd_mu_zl_kernel<T, PMAX, V>), dim3(grid), dim3(FD_ZL_WG), lds_mu, s, a, zb);
      else
        hipLaunchKernelGGL((fd_c_zl_kernel<T, V>), dim3(grid), dim3(FD_ZL_WG),
                           size_t(R + 2) * a.nx * sizeof(T), s, a, zb);
      return grid;
    }
    const int grid = int((nv / zb + 255) / 256 + 7) / 8 * 8;
    if (which == 0 && full) hipLaunchKernelGGL((fd_mu_z_kernel<T, PMAX, V, true>), dim3(grid), dim3(256), 0, s, a, zb);
    else if (which == 0) hipLaunchKernelGGL((fd_mu_z_kernel<T, PMAX, V>), dim3(grid), dim3(256), 0, s, a, zb);
    else hipLaunchKernelGGL((fd_c_z_kernel<T, V>), dim3(grid), dim3(256), 0, s, a, zb);
    return grid;
  }
  int grid = int((nv + 255) / 256);
  if (bands) grid = (grid + 7) / 8 * 8;
  if (which == 0 && full) hipLaunchKernelGGL((fd_mu_kernel<T, PMAX, V, true>), dim3(grid), dim3(256), 0, s, a, bands);
  else if (which == 0) hipLaunchKernelGGL((fd_mu_kernel<T, PMAX, V>), dim3(grid), dim3(256), 0, s, a, bands);
  else hipLaunchKernelGGL((fd_c_kernel<T, V>), dim3(grid), dim3(256), 0, s, a, bands);
  return grid;
}

template <typename T, int PMAX>
static int fd_go(int which, const FdArgs<T>& a, hipStream_t s) {
  if (which < 2) {
    const int v = fd_vec_width<T>(a.P);
    if constexpr (sizeof(T) == 4) {
      if (v == 4) return fd_go_v<T, PMAX, 4>(which, a, s);
    }
    if (v == 2) return fd_go_v<T, PMAX, 2>(which, a, s);
    return fd_go_v<T, PMAX, 1>(which, a, s);
  }
  // the energy pass: vectors as wide as the step kernels use
  const int v = fd_vec_width<T>(a.P);
  const int grid = int((a.P / v + 255) / 256);
  if constexpr (sizeof(T) == 4) {
    if (v == 4) {
      hipLaunchKernelGGL((fd_energy_kernel<T, PMAX, 4>), dim3(grid), dim3(256), 0, s, a);
      return grid;
    }
  }
  if (v == 2)
    hipLaunchKernelGGL((fd_energy_kernel<T, PMAX, 2>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((fd_energy_kernel<T, PMAX, 1>), dim3(grid), dim3(256), 0, s, a);
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
