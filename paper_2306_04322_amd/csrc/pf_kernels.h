// Kernel templates of the FS step.
//
// Data layout in HBM (complex values interleaved re/im):
//   real fields   [F][Nz][Ny][Nx]            element type T
//   x-spectra     [G][Nz][Ny][Sx] + [G][Nz][Ny] c2<T>: row r holds the
//                                            real-to-complex transform along x
//                                            of row r, values kx = 0 .. Nx/2 - 1
//                                            at row stride Sx (128-byte
//                                            multiple); the Nyquist values
//                                            kx = Nx/2 of all rows follow as one
//                                            array (offset nyo in the field),
//                                            contiguous along y
// A "row" is one (z, y) line along x; rows = Ny * Nz.  Keeping the Nyquist
// column apart lets the strided passes cover kx < Nx/2 with full tiles and
// the Nyquist column with a few items that take many outer rows at once
// (in 3D a 16-column tile of it alone cost one work item in nine).
//
// Row pass: transforms along the contiguous x axis.  Depending on `flags`
// it loads real rows or inverse-transforms x-spectra back to real rows
// (C2R), optionally stores the real rows, evaluates the free-energy
// derivative and forward-transforms (R2C) the right-hand-side combinations,
// and accumulates double-precision sums.  Two forms: rowpass_kernel (one
// wavefront per transform, rows staged in an LDS row buffer) for rows of
// 512 and 1024 points, and xpass_kernel (one team of lanes per row, all
// fields of the row in registers) for shorter and longer rows (the launcher
// in k_row.inc chooses; the LDS form only where its buffer fits).
//
// Column pass (col_kernel): transforms along a strided axis (y, or z in
// 3D) for a tile of C consecutive x-spectrum columns.  Lanes are laid out
// column-fastest so every global access of a wavefront covers contiguous
// row segments of C values (128 bytes on axes shorter than 512 points, 16
// or 32 bytes on the longer ones, where tiles are narrower).  Modes: forward only, inverse only, the k-space
// update of Eq. (12)-(15) between a forward and an inverse transform, the
// adjoint multipliers, and the spectral gradient-energy sums.
#pragma once

#include <hip/hip_runtime.h>

#include "pf_fe.h"
#include "pf_fft.h"

// Tuning parameters (compile-time; the defaults are the measured best on
// MI355X for the 2D 1024^2 and 3D 256^3 workloads).
#ifndef PF_COL_CB_LONG_F32
#define PF_COL_CB_LONG_F32 4  // columns per tile, float, transform length >= 512
#endif
#ifndef PF_COL_CB_LONG_F64
#define PF_COL_CB_LONG_F64 2  // columns per tile, double, transform length >= 512
#endif
#ifndef PF_COL_MIN_WAVES
#define PF_COL_MIN_WAVES 1  // register budget of the column pass (waves per SIMD)
#endif
#ifndef PF_ROW_MIN_WAVES
#define PF_ROW_MIN_WAVES 1  // register budget of the steady-state row pass
#endif
#ifndef PF_ROW_ROWS_LONG
#define PF_ROW_ROWS_LONG 4  // rows per row-pass work-group, float, Nx = 1024
#endif
#ifndef PF_ROW_MULT_2048
#define PF_ROW_MULT_2048 2  // LDS-form work-group multiple, float, Nx = 2048 (now the adjoint only)
#endif
#ifndef PF_ROW_MULT_SHORT
#define PF_ROW_MULT_SHORT 1  // row-pass work-group multiple, float, Nx < 1024 (2 and 4 measured slower)
#endif
#ifndef PF_ROW_NW
#define PF_ROW_NW 4  // wavefronts per row-pass work-group (0: p_max + 1)
#endif
#ifndef PF_COL_PINGPONG
#define PF_COL_PINGPONG 1  // two LDS exchange areas in the column pass
#endif
#ifndef PF_FAST_RCP
#define PF_FAST_RCP 1  // float k-space multipliers through the hardware reciprocal
#endif
#ifndef PF_COL_WG_MAX_LONG
#define PF_COL_WG_MAX_LONG 1024  // largest column work-group, float, length 4096 (2-column tiles)
#endif
#ifndef PF_XROW_E8_F64_MIN
#define PF_XROW_E8_F64_MIN 4096  // double rows from this length: 8 elements per lane (measured: 4096 faster, 2048 slower)
#endif
#ifndef PF_XROW_MIN_WAVES
#define PF_XROW_MIN_WAVES 2  // register budget, register-form row pass (waves per SIMD)
#endif
#ifndef PF_COL_E_LONG_F32
#define PF_COL_E_LONG_F32 8  // elements per lane, float column transforms of length >= 512
#endif

namespace pf {

enum {
  X_LOAD_REAL = 1,   // read real rows (else C2R of s_in)
  X_STORE_REAL = 2,  // write the real rows to u_out
  X_FWD_DERIV = 4,   // R2C of [df/dc, eta_i - dt L df/deta_i] -> b_out fields 1..F
  X_FWD_RAW = 8,     // R2C of the F real rows as they are -> b_out
  X_ESUM = 16,       // double sums of f(u) and c -> partials[block][2]
  X_WITH_C = 32,     // with X_FWD_DERIV: also R2C of c -> b_out field 0
  X_CSUM = 64        // double sum of c only -> partials[block][1] ([0] = 0)
};

// 1 / x for the k-space multipliers (x >= 1).  float: the hardware
// reciprocal (error within 1 ulp) instead of the correctly rounded division
// sequence; double: the division.
template <typename T>
__device__ __forceinline__ T recip(T x) {
  if constexpr (sizeof(T) == 4 && PF_FAST_RCP) return __builtin_amdgcn_rcpf(x);
  else return T(1) / x;
}

template <typename T>
struct XArgs {
  const T* u_in;
  T* u_out;
  const c2<T>* s_in;
  c2<T>* b_out;
  const double2* twx;  // exp(-2 pi i q / Nx), q < Nx, double
  double* partials;
  long long fs_real;  // field stride of real arrays (elements)
  long long fs_spec;  // field stride of x-spectra (complex elements)
  long long nyo;      // offset of the Nyquist values within an x-spectrum field
  int rows, Sx, F, flags;
  FeParams<T> fe;
  T dtL;
};

// Row pass geometry for a real length NX.
template <typename T, int NX, int PMAX>
struct XGeom {
  static constexpr int NH = NX / 2;
  static constexpr int EW = (sizeof(T) == 8 && NX >= PF_XROW_E8_F64_MIN && PMAX <= 4) ? 8
                          : (sizeof(T) == 8 || PMAX > 4) ? 4 : 8;
  static constexpr int E = NH < EW ? NH : EW;
  static constexpr int TEAM = NH / E;
  static constexpr int ROWS = TEAM >= 64 ? 1 : 64 / TEAM;
  static constexpr int WG = ROWS * TEAM;
  static constexpr int REGION = lds_span(NH) + 1;  // LDS complex values per team
  // register budget of the fixed-flag instantiations: two work-groups per
  // SIMD where a work-group has at most one wavefront per SIMD (with up to
  // five fields; eight order parameters would spill)
  static constexpr int MIN_WAVES = (WG <= 256 && PMAX <= 4 && !(sizeof(T) == 8 && E == 8)) ? PF_XROW_MIN_WAVES : 1;
};

// Loads of one x-spectrum row for row_c2r: v[m] = X_k, k = t + TEAM m, and
// xn = X_NH (lane t = 0; zero elsewhere and for inactive rows).  Issued for
// all fields of a row before the first transform, so their latencies
// overlap.
template <typename T, int NX, int E>
__device__ __forceinline__ void row_load(c2<T>* v, c2<T>& xn, const c2<T>* __restrict__ src,
                                         const c2<T>* __restrict__ nyq, bool active, int t) {
  constexpr int TEAM = NX / 2 / E;
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = active ? src[t + TEAM * m] : mk<T>(T(0), T(0));
  xn = (active && t == 0) ? *nyq : mk<T>(T(0), T(0));
}

// C2R of one row loaded by row_load (v[m] = X_k, xn = X_NH) -> v[m] =
// (x[2k], x[2k+1]), k = t + TEAM m, with x the unnormalised inverse over the
// Hermitian extension (x_j = sum_k X_k exp(+2 pi i j k / NX)).
template <typename T, int NX, int E>
__device__ __forceinline__ void row_c2r(c2<T>* v, c2<T> xn, int t, c2<T>* my,
                                        const LaneTwiddles<T, NX / 2, E>& lt,
                                        const Twiddles<T, NX / 2, E>& tws) {
  constexpr int NH = NX / 2;
  constexpr int TEAM = NH / E;
#pragma unroll
  for (int m = 0; m < E; ++m) my[t + TEAM * m] = v[m];
  if (t == 0) my[NH] = xn;
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + TEAM * m;
    const c2<T> Y = conj<T>(my[NH - k]);
    const c2<T> s = add<T>(v[m], Y);
    const c2<T> d = cmulc<T>(sub<T>(v[m], Y), lt.w[m]);  // * exp(+2 pi i k / NX)
    v[m] = mk<T>(s.x - d.y, s.y + d.x);                 // s + i d
  }
  __syncthreads();
  team_fft<T, NH, E, true, 1>(v, t, my, tws);
}

// R2C of one row held as v[m] = (x[2k], x[2k+1]); writes X[0..NH-1] to dst
// and X[NH] to *nyq.
template <typename T, int NX, int E>
__device__ __forceinline__ void row_r2c(c2<T>* v, c2<T>* __restrict__ dst, c2<T>* __restrict__ nyq,
                                        bool active, int t,
                                        c2<T>* my, const LaneTwiddles<T, NX / 2, E>& lt,
                                        const Twiddles<T, NX / 2, E>& tws) {
  constexpr int NH = NX / 2;
  constexpr int TEAM = NH / E;
  team_fft<T, NH, E, false, 1>(v, t, my, tws);
#pragma unroll
  for (int m = 0; m < E; ++m) my[t + TEAM * m] = v[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + TEAM * m;
    const c2<T> Z = v[m];
    const c2<T> Zc = conj<T>(my[(NH - k) & (NH - 1)]);
    const c2<T> s = add<T>(Z, Zc);  // 2 A_k
    const c2<T> d = sub<T>(Z, Zc);  // 2 i B_k
    const c2<T> B2 = mk<T>(d.y, -d.x);  // 2 B_k
    const c2<T> WB = cmul<T>(B2, lt.w[m]);
    if (active) dst[k] = mk<T>(T(0.5) * (s.x + WB.x), T(0.5) * (s.y + WB.y));
    if (k == 0 && active) *nyq = mk<T>(T(0.5) * (s.x - B2.x), T(0.5) * (s.y - B2.y));
  }
  __syncthreads();
}

// Row pass, register form: one team of NX/(2E) lanes per row holds all F
// fields of its row in registers (the pointwise phase needs no LDS), and the
// x-spectra of all fields are loaded before the first transform.  Used for
// rows of up to 256 points and from 2048 points (the launcher chooses).
// FX >= 0 fixes the flags apart from X_STORE_REAL, and FEK >= 0 the
// free-energy kind with p = PMAX, as in rowpass_kernel below.
template <typename T, int NX, int PMAX, int FX = -1, int FEK = -1>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, XGeom<T, NX, PMAX>::WG),
                               amdgpu_waves_per_eu(FX >= 0 ? XGeom<T, NX, PMAX>::MIN_WAVES : 1)))
xpass_kernel(XArgs<T> a) {
  using G = XGeom<T, NX, PMAX>;
  constexpr int NH = G::NH, E = G::E, TEAM = G::TEAM, ROWS = G::ROWS;
  constexpr int FB = PMAX + 1;
  __shared__ c2<T> lds[ROWS * G::REGION];
  __shared__ double red[2 * (G::WG / 64 + 1)];
  const int lane = threadIdx.x;
  const int team = lane / TEAM;
  const int t = lane - team * TEAM;
  const int row = blockIdx.x * ROWS + team;
  const bool active = row < a.rows;
  const long long rrow = active ? row : 0;
  c2<T>* my = lds + team * G::REGION;
  const int F = FEK >= 0 ? PMAX + 1 : a.F;
  const int p = F - 1;
  const int flags = FX >= 0 ? (FX | (a.flags & X_STORE_REAL)) : a.flags;
  Twiddles<T, NH, E> tws;
  tws.load(t, a.twx, 2);
  LaneTwiddles<T, NH, E> lt;  // exp(-2 pi i k / NX), k = t + TEAM m
  lt.load(t, a.twx);

  c2<T> u[FB][E];
  if (flags & X_LOAD_REAL) {
#pragma unroll
    for (int f = 0; f < FB; ++f)
      if (f < F) {
        const c2<T>* src = reinterpret_cast<const c2<T>*>(a.u_in + f * a.fs_real + rrow * NX);
#pragma unroll
        for (int m = 0; m < E; ++m) u[f][m] = active ? src[t + TEAM * m] : mk<T>(T(0), T(0));
      }
  } else {
    c2<T> xn[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f)
      if (f < F)
        row_load<T, NX, E>(u[f], xn[f], a.s_in + f * a.fs_spec + rrow * a.Sx,
                           a.s_in + f * a.fs_spec + a.nyo + rrow, active, t);
#pragma unroll
    for (int f = 0; f < FB; ++f)
      if (f < F) row_c2r<T, NX, E>(u[f], xn[f], t, my, lt, tws);
  }

  if ((flags & X_STORE_REAL) && active) {
#pragma unroll
    for (int f = 0; f < FB; ++f)
      if (f < F) {
        c2<T>* dst = reinterpret_cast<c2<T>*>(a.u_out + f * a.fs_real + rrow * NX);
#pragma unroll
        for (int m = 0; m < E; ++m) dst[t + TEAM * m] = u[f][m];
      }
  }

  if (flags & (X_ESUM | X_CSUM)) {
    double acc[2] = {0.0, 0.0};
    if (active) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const T c = h ? u[0][m].y : u[0][m].x;
          if (flags & X_ESUM) {
            T eta[PMAX];
#pragma unroll
            for (int i = 0; i < PMAX; ++i) eta[i] = (i < p) ? (h ? u[1 + i][m].y : u[1 + i][m].x) : T(0);
            acc[0] += fe_density<T, PMAX>(a.fe, p, c, eta);
          }
          acc[1] += double(c);
        }
      }
    }
    block_sum<2>(acc, red);
    if (threadIdx.x == 0) {
      a.partials[2 * blockIdx.x + 0] = acc[0];
      a.partials[2 * blockIdx.x + 1] = acc[1];
    }
  }

  if (flags & X_FWD_DERIV) {
    // outputs: 0 -> c (X_WITH_C only), 1 -> df/dc, 2 + i -> eta_i - dt L df/deta_i
    c2<T> gcv[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      T gcx, gcy;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        T eta[PMAX], ge[PMAX];
#pragma unroll
        for (int i = 0; i < PMAX; ++i) {
          eta[i] = (i < p) ? (h ? u[1 + i][m].y : u[1 + i][m].x) : T(0);
          ge[i] = T(0);
        }
        const T c = h ? u[0][m].y : u[0][m].x;
        T gc;
        fe_grad<T, PMAX, FEK, (FEK >= 0 ? PMAX : 0)>(a.fe, p, c, eta, gc, ge);
        if (h) gcy = gc; else gcx = gc;
#pragma unroll
        for (int i = 0; i < PMAX; ++i)
          if (i < p) {
            const T b = eta[i] - a.dtL * ge[i];
            if (h) u[1 + i][m].y = b; else u[1 + i][m].x = b;
          }
      }
      gcv[m] = mk<T>(gcx, gcy);
    }
    if (flags & X_WITH_C)
      row_r2c<T, NX, E>(u[0], a.b_out + rrow * a.Sx, a.b_out + a.nyo + rrow, active, t, my, lt, tws);
    row_r2c<T, NX, E>(gcv, a.b_out + 1 * a.fs_spec + rrow * a.Sx, a.b_out + 1 * a.fs_spec + a.nyo + rrow,
                      active, t, my, lt, tws);
#pragma unroll
    for (int i = 0; i < PMAX; ++i)
      if (i < p)
        row_r2c<T, NX, E>(u[1 + i], a.b_out + (2 + i) * a.fs_spec + rrow * a.Sx,
                          a.b_out + (2 + i) * a.fs_spec + a.nyo + rrow, active, t, my, lt, tws);
  } else if (flags & X_FWD_RAW) {
#pragma unroll
    for (int f = 0; f < FB; ++f)
      if (f < F)
        row_r2c<T, NX, E>(u[f], a.b_out + f * a.fs_spec + rrow * a.Sx, a.b_out + f * a.fs_spec + a.nyo + rrow,
                          active, t, my, lt, tws);
  }
}

// Input half of a C2R by one wavefront team: pairs each X_k of the
// x-spectrum row (src[0..NH-1], X_NH = *nyq) with conj(X_{NH-k}) and leaves in v[m] the
// complex sequence whose length-NH inverse FFT gives the real row as pairs
// (x[2k], x[2k+1]), k = t + TEAM m.  `lt` holds exp(-2 pi i k / (2 NH)).
// float rows of Nx <= 512 (several teams per wavefront): the row is read
// once from global memory and the mirrored values come from the team's LDS
// area `ar`, which saves the registers of a second set of loads (one more
// wavefront per SIMD on 256-point rows); otherwise both reads come from
// global memory (measured faster where occupancy does not change).
template <typename T, int NH, int E>
__device__ __forceinline__ void wave_c2r_pre(c2<T>* v, const c2<T>* __restrict__ src,
                                             const c2<T>* __restrict__ nyq, c2<T>* ar,
                                             int t, const LaneTwiddles<T, NH, E>& lt) {
  constexpr int TEAM = NH / E;
  constexpr bool STAGE = sizeof(T) == 4 && TEAM < 64;
  c2<T> X[E];
#pragma unroll
  for (int m = 0; m < E; ++m) X[m] = src[t + TEAM * m];
  if constexpr (STAGE) {
    const c2<T> xn = t == 0 ? *nyq : src[0];
#pragma unroll
    for (int m = 0; m < E; ++m) ar[pad(t + TEAM * m)] = X[m];
    if (t == 0) ar[pad(NH)] = xn;
    team_sync<true>();
  }
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + TEAM * m;
    const c2<T> Y = conj<T>(STAGE ? ar[pad(NH - k)] : (k == 0 ? *nyq : src[(NH - k) & (NH - 1)]));
    const c2<T> sm = add<T>(X[m], Y);
    const c2<T> d = cmulc<T>(sub<T>(X[m], Y), lt.w[m]);  // * exp(+2 pi i k / NX)
    v[m] = mk<T>(sm.x - d.y, sm.y + d.x);
  }
  if constexpr (STAGE) team_sync<true>();
}

// ---------------------------------------------------------------------------
// Row pass, one wavefront per transform.  The work-group owns ROWS rows and
// stages them in an LDS row buffer of F + 1 real rows each (slot 0 = c,
// slot 1 = df/dc, slot 2 + i = eta_i, so the right-hand sides overwrite
// their inputs in place).  Phase 1: each wavefront inverse-transforms (C2R)
// one (row, field) x-spectrum, using that field's slot as its FFT exchange
// area, and leaves the real row in the slot.  Phase 2: all lanes evaluate
// the pointwise part (real-row store, double sums, derivative) on the row
// buffer.  Phase 3: each wavefront forward-transforms (R2C) one (row,
// output) slot and stores its x-spectrum.  FFT exchanges inside a phase are
// wavefront-local, so only the two phase boundaries synchronise the
// work-group.  Usable when a transform fits one wavefront (Nx <= 2048) and
// the row buffer fits LDS; the forward launcher takes it for 512 and 1024
// points, the adjoint wherever it is usable (else xpass_kernel /
// adj_row_kernel).
// SM selects the form for grids with few rows: one row per work-group and
// just enough wavefronts for its F transforms, which spreads a small grid
// over more compute units than 1024-point work-groups would.
template <typename T, int NX, int PMAX, bool SM = false>
struct RGeom {
  static constexpr int NH = NX / 2;
  static constexpr int E = NH >= 512 ? (NH / 64 < 16 ? NH / 64 : 16) : (NH < 8 ? NH : 8);
  static constexpr int TEAM = NH / E;
  static constexpr bool WAVE_OK = TEAM <= 64;
  static constexpr int UPW = WAVE_OK ? 64 / TEAM : 1;  // transforms per wavefront
  static constexpr int SLOTS = PMAX + 2;
  static constexpr int SLOT_C = lds_span(NH);  // complex values per slot (padded layout)
  static constexpr long ROW_BYTES = long(SLOTS) * SLOT_C * 2 * long(sizeof(T));
  // Float rows: MULT times the rows and the wavefronts of the base form
  // (1024/Nx rows or one row, PF_ROW_NW wavefronts).  Meant to spread the
  // transforms of rows whose F does not divide over the wavefronts (F = 5
  // over 4) evenly over the CU's SIMDs; measured faster at Nx = 1024 (four
  // rows) and 2048 (two rows) only.  (The forward row pass now takes the
  // register form at 2048 points; the adjoint row pass keeps this one.)
  static constexpr int BASE_ROWS = SM ? 1 : (NX >= 1024 ? 1 : 1024 / NX);
  static constexpr int MULT_WANT = NX == 2048 ? PF_ROW_MULT_2048 : NX == 1024 ? PF_ROW_ROWS_LONG : PF_ROW_MULT_SHORT;
  static constexpr bool MULTI = !SM && NX <= 2048 && sizeof(T) == 4 && PF_ROW_NW > 0 && MULT_WANT > 1 &&
                                PF_ROW_NW * MULT_WANT <= 16 &&
                                MULT_WANT * BASE_ROWS * ROW_BYTES <= 160 * 1024;
  static constexpr int MULT = MULTI ? MULT_WANT : 1;
  static constexpr int ROWS = BASE_ROWS * MULT;
  static constexpr int NW = SM ? (PMAX + UPW) / UPW  // ceil((PMAX + 1) / UPW)
                               : (PF_ROW_NW > 0 ? PF_ROW_NW * MULT : PMAX + 1);
  static constexpr int WG = 64 * NW;
  static constexpr long LDS_BYTES = long(ROWS) * ROW_BYTES;
  static constexpr bool FITS = WAVE_OK && LDS_BYTES <= (MULTI ? 160 : 96) * 1024;
  // register budget: enough waves per SIMD for four work-groups per CU
  static constexpr int MIN_WAVES = (sizeof(T) == 4 && PMAX <= 4) ? PF_ROW_MIN_WAVES : 1;
};

// FX >= 0 fixes the flags at compile time apart from X_STORE_REAL (the
// steady-state step gets a lean instantiation); FX = -1 reads them from the
// arguments.  FEK >= 0
// fixes the free-energy kind and requires p = PMAX.
template <typename T, int NX, int PMAX, int FX, int FEK = -1, bool SM = false>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, RGeom<T, NX, PMAX, SM>::WG),
                               amdgpu_waves_per_eu(FX >= 0 ? RGeom<T, NX, PMAX, SM>::MIN_WAVES : 1)))
rowpass_kernel(XArgs<T> a) {
  using G = RGeom<T, NX, PMAX, SM>;
  constexpr int NH = G::NH, E = G::E, TEAM = G::TEAM, UPW = G::UPW, ROWS = G::ROWS;
  constexpr int NW = G::NW, SL = G::SLOTS, WG = G::WG, SC = G::SLOT_C;
  static_assert(G::FITS, "row pass v2 does not fit this size");
  // slot (r, s) holds real row r of slot s as complex pairs (x[2q], x[2q+1])
  // at padded position pad(q)
  __shared__ __align__(16) c2<T> rb[ROWS * SL * SC];
  __shared__ double red[2 * (NW + 1)];
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int unit = lane / TEAM;
  const int t = lane - unit * TEAM;
  const int row0 = blockIdx.x * ROWS;
  const int F = FEK >= 0 ? PMAX + 1 : a.F;  // the fixed-kind instantiations have p = PMAX
  const int p = F - 1;
  // the store flag stays a run-time choice even in the fixed instantiations,
  // so a recomputation that also stores the states runs the same arithmetic
  const int flags = FX >= 0 ? (FX | (a.flags & X_STORE_REAL)) : a.flags;
  Twiddles<T, NH, E> tws;
  tws.load(t, a.twx, 2);
  LaneTwiddles<T, NH, E> lt;  // exp(-2 pi i k / NX), k = t + TEAM m
  lt.load(t, a.twx);

  // phase 1: real rows into the row buffer
  if (flags & X_LOAD_REAL) {
    // (with F fixed the trip count is a constant and the loads of all
    // iterations can be issued before the first store)
    const int n2 = ROWS * F * NH;
#pragma unroll
    for (int q = tid; q < n2; q += WG) {
      const int x2 = q % NH;
      const int rf = q / NH;
      const int f = rf % F;
      const int r = rf / F;
      const int row = row0 + r;
      if (row < a.rows) {
        const c2<T>* src = reinterpret_cast<const c2<T>*>(a.u_in + f * a.fs_real + (long long)row * NX);
        c2<T>* ar = rb + (r * SL + (f == 0 ? 0 : f + 1)) * SC;
        ar[pad(x2)] = src[x2];
      }
    }
  } else {
    const int njobs = ROWS * F;
    for (int base = wave * UPW; base < njobs; base += NW * UPW) {
      const int j = base + unit;
      const int r = j / F;
      const int f = j - r * F;
      if (j < njobs && row0 + r < a.rows) {
        const c2<T>* src = a.s_in + f * a.fs_spec + (long long)(row0 + r) * a.Sx;
        const c2<T>* nyq = a.s_in + f * a.fs_spec + a.nyo + (row0 + r);
        c2<T>* ar = rb + (r * SL + (f == 0 ? 0 : f + 1)) * SC;
        c2<T> v[E];
        wave_c2r_pre<T, NH, E>(v, src, nyq, ar, t, lt);
        team_fft<T, NH, E, true, 1, true>(v, t, ar, tws);
        team_sync<true>();
#pragma unroll
        for (int m = 0; m < E; ++m) ar[pad(t + TEAM * m)] = v[m];
      }
    }
  }
  __syncthreads();

  // phase 2: pointwise work on the row buffer, two adjacent points per lane
  double acc[2] = {0.0, 0.0};
  const int pp = FEK >= 0 ? PMAX : p;
  const int npairs = ROWS * NH;
  for (int q = tid; q < npairs; q += WG) {
    const int r = q / NH;
    const int x2 = q - r * NH;
    const int row = row0 + r;
    if (row < a.rows) {
      c2<T>* pt = rb + r * SL * SC + pad(x2);
      const c2<T> c = pt[0];
      c2<T> eta[PMAX];
#pragma unroll
      for (int i = 0; i < PMAX; ++i) eta[i] = (i < pp) ? pt[(2 + i) * SC] : mk<T>(T(0), T(0));
      if (flags & X_STORE_REAL) {
        const long long off = (long long)row * NH + x2;
        reinterpret_cast<c2<T>*>(a.u_out)[off] = c;
#pragma unroll
        for (int i = 0; i < PMAX; ++i)
          if (i < pp) reinterpret_cast<c2<T>*>(a.u_out + (1 + i) * a.fs_real)[off] = eta[i];
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const T ch = h ? c.y : c.x;
        T e[PMAX];
#pragma unroll
        for (int i = 0; i < PMAX; ++i) e[i] = h ? eta[i].y : eta[i].x;
        if (flags & X_ESUM) acc[0] += fe_density<T, PMAX>(a.fe, pp, ch, e);
        if (flags & (X_ESUM | X_CSUM)) acc[1] += double(ch);
        if (flags & X_FWD_DERIV) {
          T gc, ge[PMAX];
#pragma unroll
          for (int i = 0; i < PMAX; ++i) ge[i] = T(0);
          fe_grad<T, PMAX, FEK, (FEK >= 0 ? PMAX : 0)>(a.fe, pp, ch, e, gc, ge);
          if (h) pt[SC].y = gc; else pt[SC].x = gc;
#pragma unroll
          for (int i = 0; i < PMAX; ++i)
            if (i < pp) {
              const T bi = e[i] - a.dtL * ge[i];
              if (h) pt[(2 + i) * SC].y = bi; else pt[(2 + i) * SC].x = bi;
            }
        }
      }
    }
  }
  if (flags & (X_ESUM | X_CSUM)) {
    block_sum<2>(acc, red);
    if (tid == 0) {
      a.partials[2 * blockIdx.x + 0] = acc[0];
      a.partials[2 * blockIdx.x + 1] = acc[1];
    }
  }
  __syncthreads();

  // phase 3: forward transforms of the slots
  if (flags & (X_FWD_DERIV | X_FWD_RAW)) {
    const bool deriv = (flags & X_FWD_DERIV) != 0;
    const int skip = (deriv && !(flags & X_WITH_C)) ? 1 : 0;  // output 0 (c) not needed
    const int nout = deriv ? F + 1 - skip : F;
    const int njobs = ROWS * nout;
    for (int base = wave * UPW; base < njobs; base += NW * UPW) {
      const int j = base + unit;
      const int r = j / nout;
      const int o = j - r * nout + skip;
      if (j < njobs && row0 + r < a.rows) {
        const int sl = deriv ? o : (o == 0 ? 0 : o + 1);
        c2<T>* ar = rb + (r * SL + sl) * SC;
        c2<T> v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = ar[pad(t + TEAM * m)];
        team_sync<true>();
        team_fft<T, NH, E, false, 1, true>(v, t, ar, tws);
        team_sync<true>();
#pragma unroll
        for (int m = 0; m < E; ++m) ar[pad(t + TEAM * m)] = v[m];
        team_sync<true>();
        c2<T>* dst = a.b_out + o * a.fs_spec + (long long)(row0 + r) * a.Sx;
        c2<T>* dstn = a.b_out + o * a.fs_spec + a.nyo + (row0 + r);
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int k = t + TEAM * m;
          const c2<T> Z = v[m];
          const c2<T> Zc = conj<T>(ar[pad((NH - k) & (NH - 1))]);
          const c2<T> sm = add<T>(Z, Zc);
          const c2<T> d = sub<T>(Z, Zc);
          const c2<T> B2 = mk<T>(d.y, -d.x);
          const c2<T> WB = cmul<T>(B2, lt.w[m]);
          dst[k] = mk<T>(T(0.5) * (sm.x + WB.x), T(0.5) * (sm.y + WB.y));
          if (k == 0) *dstn = mk<T>(T(0.5) * (sm.x - B2.x), T(0.5) * (sm.y - B2.y));
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint row pass.  Input: the x-spectra s_in of (e_c, b_c, e_1..e_p),
// already transformed back along the strided axes, where
//   e_c = (I - S_c) lambda_c,  b_c = Q_c lambda_c,  e_i = (I - S_eta) lambda_i
// (the column pass forms e from k-space as x/(1+x) lambda^ with
// x = dt M kappa_c |xi|^4 or dt L kappa_eta |xi|^2, so a smooth lambda does
// not lose its digits to the subtraction lambda - S lambda).  Per point:
//   a = lambda^(n+1) - e,  v = (dt M b_c, dt L a_1, ..., dt L a_p)
//   lambda^n = (a_c, a_1, ..., a_p) - H_f(u^n) v
// stored over lambda^(n+1) in `lam`; the double dot products of the
// parameter gradients
//   q0 = <b_c, df/dc(u^n)>,  q1 = <e_c, c^(n+1) - mean(c)>,
//   q2 = sum_i <a_i, df/deta_i(u^n)>,  q3 = sum_i <e_i, eta_i^(n+1)>
// go to partials[block][4] (e_c has zero mean, so removing the held mean of
// c changes nothing in exact arithmetic and keeps the sum well conditioned);
// optionally lambda^n is R2C-transformed (the first transform of the next
// adjoint step) into b_out.
template <typename T>
struct AdjArgs {
  const c2<T>* s_in;
  const T* u_n;
  const T* u_np1;
  T* lam;
  c2<T>* b_out;
  const double2* twx;
  const double* mean_c;
  double* partials;
  long long fs_real, fs_spec;
  long long nyo;  // offset of the Nyquist values within an x-spectrum field
  int rows, Sx, F, do_fwd;
  FeParams<T> fe;
  T dtM, dtL;
};

template <typename T, int NX, int PMAX>
struct AGeom {
  static constexpr int NH = NX / 2;
  static constexpr int E = NH < 4 ? NH : 4;
  static constexpr int TEAM = NH / E;
  static constexpr int ROWS = TEAM >= 64 ? 1 : 64 / TEAM;
  static constexpr int WG = ROWS * TEAM;
  static constexpr int REGION = lds_span(NH) + 1;
};

// FIXF: F = PMAX + 1 at compile time.
template <typename T, int NX, int PMAX, bool FIXF = false>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, AGeom<T, NX, PMAX>::WG)))
adj_row_kernel(AdjArgs<T> a) {
  using G = AGeom<T, NX, PMAX>;
  constexpr int E = G::E, TEAM = G::TEAM, ROWS = G::ROWS;
  constexpr int FB = PMAX + 1;
  __shared__ c2<T> lds[ROWS * G::REGION];
  __shared__ double red[4 * (G::WG / 64 + 1)];
  const int lane = threadIdx.x;
  const int team = lane / TEAM;
  const int t = lane - team * TEAM;
  const int row = blockIdx.x * ROWS + team;
  const bool active = row < a.rows;
  const long long rrow = active ? row : 0;
  c2<T>* my = lds + team * G::REGION;
  const int F = FIXF ? PMAX + 1 : a.F;
  const int p = F - 1;
  Twiddles<T, G::NH, E> tws;
  tws.load(t, a.twx, 2);
  LaneTwiddles<T, G::NH, E> lt;  // exp(-2 pi i k / NX), k = t + TEAM m
  lt.load(t, a.twx);

  // w[0] = e_c, w[1..p] = e_i, bc = b_c; w is overwritten by lambda^n
  c2<T> w[FB][E], bc[E], xn[FB + 1];
  row_load<T, NX, E>(w[0], xn[0], a.s_in + rrow * a.Sx, a.s_in + a.nyo + rrow, active, t);
  row_load<T, NX, E>(bc, xn[FB], a.s_in + a.fs_spec + rrow * a.Sx, a.s_in + a.fs_spec + a.nyo + rrow,
                     active, t);
#pragma unroll
  for (int i = 0; i < PMAX; ++i)
    if (i < p)
      row_load<T, NX, E>(w[1 + i], xn[1 + i], a.s_in + (2 + i) * a.fs_spec + rrow * a.Sx,
                         a.s_in + (2 + i) * a.fs_spec + a.nyo + rrow, active, t);
  row_c2r<T, NX, E>(w[0], xn[0], t, my, lt, tws);
  row_c2r<T, NX, E>(bc, xn[FB], t, my, lt, tws);
#pragma unroll
  for (int i = 0; i < PMAX; ++i)
    if (i < p) row_c2r<T, NX, E>(w[1 + i], xn[1 + i], t, my, lt, tws);

  double q[4] = {0.0, 0.0, 0.0, 0.0};
  const double cmean = *a.mean_c;
  if (active) {
    const long long off = rrow * NX;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int idx = 2 * (t + TEAM * m);
      c2<T> un[FB], un1[FB], lm[FB];
#pragma unroll
      for (int f = 0; f < FB; ++f)
        if (f < F) {
          un[f] = *reinterpret_cast<const c2<T>*>(a.u_n + f * a.fs_real + off + idx);
          un1[f] = *reinterpret_cast<const c2<T>*>(a.u_np1 + f * a.fs_real + off + idx);
          lm[f] = *reinterpret_cast<const c2<T>*>(a.lam + f * a.fs_real + off + idx);
        }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        T eta[PMAX], ge[PMAX], ve[PMAX], oe[PMAX], ai[PMAX];
#pragma unroll
        for (int i = 0; i < PMAX; ++i) {
          eta[i] = (i < p) ? (h ? un[1 + i].y : un[1 + i].x) : T(0);
          const T li = (i < p) ? (h ? lm[1 + i].y : lm[1 + i].x) : T(0);
          const T ei = (i < p) ? (h ? w[1 + i][m].y : w[1 + i][m].x) : T(0);
          ai[i] = li - ei;
          ve[i] = a.dtL * ai[i];
          ge[i] = T(0);
          oe[i] = T(0);
        }
        const T c = h ? un[0].y : un[0].x;
        const T ec = h ? w[0][m].y : w[0][m].x;
        const T lc = h ? lm[0].y : lm[0].x;
        const T ac = lc - ec;
        const T b = h ? bc[m].y : bc[m].x;
        T gc, oc;
        fe_grad<T, PMAX>(a.fe, p, c, eta, gc, ge);
        fe_hvp<T, PMAX>(a.fe, p, c, eta, a.dtM * b, ve, oc, oe);
        const T cn1 = h ? un1[0].y : un1[0].x;
        q[0] += double(b) * double(gc);
        q[1] += double(ec) * (double(cn1) - cmean);
        const T nc = ac - oc;
        if (h) w[0][m].y = nc; else w[0][m].x = nc;
#pragma unroll
        for (int i = 0; i < PMAX; ++i)
          if (i < p) {
            const T ei = h ? w[1 + i][m].y : w[1 + i][m].x;
            const T en1 = h ? un1[1 + i].y : un1[1 + i].x;
            q[2] += double(ai[i]) * double(ge[i]);
            q[3] += double(ei) * double(en1);
            const T ni = ai[i] - oe[i];
            if (h) w[1 + i][m].y = ni; else w[1 + i][m].x = ni;
          }
      }
#pragma unroll
      for (int f = 0; f < FB; ++f)
        if (f < F) *reinterpret_cast<c2<T>*>(a.lam + f * a.fs_real + off + idx) = w[f][m];
    }
  }
  block_sum<4>(q, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) a.partials[4 * blockIdx.x + k] = q[k];
  }
  if (a.do_fwd) {
#pragma unroll
    for (int f = 0; f < FB; ++f)
      if (f < F)
        row_r2c<T, NX, E>(w[f], a.b_out + f * a.fs_spec + rrow * a.Sx, a.b_out + f * a.fs_spec + a.nyo + rrow,
                          active, t, my, lt, tws);
  }
}

// Adjoint row pass, one wavefront per transform (the forward row pass's
// structure and geometry).  Slots: 0 = e_c, 1 = b_c, 2 + i = e_i; the
// pointwise phase overwrites slots 0 and 2 + i with lambda^n for the
// forward transforms of phase 3.
// FIXF: F = PMAX + 1 at compile time.
template <typename T, int NX, int PMAX, bool FIXF = false>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, RGeom<T, NX, PMAX>::WG)))
adjrow_kernel(AdjArgs<T> a) {
  using G = RGeom<T, NX, PMAX>;
  constexpr int NH = G::NH, E = G::E, TEAM = G::TEAM, UPW = G::UPW, ROWS = G::ROWS;
  constexpr int NW = G::NW, SL = G::SLOTS, WG = G::WG, SC = G::SLOT_C;
  static_assert(G::FITS, "adjoint row pass v2 does not fit this size");
  __shared__ __align__(16) c2<T> rb[ROWS * SL * SC];
  __shared__ double red[4 * (NW + 1)];
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int unit = lane / TEAM;
  const int t = lane - unit * TEAM;
  const int row0 = blockIdx.x * ROWS;
  const int F = FIXF ? PMAX + 1 : a.F;
  const int p = F - 1;
  Twiddles<T, NH, E> tws;
  tws.load(t, a.twx, 2);
  LaneTwiddles<T, NH, E> lt;
  lt.load(t, a.twx);

  // phase 1: C2R of the F + 1 adjoint x-spectra into slots 0..F
  {
    const int nin = F + 1;
    const int njobs = ROWS * nin;
    for (int base = wave * UPW; base < njobs; base += NW * UPW) {
      const int j = base + unit;
      const int r = j / nin;
      const int sl = j - r * nin;
      if (j < njobs && row0 + r < a.rows) {
        const c2<T>* src = a.s_in + sl * a.fs_spec + (long long)(row0 + r) * a.Sx;
        const c2<T>* nyq = a.s_in + sl * a.fs_spec + a.nyo + (row0 + r);
        c2<T>* ar = rb + (r * SL + sl) * SC;
        c2<T> v[E];
        wave_c2r_pre<T, NH, E>(v, src, nyq, ar, t, lt);
        team_fft<T, NH, E, true, 1, true>(v, t, ar, tws);
        team_sync<true>();
#pragma unroll
        for (int m = 0; m < E; ++m) ar[pad(t + TEAM * m)] = v[m];
      }
    }
  }
  __syncthreads();

  // phase 2: Hessian-vector product, new lambda, parameter-gradient dots
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  const double cmean = *a.mean_c;
  const int npairs = ROWS * NH;
  for (int qi = tid; qi < npairs; qi += WG) {
    const int r = qi / NH;
    const int x2 = qi - r * NH;
    const int row = row0 + r;
    if (row < a.rows) {
      c2<T>* pt = rb + r * SL * SC + pad(x2);
      const long long off = (long long)row * NH + x2;
      c2<T> un[PMAX + 1], un1[PMAX + 1], lm[PMAX + 1];
#pragma unroll
      for (int f = 0; f < PMAX + 1; ++f)
        if (f < F) {
          un[f] = reinterpret_cast<const c2<T>*>(a.u_n + f * a.fs_real)[off];
          un1[f] = reinterpret_cast<const c2<T>*>(a.u_np1 + f * a.fs_real)[off];
          lm[f] = reinterpret_cast<const c2<T>*>(a.lam + f * a.fs_real)[off];
        }
      const c2<T> ecv = pt[0];
      const c2<T> bcv = pt[SC];
      c2<T> ev[PMAX];
#pragma unroll
      for (int i = 0; i < PMAX; ++i) ev[i] = (i < p) ? pt[(2 + i) * SC] : mk<T>(T(0), T(0));
      c2<T> nl[PMAX + 1];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        T eta[PMAX], ge[PMAX], ve[PMAX], oe[PMAX], ai[PMAX];
#pragma unroll
        for (int i = 0; i < PMAX; ++i) {
          eta[i] = (i < p) ? (h ? un[1 + i].y : un[1 + i].x) : T(0);
          const T li = (i < p) ? (h ? lm[1 + i].y : lm[1 + i].x) : T(0);
          const T ei = (i < p) ? (h ? ev[i].y : ev[i].x) : T(0);
          ai[i] = li - ei;
          ve[i] = a.dtL * ai[i];
          ge[i] = T(0);
          oe[i] = T(0);
        }
        const T c = h ? un[0].y : un[0].x;
        const T ec = h ? ecv.y : ecv.x;
        const T lc = h ? lm[0].y : lm[0].x;
        const T ac = lc - ec;
        const T b = h ? bcv.y : bcv.x;
        T gc, oc;
        fe_grad<T, PMAX>(a.fe, p, c, eta, gc, ge);
        fe_hvp<T, PMAX>(a.fe, p, c, eta, a.dtM * b, ve, oc, oe);
        const T cn1 = h ? un1[0].y : un1[0].x;
        q[0] += double(b) * double(gc);
        q[1] += double(ec) * (double(cn1) - cmean);
        const T nc = ac - oc;
        if (h) nl[0].y = nc; else nl[0].x = nc;
#pragma unroll
        for (int i = 0; i < PMAX; ++i)
          if (i < p) {
            const T ei = h ? ev[i].y : ev[i].x;
            const T en1 = h ? un1[1 + i].y : un1[1 + i].x;
            q[2] += double(ai[i]) * double(ge[i]);
            q[3] += double(ei) * double(en1);
            const T ni = ai[i] - oe[i];
            if (h) nl[1 + i].y = ni; else nl[1 + i].x = ni;
          }
      }
      pt[0] = nl[0];
      reinterpret_cast<c2<T>*>(a.lam)[off] = nl[0];
#pragma unroll
      for (int i = 0; i < PMAX; ++i)
        if (i < p) {
          pt[(2 + i) * SC] = nl[1 + i];
          reinterpret_cast<c2<T>*>(a.lam + (1 + i) * a.fs_real)[off] = nl[1 + i];
        }
    }
  }
  block_sum<4>(q, red);
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) a.partials[4 * blockIdx.x + k] = q[k];
  }
  __syncthreads();

  // phase 3: R2C of lambda^n (slots 0 and 2 + i) for the next adjoint step
  if (a.do_fwd) {
    const int njobs = ROWS * F;
    for (int base = wave * UPW; base < njobs; base += NW * UPW) {
      const int j = base + unit;
      const int r = j / F;
      const int f = j - r * F;
      if (j < njobs && row0 + r < a.rows) {
        c2<T>* ar = rb + (r * SL + (f == 0 ? 0 : f + 1)) * SC;
        c2<T> v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = ar[pad(t + TEAM * m)];
        team_sync<true>();
        team_fft<T, NH, E, false, 1, true>(v, t, ar, tws);
        team_sync<true>();
#pragma unroll
        for (int m = 0; m < E; ++m) ar[pad(t + TEAM * m)] = v[m];
        team_sync<true>();
        c2<T>* dst = a.b_out + f * a.fs_spec + (long long)(row0 + r) * a.Sx;
        c2<T>* dstn = a.b_out + f * a.fs_spec + a.nyo + (row0 + r);
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int k = t + TEAM * m;
          const c2<T> Z = v[m];
          const c2<T> Zc = conj<T>(ar[pad((NH - k) & (NH - 1))]);
          const c2<T> sm = add<T>(Z, Zc);
          const c2<T> d = sub<T>(Z, Zc);
          const c2<T> B2 = mk<T>(d.y, -d.x);
          const c2<T> WB = cmul<T>(B2, lt.w[m]);
          dst[k] = mk<T>(T(0.5) * (sm.x + WB.x), T(0.5) * (sm.y + WB.y));
          if (k == 0) *dstn = mk<T>(T(0.5) * (sm.x - B2.x), T(0.5) * (sm.y - B2.y));
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Column pass.

enum { COL_FWD = 0, COL_INV = 1, COL_UPDATE = 2, COL_ADJ = 3, COL_ENERGY = 4,
       COL_UPDATE_FIRST = 5 /* launch-time only: COL_UPDATE with first = 1 */ };

template <typename T>
struct ColArgs {
  const c2<T>* src;
  c2<T>* dst;
  const double2* tw;   // exp(-2 pi i q / N) for the transformed axis, double
  const T* kcol;       // |xi|^2 table indexed by the column (x frequency)
  const T* kaxis;      // |xi|^2 table of the transformed axis
  const T* kouter;     // |xi|^2 table indexed by the outer index (3D z pass), or null
  double* mean_c;        // double mean of c (held k = 0 mode); written by the first update
  c2<T>* cstate;         // carried spectrum of c (update mode), x-spectrum layout
  double* partials;
  long long fs_src, fs_dst;  // field strides (complex elements)
  long long ls;              // stride between consecutive transform elements
  long long os;              // stride between outer planes
  long long nyo;             // offset of the Nyquist values within a field
  long long nls, nos;        // Nyquist values: element stride, outer-row stride
  int ncols;                 // regular columns (Nx/2: kx = 0 .. Nx/2 - 1)
  int nyq;                   // Nx/2, the Nyquist column (Hermitian weight 1 at columns 0 and nyq)
  int F, mode;
  int first;  // update mode: take c^ from src field 0 (and transform it) instead of cstate
  int nrec;   // first update: row-pass records {sum f, sum c} in partials to take the mean of c from
  int f0;     // forward/inverse modes: first field transformed
  T dtM, dtMkc, dtL, dtLke, invP;
  double invPd;  // 1 / P in double
};

// Column-pass geometry.  E elements per lane (8; N when N <= 8; for float
// axes of 512 points or more, PF_COL_E_LONG_F32), N / E lanes per column,
// C consecutive columns per work-group: a few columns on the long axes
// (N >= 512) so that a 2D grid yields several work-groups per compute unit,
// 128-byte row segments otherwise; at least one wavefront and at most 512
// lanes per group (PF_COL_WG_MAX_LONG for 4096-point float axes).
template <typename T, int N>
struct ColGeom {
  static constexpr int E = N <= 8 ? N : ((N >= 512 && sizeof(T) == 4) ? PF_COL_E_LONG_F32 : 8);
  static constexpr int TEAM = N / E;
  static constexpr int CB = N >= 512 ? (sizeof(T) == 8 ? PF_COL_CB_LONG_F64 : PF_COL_CB_LONG_F32)
                                    : (sizeof(T) == 8 ? 8 : 16);
  static constexpr int C0 = (CB * TEAM < 64) ? 64 / TEAM : CB;
  static constexpr int WGMAX = (sizeof(T) == 4 && N >= 4096) ? PF_COL_WG_MAX_LONG : 512;
  static constexpr int C = (C0 * TEAM > WGMAX) ? (WGMAX / TEAM > 0 ? WGMAX / TEAM : 1) : C0;
  static constexpr int WG = C * TEAM;
  static constexpr int MIN_WAVES = sizeof(T) == 4 ? PF_COL_MIN_WAVES : 1;
};

// Work order of the column pass (see col_kernel), the faster choice for
// each case on MI355X: 0 = field group fastest over a contiguous run of
// items per XCD (2D double of length below PF_COL_ORDER1_F64_MIN),
// 1 = per-XCD chunks of tiles (2D float; 2D double of longer columns, whose
// narrow tiles share cache lines that the chunk order keeps in one L2 while
// they are used), 2 = outer rows dealt to the XCDs round-robin (3D passes).
#ifndef PF_COL_ORDER3D
#define PF_COL_ORDER3D 2
#endif
#ifndef PF_COL_ORDER1_F64_MIN
#define PF_COL_ORDER1_F64_MIN 4096
#endif
template <typename T, int N>
__host__ __device__ inline int col_order(int nouter) {
  return nouter > 1 ? PF_COL_ORDER3D : (sizeof(T) == 4 || N >= PF_COL_ORDER1_F64_MIN) ? 1 : 0;
}

// One work-group per (column tile, outer index, field group), plus, ahead of
// them, one per (block of C outer indices, field group) for the Nyquist
// column, whose values sit apart from the tiles (see the layout above); a
// Nyquist item's C lane columns are C outer rows.  Field groups:
// forward/inverse: one per field; update and adjoint: the c group (which
// needs c^ and g^ together) and one per eta_i; energy: one per field.
// Blocks are dealt to the eight XCDs round-robin (block b runs on XCD b % 8),
// so the logical work index is chosen to give each XCD the same mix of c
// groups (two arrays in and out) and eta groups (one), with neighbouring
// tiles of a field on one L2 (2D: tiles share cache lines) or the XCDs
// moving through neighbouring rows of each plane together (3D: HBM
// locality); col_order selects the order.
template <typename T, int N, int MODE>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, ColGeom<T, N>::WG),
                               amdgpu_waves_per_eu(ColGeom<T, N>::MIN_WAVES)))
col_kernel(ColArgs<T> a, int tiles, int nouter, int ngroups, int nslots, int nqb) {
  using G = ColGeom<T, N>;
  constexpr int E = G::E, TEAM = G::TEAM, C = G::C;
  int L, g, tile, o;
  const int order = col_order<T, N>(nouter);
  // blocks [0, nqb): Nyquist items, C outer rows of the Nyquist column each
  // (nqb is a multiple of 8, so the XCD of a regular block is unchanged)
  const int nqi = (nouter + C - 1) / C;  // Nyquist items per field group
  if (int(blockIdx.x) < nqb) {
    const int j = blockIdx.x;
    if (j >= nqi * ngroups) return;
    g = j / nqi;
    o = (j - g * nqi) * C;  // first outer row
    tile = -1;
    L = tiles * nouter * ngroups + j;
  } else if (order == 2) {
    // outer row o on XCD o % 8, rows of one XCD in increasing order, field
    // group by group: at any time the XCDs stream through neighbouring rows
    // of each plane (one contiguous region per plane rather than eight)
    const int b = int(blockIdx.x) - nqb;
    const int nu = tiles * nouter;
    const int rpx = (nouter + 7) / 8;
    const int j = b >> 3;
    g = j / nslots;
    const int jj = j - g * nslots;
    const int r = jj / tiles;
    tile = jj - r * tiles;
    o = r * 8 + (b & 7);
    if (g >= ngroups || o >= nouter || r >= rpx) return;
    L = g * nu + o * tiles + tile;  // dense record index
  } else if (order == 1) {
    // units u = (outer, tile), tile fastest, cut into eight contiguous
    // chunks of `nslots` units; XCD x takes chunk x for every field group,
    // group by group, so neighbouring tiles of one field run back to back on
    // one L2 and every XCD gets the same mix of c and eta groups.
    const int b = int(blockIdx.x) - nqb;
    const int nu = tiles * nouter;
    const int j = b >> 3;
    g = j / nslots;
    const int u = (b & 7) * nslots + (j - g * nslots);
    if (g >= ngroups || u >= nu) return;
    L = g * nu + u;  // dense record index
    tile = u % tiles;
    o = u / tiles;
  } else {
    // field group fastest over a contiguous run of work items per XCD
    const int b = int(blockIdx.x) - nqb;
    L = (b & 7) * nslots + (b >> 3);
    if (L >= tiles * nouter * ngroups) return;
    g = L % ngroups;
    const int rest = L / ngroups;
    tile = rest % tiles;
    o = rest / tiles;
  }
  __shared__ c2<T> lds[(PF_COL_PINGPONG ? 2 : 1) * lds_span(N) * C];
  __shared__ double red[2 * (G::WG / 64 + 1)];
  const int lane = threadIdx.x;
  const int cc = lane % C;
  const int t = lane / C;
  const bool nyqi = tile < 0;  // work-group uniform
  // a Nyquist item's lanes cc are C consecutive outer rows of column nyq
  const int col = nyqi ? a.nyq : tile * C + cc;
  const int orow = nyqi ? o + cc : o;
  const bool active = nyqi ? orow < nouter : col < a.ncols;
  c2<T>* my = lds + cc;
  c2<T>* my2 = PF_COL_PINGPONG ? lds + lds_span(N) * C + cc : nullptr;
  int par = 0;  // exchange parity across the transforms of this work-group

  // Element t + TEAM m of this lane's column sits at a work-group-uniform
  // 64-bit base (field, outer plane, tile, m) plus a 32-bit per-lane byte
  // offset that is the same for every m, so the address arithmetic runs on
  // the scalar unit.  The offset is below 2^32 for every supported shape
  // (at most C + TEAM ls complex values).
  const long long ls = nyqi ? a.nls : a.ls;
  const long long wg0 = nyqi ? a.nyo + (long long)o * a.nos : (long long)o * a.os + (long long)tile * C;
  const unsigned lbo = (unsigned(cc) * unsigned(nyqi ? a.nos : 1) + unsigned(t) * unsigned(ls)) *
                       unsigned(sizeof(c2<T>));
  auto load = [&](const c2<T>* src, c2<T>* v) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const char* pm = reinterpret_cast<const char*>(src + wg0 + (long long)m * TEAM * ls);
      v[m] = active ? *reinterpret_cast<const c2<T>*>(pm + lbo) : mk<T>(T(0), T(0));
    }
  };
  auto store = [&](c2<T>* dst, const c2<T>* v) {
    if (active) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        char* pm = reinterpret_cast<char*>(dst + wg0 + (long long)m * TEAM * ls);
        *reinterpret_cast<c2<T>*>(pm + lbo) = v[m];
      }
    }
  };
  const T kc = a.kcol[active ? col : 0] + (a.kouter ? a.kouter[active ? orow : 0] : T(0));
  Twiddles<T, N, E> tws;
  tws.load(t, a.tw, 1);
  // the axis part of |xi|^2 of this lane's elements; the steady update reads
  // it before the transforms (a work-group barrier keeps later reads from
  // moving up), the others where it is used
  constexpr bool KPRE = MODE == COL_UPDATE;
  T kax[E];
  if constexpr (KPRE) {
#pragma unroll
    for (int m = 0; m < E; ++m) kax[m] = a.kaxis[t + TEAM * m];
  }
  auto kaxis = [&](int m) -> T { return KPRE ? kax[m] : a.kaxis[t + TEAM * m]; };

  c2<T> v[E];
  if constexpr (MODE == COL_FWD || MODE == COL_INV) {
    load(a.src + (g + a.f0) * a.fs_src, v);
    if constexpr (MODE == COL_FWD) par = team_fft<T, N, E, false, C>(v, t, my, tws, my2, par);
    else par = team_fft<T, N, E, true, C>(v, t, my, tws, my2, par);
    store(a.dst + (g + a.f0) * a.fs_dst, v);
  } else if constexpr (MODE == COL_UPDATE || MODE == COL_UPDATE_FIRST) {
    if (g == 0) {
      // c (carried spectrum, Algorithm 1): c^ <- (c^ - dt M k2 g^) / (1 + dt M kappa_c k2^2);
      // the inverse transform gets c^ / P with the k = 0 mode held in double.
      // Both column arrays are loaded up front so their latencies overlap.
      c2<T> gg[E];
      load(a.src + a.fs_src, gg);
      if constexpr (MODE == COL_UPDATE_FIRST) {
        load(a.src, v);
      } else {
        load(a.cstate, v);
      }
      par = team_fft<T, N, E, false, C>(gg, t, my, tws, my2, par);
      if constexpr (MODE == COL_UPDATE_FIRST) par = team_fft<T, N, E, false, C>(v, t, my, tws, my2, par);
      // the held k = 0 mode: P times the double-precision mean of c.  On the
      // first step of a call the work item that holds it (tile 0, outer row
      // 0) adds up the row pass's per-group sums of c in a fixed order and
      // keeps the mean for the later steps; the row pass has completed (a
      // kernel boundary), so no fence is needed.
      double cmean = 0.0;
      if constexpr (MODE == COL_UPDATE_FIRST) {
        if (tile == 0 && o == 0) {  // work-group uniform
          double acc[1] = {0.0};
          for (int r = threadIdx.x; r < a.nrec; r += blockDim.x) acc[0] += a.partials[2 * (long long)r + 1];
          block_sum<1>(acc, red);
          if (threadIdx.x == 0) {
            cmean = acc[0] * a.invPd;
            *a.mean_c = cmean;
          }
        }
      } else {
        if (col == 0 && o == 0 && t == 0) cmean = *a.mean_c;
      }
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const T k2 = kc + kaxis(m);
        const T D = recip<T>(T(1) + a.dtMkc * k2 * k2);
        const T sk = a.dtM * k2;
        v[m] = mk<T>((v[m].x - sk * gg[m].x) * D, (v[m].y - sk * gg[m].y) * D);
      }
      store(a.cstate, v);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int e = t + TEAM * m;
        v[m] = mk<T>(v[m].x * a.invP, v[m].y * a.invP);
        if (col == 0 && o == 0 && e == 0) v[m] = mk<T>(T(cmean), T(0));
      }
      par = team_fft<T, N, E, true, C>(v, t, my, tws, my2, par);
      store(a.dst, v);
    } else {
      // eta_g: b^ / (1 + dt L kappa_eta k2)
      load(a.src + (g + 1) * a.fs_src, v);
      par = team_fft<T, N, E, false, C>(v, t, my, tws, my2, par);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const T k2 = kc + kaxis(m);
        const T D = a.invP * recip<T>(T(1) + a.dtLke * k2);
        v[m] = mk<T>(v[m].x * D, v[m].y * D);
      }
      par = team_fft<T, N, E, true, C>(v, t, my, tws, my2, par);
      store(a.dst + g * a.fs_dst, v);
    }
  } else if constexpr (MODE == COL_ADJ) {
    if (g == 0) {
      // e_c = x/(1+x) lambda_c^ (x = dt M kappa_c k2^2), b_c = D_c k2 lambda_c^
      c2<T> bb[E];
      load(a.src, v);
      par = team_fft<T, N, E, false, C>(v, t, my, tws, my2, par);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const T k2 = kc + kaxis(m);
        const T x = a.dtMkc * k2 * k2;
        const T D = a.invP * recip<T>(T(1) + x);
        bb[m] = mk<T>(v[m].x * D * k2, v[m].y * D * k2);
        v[m] = mk<T>(v[m].x * D * x, v[m].y * D * x);
      }
      par = team_fft<T, N, E, true, C>(v, t, my, tws, my2, par);
      store(a.dst, v);
      par = team_fft<T, N, E, true, C>(bb, t, my, tws, my2, par);
      store(a.dst + a.fs_dst, bb);
    } else {
      // e_g = y/(1+y) lambda_g^ (y = dt L kappa_eta k2)
      load(a.src + g * a.fs_src, v);
      par = team_fft<T, N, E, false, C>(v, t, my, tws, my2, par);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const T k2 = kc + kaxis(m);
        const T y = a.dtLke * k2;
        const T D = a.invP * y * recip<T>(T(1) + y);
        v[m] = mk<T>(v[m].x * D, v[m].y * D);
      }
      par = team_fft<T, N, E, true, C>(v, t, my, tws, my2, par);
      store(a.dst + (g + 1) * a.fs_dst, v);
    }
  } else {  // COL_ENERGY: sum of w_kx k2 |u^|^2 of field g
    static_assert(MODE == COL_ENERGY, "unknown column mode");
    double acc[2] = {0.0, 0.0};
    const double wcol = (col == 0 || col == a.nyq) ? 1.0 : 2.0;
    load(a.src + g * a.fs_src, v);
    par = team_fft<T, N, E, false, C>(v, t, my, tws, my2, par);
    if (active) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const double k2 = double(kc) + double(kaxis(m));
        const double re = double(v[m].x), im = double(v[m].y);
        acc[g == 0 ? 0 : 1] += wcol * k2 * (re * re + im * im);
      }
    }
    block_sum<2>(acc, red);
    if (threadIdx.x == 0) {
      a.partials[2 * (long long)L + 0] = acc[0];
      a.partials[2 * (long long)L + 1] = acc[1];
    }
  }
}

// Explicit FD step and FD energy (k_fd.hip).
template <typename T>
struct FdArgs {
  const T* in;
  T* out;
  T* mu;
  double* partials;
  long long P;  // points per field
  int nx, ny, nz, lx, ly, ndim, F;
  T ix2, iy2, iz2;  // 1 / dx_d^2
  T dtM, kc, dtL, ke;
  double ix, iy, iz;  // 1 / dx_d
  FeParams<T> fe;
};

// Single work-group fixed-order sum of `n` records of `width` doubles:
// out[i] = scale[i] * sum_r partials[r * width + i]  (added to out[i] when
// `accumulate` is set).
__global__ void __launch_bounds__(256) reduce_kernel(const double* __restrict__ partials, int n,
                                                     int width, double* __restrict__ out,
                                                     double s0, double s1, double s2, double s3,
                                                     int accumulate);

}  // namespace pf
