// Device-side FFT building blocks for gfx950.
//
// A length-N complex transform is executed by a "team" of N/E lanes, each
// lane holding E elements in registers.  Lane t of a team always holds
// element t + TEAM*m in register m, both on entry (time order) and on exit
// (frequency order), so the first pass reads straight from registers loaded
// with coalesced global loads and the last pass leaves the result in
// registers ready for coalesced stores.
//
// The transform is a mixed-radix Stockham autosort FFT: for a pass of radix
// R after NS points have been combined, butterfly j (0 <= j < N/R) reads
// x[j + r N/R], multiplies input r by exp(-+2 pi i r k / (NS R)) with
// k = j mod NS, applies an R-point DFT and writes y[(j - k) R + k + r NS].
// Between passes the data goes through LDS; the last pass writes its
// outputs back to the same registers it read (its output index equals its
// input index), so an N = E^P transform needs P - 1 LDS exchanges.
//
// Twiddles come from a per-axis double-precision table
// W[q] = exp(-2 pi i q / Naxis) that the host computes in extended precision;
// a length-N transform on an axis of length Naxis reads W[q * (Naxis / N)].
// Each lane reads one table entry per pass and forms the other powers it
// needs by double-precision complex multiplication, rounding once to the
// working precision, so a kernel issues a handful of table loads per lane
// and none sits in the dependency chain of a pass.
#pragma once

#include <hip/hip_runtime.h>

namespace pf {

template <typename T> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };
template <typename T> using c2 = typename vec2<T>::type;

template <typename T>
__device__ __forceinline__ c2<T> mk(T x, T y) {
  c2<T> r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename T>
__device__ __forceinline__ c2<T> add(c2<T> a, c2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ c2<T> sub(c2<T> a, c2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ c2<T> cmul(c2<T> a, c2<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ c2<T> cmulc(c2<T> a, c2<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ c2<T> conj(c2<T> a) { return mk<T>(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ c2<T> scale(c2<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  double2 r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename T>
__device__ __forceinline__ c2<T> rnd(double2 a) { return mk<T>(T(a.x), T(a.y)); }

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// LDS position of exchange element i: one padding slot after every eight
// elements.  The Stockham writes of a pass land at strides of 8 R or 64
// elements across lanes, which without padding fall into the same LDS banks;
// with it they spread over all banks.  An exchange area of N elements
// occupies lds_span(N) slots.
__device__ __forceinline__ constexpr int pad(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int lds_span(int n) { return n + (n >> 3) + 1; }

// Multiply by exp(-2 pi i K / R) (forward) or exp(+2 pi i K / R) (inverse)
// for R <= 16, 0 <= K < R/2.  Exact sixteenth roots of unity: cos(pi/8),
// sin(pi/8) and sqrt(1/2) to 23 digits.
template <int R, int K, bool INV, typename T>
__device__ __forceinline__ c2<T> rot(c2<T> a) {
  constexpr int k16 = K * (16 / R);
  constexpr double C1 = 0.92387953251128675612818;  // cos(pi/8)
  constexpr double S1 = 0.38268343236508977172846;  // sin(pi/8)
  constexpr double R2 = 0.70710678118654752440084;  // sqrt(1/2)
  if constexpr (k16 == 0) {
    return a;
  } else if constexpr (k16 == 4) {
    // forward: * (-i); inverse: * (+i)
    return INV ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
  } else {
    constexpr double cs = (k16 == 1) ? C1 : (k16 == 2) ? R2 : (k16 == 3) ? S1
                        : (k16 == 5) ? -S1 : (k16 == 6) ? -R2 : -C1;
    constexpr double sn = (k16 == 1) ? S1 : (k16 == 2) ? R2 : (k16 == 3) ? C1
                        : (k16 == 5) ? C1 : (k16 == 6) ? R2 : S1;
    // w = cs - i sn (forward) or cs + i sn (inverse)
    const T c = T(cs);
    const T s = INV ? T(sn) : T(-sn);
    return mk<T>(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// R-point DFT in registers, natural order in and out (radix-2 decimation in
// time, unrolled at compile time).
template <typename T, int R, bool INV>
struct Dft;

template <typename T, bool INV>
struct Dft<T, 1, INV> {
  __device__ __forceinline__ static void run(c2<T>*) {}
};

template <int K, int R, bool INV, typename T>
struct Combine {
  __device__ __forceinline__ static void run(c2<T>* x, const c2<T>* e, const c2<T>* o) {
    Combine<K - 1, R, INV, T>::run(x, e, o);
    const c2<T> t = rot<R, K - 1, INV, T>(o[K - 1]);
    x[K - 1] = add<T>(e[K - 1], t);
    x[K - 1 + R / 2] = sub<T>(e[K - 1], t);
  }
};
template <int R, bool INV, typename T>
struct Combine<0, R, INV, T> {
  __device__ __forceinline__ static void run(c2<T>*, const c2<T>*, const c2<T>*) {}
};

template <typename T, int R, bool INV>
struct Dft {
  __device__ __forceinline__ static void run(c2<T>* x) {
    c2<T> e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    Dft<T, R / 2, INV>::run(e);
    Dft<T, R / 2, INV>::run(o);
    Combine<R / 2, R, INV, T>::run(x, e, o);
  }
};

// Radix of the first pass: the remainder when log2(N) is not a multiple of
// log2(E); every later pass has radix E.
template <int N, int E>
constexpr int first_radix() {
  return (ilog2(N) % ilog2(E)) ? (1 << (ilog2(N) % ilog2(E))) : E;
}

// Number of passes of a length-N transform with E elements per lane: an
// optional first pass of radix first_radix<N, E>() < E, then radix-E passes.
template <int N, int E>
constexpr int num_passes() {
  return ilog2(N) / ilog2(E) + ((ilog2(N) % ilog2(E)) ? 1 : 0);
}

// Per-lane twiddles of one team transform, loaded once and reused by every
// transform of that length the lane performs (the inverse uses their
// conjugates).  Pass p >= 1 has radix E, one butterfly per lane (j = t), and
// needs exp(-2 pi i r k / (NS_p E)) for r = 1..E-1, k = t mod NS_p.
template <typename T, int N, int E>
struct Twiddles {
  static constexpr int P = num_passes<N, E>();
  static constexpr int NT = (P - 1) * (E - 1) > 0 ? (P - 1) * (E - 1) : 1;
  c2<T> w[NT];
  // tw: the axis table in double; tws = Naxis / N
  __device__ __forceinline__ void load(int t, const double2* __restrict__ tw, int tws) {
    int ns = first_radix<N, E>();
#pragma unroll
    for (int p = 1; p < P; ++p) {
      const int k = t & (ns - 1);
      const int step = N / (ns * E);
      const double2 w1 = tw[(k * step) * tws];
      double2 wr = w1;
#pragma unroll
      for (int r = 1; r < E; ++r) {
        w[(p - 1) * (E - 1) + (r - 1)] = rnd<T>(wr);
        wr = dmul(wr, w1);
      }
      ns *= E;
    }
  }
};

// exp(-2 pi i k / N) for the E positions k = t + TEAM m a lane holds, from
// the double table of length N (one per-lane entry and one common step).
template <typename T, int N, int E>
struct LaneTwiddles {
  c2<T> w[E];
  __device__ __forceinline__ void load(int t, const double2* __restrict__ tw) {
    constexpr int TEAM = N / E;
    const double2 step = tw[TEAM];
    double2 cur = tw[t];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      w[m] = rnd<T>(cur);
      cur = dmul(cur, step);
    }
  }
};

// One Stockham pass.  `lds` points at element 0 of this team's exchange
// area; element i lives at lds[pad(i) * LS].  `tw` holds this pass's twiddles
// (radix-E passes after the first only).
template <typename T, int N, int E, int R, int NS, bool INV, bool LAST, int LS>
__device__ __forceinline__ void stockham_pass(c2<T>* v, int t, c2<T>* lds, const c2<T>* tw) {
  constexpr int TEAM = N / E;
  constexpr int BPL = E / R;  // butterflies per lane
#pragma unroll
  for (int b = 0; b < BPL; ++b) {
    const int j = t + TEAM * b;
    const int k = j & (NS - 1);
    c2<T> x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = v[b + r * BPL];
    if constexpr (NS > 1) {
      static_assert(R == E && BPL == 1, "twiddled passes are radix E");
#pragma unroll
      for (int r = 1; r < R; ++r) x[r] = INV ? cmulc<T>(x[r], tw[r - 1]) : cmul<T>(x[r], tw[r - 1]);
    }
    Dft<T, R, INV>::run(x);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b + r * BPL] = x[r];
    } else {
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[pad(base + r * NS) * LS] = x[r];
    }
  }
}

// Exchange synchronisation.  A team that fits in one wavefront only needs
// its own LDS traffic ordered: LDS operations of one wavefront execute in
// issue order, so a compiler fence at wavefront scope (which also keeps the
// compiler from moving one lane's accesses across another lane's) is
// enough.  Larger teams synchronise the whole work-group.
template <bool WAVE>
__device__ __forceinline__ void team_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// Passes of one team transform.  With a second exchange area (`lds2`
// non-null, work-group teams only) consecutive exchanges alternate between
// the two areas, so one barrier per exchange suffices: the next pass writes
// the area nobody is reading.  `par` is the parity of the exchanges already
// made by earlier transforms, so alternation continues across transforms.
template <typename T, int N, int E, bool INV, int NS, int LS, bool WAVE, int PI>
struct FftPasses {
  static constexpr int R = (NS == 1) ? first_radix<N, E>() : E;
  static constexpr bool LAST = (NS * R == N);
  __device__ __forceinline__ static void run(c2<T>* v, int t, c2<T>* lds, c2<T>* lds2,
                                             const c2<T>* twr, int par) {
    c2<T>* area = (lds2 && ((PI + par) & 1)) ? lds2 : lds;
    stockham_pass<T, N, E, R, NS, INV, LAST, LS>(v, t, area, twr + (PI > 0 ? (PI - 1) * (E - 1) : 0));
    if constexpr (!LAST) {
      constexpr int TEAM = N / E;
      team_sync<WAVE>();
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = area[pad(t + TEAM * m) * LS];
      if (!lds2) team_sync<WAVE>();
      FftPasses<T, N, E, INV, NS * R, LS, WAVE, PI + 1>::run(v, t, lds, lds2, twr, par);
    }
  }
};

// Length-N complex FFT by a team; unnormalised in both directions.  `tw`
// holds the lane's twiddles (Twiddles<T, N, E>::load).  With WAVE = false
// every lane of the work-group must call this (it contains work-group
// barriers); with WAVE = true the team must lie within one wavefront and
// only that team's lanes take part.  `lds2`, when given (WAVE = false only),
// is a second exchange area of the same size; `par` is the exchange parity
// returned by the previous transform that used the same two areas (0 for
// the first), and the new parity is returned.  With two areas the caller
// must not touch either area between the transform's return and the next
// work-group barrier of its own (the last exchange may still be read).
template <typename T, int N, int E, bool INV, int LS, bool WAVE = false>
__device__ __forceinline__ int team_fft(c2<T>* v, int t, c2<T>* lds, const Twiddles<T, N, E>& tw,
                                        c2<T>* lds2 = nullptr, int par = 0) {
  static_assert(N >= E && E >= 2 && (N % E) == 0, "bad FFT team shape");
  static_assert(!WAVE || N / E <= 64, "a wave-synchronised team must fit one wavefront");
  FftPasses<T, N, E, INV, 1, LS, WAVE, 0>::run(v, t, lds, lds2, tw.w, par);
  return par + Twiddles<T, N, E>::P - 1;
}

}  // namespace pf
