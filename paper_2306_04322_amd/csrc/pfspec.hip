// libpfspec host runtime: configuration checks, plan tables, workspace
// layout, launch sequencing on the caller's stream, and the C ABI of
// include/pfspec.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pfspec.h"
#include "pf_kernels.h"
#include "pf_launch.h"

using namespace pf;

namespace {

thread_local std::string g_err;

pf_status fail(pf_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

bool is_pow2(long long n) { return n > 0 && (n & (n - 1)) == 0; }
int log2i(long long n) {
  int l = 0;
  while ((1LL << l) < n) ++l;
  return l;
}
size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

enum { PROF_ROW = 0, PROF_COL = 1, PROF_FD = 2, PROF_RED = 3, PROF_ADJ = 4, PROF_NCLS = 5 };

struct ProfRec {
  hipEvent_t a, b;
  int cls;
};

}  // namespace

struct pf_handle {
  pf_config cfg;
  int nd, nx, ny, nz, F, p, nxh, Sx, rows;
  long long nyo;  // offset of the Nyquist values within an x-spectrum field
  long long P;
  size_t es;  // bytes per real element
  double M, kc, L, ke;
  double dV;
  // host tables in double: twiddles (re, im interleaved) and |xi|^2 per axis
  std::vector<double> tw[3], kt[3];
  // workspace layout (byte offsets)
  size_t off_B, off_S, off_C, off_tw[3], off_k[3], off_part, off_scal, ws_need;
  size_t spec_field;  // complex elements per x-spectrum field
  long long nparts;
  std::vector<unsigned char> staging;
  void* fields = nullptr;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  // profiling
  double last_dt = 0.0;  // time step of the last pf_step_fs call
  bool prof_on = false;
  std::vector<ProfRec> prof_pool;
  size_t prof_used = 0;
};

// Device scratch of pf_step_fs_static: the step's workspace (spectra,
// tables, partial sums) for callers that cannot allocate device memory.  One
// copy per GPU, held by the process from the library's load to its exit.
// Host code must not pass `scratch` itself to a kernel or a copy: its host
// name is a stand-in, not a device address.  The device address comes from
// hipGetSymbolAddress, once per device (static_scratch_ptr).
static constexpr size_t kStaticScratchBytes = PF_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

// Device address of `scratch` on the current device, looked up on the first
// call per device and kept.  NULL with a message in g_err on failure.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* static_scratch_ptr(std::string& why) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    why = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    why = "device index out of range";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

int prof_begin(pf_handle* h, int cls) {
  if (!h->prof_on) return -1;
  if (h->prof_used == h->prof_pool.size()) {
    if (h->prof_pool.size() >= 200000) return -1;
    ProfRec r;
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return -1;
    h->prof_pool.push_back(r);
  }
  const int i = int(h->prof_used++);
  h->prof_pool[i].cls = cls;
  (void)hipEventRecord(h->prof_pool[i].a, h->stream);
  return i;
}
void prof_end(pf_handle* h, int i) {
  if (i >= 0) (void)hipEventRecord(h->prof_pool[i].b, h->stream);
}

pf_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(PF_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return PF_OK;
}

void axis_tables(int n, double dx, int kmode, bool half, std::vector<double>& tw,
                 std::vector<double>& kt) {
  tw.resize(2 * size_t(n));
  for (int q = 0; q < n; ++q) {
    const long double ang = -2.0L * 3.14159265358979323846264338327950288L * q / n;
    tw[2 * q] = double(cosl(ang));
    tw[2 * q + 1] = double(sinl(ang));
  }
  const int nk = half ? n / 2 + 1 : n;
  kt.resize(nk);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < nk; ++i) {
    const int m = (i <= n / 2) ? i : i - n;  // Eq. (16): [0..N/2, -(N/2-1)..-1]
    const double xi = 2.0 * pi * m / (n * dx);
    double v;
    if (kmode == PF_K_SPECTRAL) v = xi * xi;
    else if (kmode == PF_K_FD2) v = -2.0 * (std::cos(dx * xi) - 1.0) / (dx * dx);
    else v = -(16.0 * std::cos(dx * xi) - std::cos(2.0 * dx * xi) - 15.0) / (6.0 * dx * dx);
    kt[i] = v;
  }
}

template <typename T>
FeParams<T> fe_params(const pf_handle* h) {
  FeParams<T> f;
  f.kind = (h->cfg.fe == PF_FE_PAPER) ? FE_PAPER : FE_POLY;
  for (int i = 0; i < 12; ++i) f.k[i] = T(h->cfg.fe_coef[i]);
  return f;
}

template <typename T>
const double2* twp(const pf_handle* h, int ax) {
  return reinterpret_cast<const double2*>(h->ws + h->off_tw[ax]);
}
template <typename T>
const T* ktp(const pf_handle* h, int ax) {
  return reinterpret_cast<const T*>(h->ws + h->off_k[ax]);
}
template <typename T>
c2<T>* specB(const pf_handle* h) { return reinterpret_cast<c2<T>*>(h->ws + h->off_B); }
template <typename T>
c2<T>* specS(const pf_handle* h) { return reinterpret_cast<c2<T>*>(h->ws + h->off_S); }
template <typename T>
c2<T>* specC(const pf_handle* h) { return reinterpret_cast<c2<T>*>(h->ws + h->off_C); }
double* partials(const pf_handle* h) { return reinterpret_cast<double*>(h->ws + h->off_part); }
double* scal(const pf_handle* h) { return reinterpret_cast<double*>(h->ws + h->off_scal); }

// scalar slots in the workspace
enum { SC_MEANC = 1, SC_EN = 4, SC_DPAR = 12 };

template <typename T>
XArgs<T> xargs(const pf_handle* h) {
  XArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.twx = twp<T>(h, 0);
  a.partials = partials(h);
  a.fs_real = h->P;
  a.fs_spec = (long long)h->spec_field;
  a.rows = h->rows;
  a.Sx = h->Sx;
  a.nyo = h->nyo;
  a.F = h->F;
  a.fe = fe_params<T>(h);
  return a;
}

template <typename T>
pf_status row(pf_handle* h, XArgs<T>& a, int* nblk) {
  const int pi = prof_begin(h, PROF_ROW);
  const int g = row_launch<T>(h->nx, h->p, a, h->stream);
  prof_end(h, pi);
  if (g < 0) return fail(PF_ERR_UNSUPPORTED, "row pass: unsupported Nx");
  if (nblk) *nblk = g;
  return check_launch("row pass");
}

template <typename T>
ColArgs<T> cargs(const pf_handle* h, double dt) {
  ColArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.kcol = ktp<T>(h, 0);
  a.mean_c = scal(h) + SC_MEANC;
  a.cstate = specC<T>(h);
  a.partials = partials(h);
  a.fs_src = a.fs_dst = (long long)h->spec_field;
  a.ncols = h->nx / 2;
  a.nyq = h->nx / 2;
  a.nyo = h->nyo;
  a.F = h->F;
  a.dtM = T(dt * h->M);
  a.dtMkc = T(dt * h->M * h->kc);
  a.dtL = T(dt * h->L);
  a.dtLke = T(dt * h->L * h->ke);
  a.invP = T(1.0 / double(h->P));
  a.invPd = 1.0 / double(h->P);
  return a;
}

// Strided-axis pass.  axis 1 = y, axis 2 = z.
template <typename T>
pf_status col(pf_handle* h, ColArgs<T>& a, int axis, int* nblk) {
  const long long plane = (long long)h->ny * h->Sx;
  int n, nouter;
  if (axis == 1) {
    n = h->ny;
    a.ls = h->Sx;
    a.os = plane;
    a.nls = 1;  // Nyquist values: [z][y], contiguous along y
    a.nos = h->ny;
    nouter = h->nz;
    a.tw = twp<T>(h, 1);
    a.kaxis = ktp<T>(h, 1);
    a.kouter = (h->nd == 3) ? ktp<T>(h, 2) : nullptr;
  } else {
    n = h->nz;
    a.ls = plane;
    a.os = h->Sx;
    a.nls = h->ny;
    a.nos = 1;
    nouter = h->ny;
    a.tw = twp<T>(h, 2);
    a.kaxis = ktp<T>(h, 2);
    a.kouter = ktp<T>(h, 1);
  }
  const int pi = prof_begin(h, PROF_COL);
  const int g = col_launch<T>(n, nouter, a, h->stream);
  prof_end(h, pi);
  if (g < 0) return fail(PF_ERR_UNSUPPORTED, "column pass: unsupported length");
  if (nblk) *nblk = g;
  return check_launch("column pass");
}

pf_status reduce(pf_handle* h, int n, int width, double* out, double s0, double s1, double s2,
                 double s3, int accumulate = 0) {
  const double sc[4] = {s0, s1, s2, s3};
  const int pi = prof_begin(h, PROF_RED);
  const int g = reduce_launch(partials(h), n, width, out, sc, accumulate, h->stream);
  prof_end(h, pi);
  if (g < 0) return fail(PF_ERR_UNSUPPORTED, "reduction: record width must be 2 or 4");
  return check_launch("reduction");
}

#define PF_TRY(x)                  \
  do {                             \
    pf_status _s = (x);            \
    if (_s != PF_OK) return _s;    \
  } while (0)

// k-space update between forward and inverse transforms along the strided
// axes: 2D one column pass; 3D y-forward, z update, y-inverse.  On the first
// step of a call the spectrum of c is transformed from B (field 0) into the
// carried state; later steps reuse the carried state and B holds only the
// F right-hand sides in fields 1..F.
template <typename T>
pf_status spectral_update(pf_handle* h, double dt, bool first, int nrec) {
  ColArgs<T> a = cargs<T>(h, dt);
  a.first = first ? 1 : 0;
  a.nrec = nrec;
  if (h->nd == 2) {
    a.src = specB<T>(h);
    a.dst = specS<T>(h);
    a.mode = COL_UPDATE;
    return col<T>(h, a, 1, nullptr);
  }
  a.src = specB<T>(h);
  a.dst = specB<T>(h);
  a.mode = COL_FWD;
  a.f0 = first ? 0 : 1;
  a.F = first ? h->F + 1 : h->F;
  PF_TRY(col<T>(h, a, 1, nullptr));
  a.f0 = 0;
  a.F = h->F;
  a.dst = specS<T>(h);
  a.mode = COL_UPDATE;
  PF_TRY(col<T>(h, a, 2, nullptr));
  a.src = specS<T>(h);
  a.dst = specS<T>(h);
  a.mode = COL_INV;
  return col<T>(h, a, 1, nullptr);
}

// nsteps FS steps from real fields `uin` to real fields `uout` (may alias).
// When `store` is non-null, the states u^1..u^n are also written there
// (field-set stride F*P), which is how the adjoint recomputes a segment.
template <typename T>
pf_status fs_run(pf_handle* h, double dt, long long nsteps, const T* uin, T* uout, T* store) {
  if (nsteps == 0) {
    if (uin != uout)
      if (hipMemcpyAsync(uout, uin, h->es * h->F * h->P, hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
        return fail(PF_ERR_HIP, "hipMemcpyAsync failed");
    return PF_OK;
  }
  XArgs<T> x = xargs<T>(h);
  x.dtL = T(dt * h->L);
  x.u_in = uin;
  x.b_out = specB<T>(h);
  x.flags = X_LOAD_REAL | X_FWD_DERIV | X_WITH_C | X_CSUM;
  // the row pass writes one record {0, sum c} per work-group; the first
  // update pass takes the mean of c (the held k = 0 mode) from them
  int nb = 0;
  PF_TRY(row<T>(h, x, &nb));
  const long long fsz = (long long)h->F * h->P;
  for (long long s = 0; s < nsteps; ++s) {
    PF_TRY(spectral_update<T>(h, dt, s == 0, nb));
    XArgs<T> y = xargs<T>(h);
    y.dtL = T(dt * h->L);
    y.s_in = specS<T>(h);
    const bool last = (s == nsteps - 1);
    if (store) {
      y.u_out = store + s * fsz;
      y.flags = X_STORE_REAL | (last ? 0 : X_FWD_DERIV);
    } else {
      y.u_out = uout;
      y.flags = last ? X_STORE_REAL : X_FWD_DERIV;
    }
    y.b_out = specB<T>(h);
    PF_TRY(row<T>(h, y, nullptr));
  }
  if (store && uout) {
    if (hipMemcpyAsync(uout, store + (nsteps - 1) * fsz, h->es * fsz, hipMemcpyDeviceToDevice,
                       h->stream) != hipSuccess)
      return fail(PF_ERR_HIP, "hipMemcpyAsync failed");
  }
  return PF_OK;
}

template <typename T>
FdArgs<T> fdargs(const pf_handle* h, double dt) {
  FdArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.P = h->P;
  a.nx = h->nx;
  a.ny = h->ny;
  a.nz = h->nz;
  a.lx = log2i(h->nx);
  a.ly = log2i(h->ny);
  a.ndim = h->nd;
  a.F = h->F;
  const double* d = h->cfg.dx;
  a.ix2 = T(1.0 / (d[0] * d[0]));
  a.iy2 = T(1.0 / (d[1] * d[1]));
  a.iz2 = T(h->nd == 3 ? 1.0 / (d[2] * d[2]) : 0.0);
  a.ix = 1.0 / d[0];
  a.iy = 1.0 / d[1];
  a.iz = h->nd == 3 ? 1.0 / d[2] : 0.0;
  a.dtM = T(dt * h->M);
  a.kc = T(h->kc);
  a.dtL = T(dt * h->L);
  a.ke = T(h->ke);
  a.fe = fe_params<T>(h);
  a.partials = partials(h);
  return a;
}

template <typename T>
pf_status fd_run(pf_handle* h, double dt, long long nsteps) {
  if (nsteps == 0) return PF_OK;
  T* A = static_cast<T*>(h->fields);
  T* Bf = reinterpret_cast<T*>(h->ws + h->off_B);  // FD buffers share the FS spectra area
  T* mu = Bf + (long long)h->F * h->P;
  const size_t bytes = h->es * h->F * h->P;
  T* cur = A;
  T* nxt = Bf;
  if (nsteps & 1) {
    if (hipMemcpyAsync(Bf, A, bytes, hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
      return fail(PF_ERR_HIP, "hipMemcpyAsync failed");
    cur = Bf;
    nxt = A;
  }
  FdArgs<T> a = fdargs<T>(h, dt);
  a.mu = mu;
  for (long long s = 0; s < nsteps; ++s) {
    a.in = cur;
    a.out = nxt;
    int pi = prof_begin(h, PROF_FD);
    fd_launch<T>(0, h->p, a, h->stream);
    fd_launch<T>(1, h->p, a, h->stream);
    prof_end(h, pi);
    PF_TRY(check_launch("FD step"));
    T* t = cur;
    cur = nxt;
    nxt = t;
  }
  return PF_OK;
}

template <typename T>
pf_status energy_run(pf_handle* h, int scheme, double out[5]) {
  double* sc = scal(h) + SC_EN;
  const double dV = h->dV;
  if (scheme == 0) {
    XArgs<T> x = xargs<T>(h);
    x.u_in = static_cast<const T*>(h->fields);
    x.b_out = specB<T>(h);
    x.flags = X_LOAD_REAL | X_FWD_RAW | X_ESUM;
    int nb = 0;
    PF_TRY(row<T>(h, x, &nb));
    PF_TRY(reduce(h, nb, 2, sc, dV, dV, 0, 0));
    ColArgs<T> a = cargs<T>(h, 0.0);
    a.src = specB<T>(h);
    a.dst = specB<T>(h);
    int ng = 0;
    if (h->nd == 3) {
      a.mode = COL_FWD;
      PF_TRY(col<T>(h, a, 1, nullptr));
      a.mode = COL_ENERGY;
      PF_TRY(col<T>(h, a, 2, &ng));
    } else {
      a.mode = COL_ENERGY;
      PF_TRY(col<T>(h, a, 1, &ng));
    }
    const double s = dV / double(h->P);
    PF_TRY(reduce(h, ng, 2, sc + 2, 0.5 * h->kc * s, 0.5 * h->ke * s, 0, 0));
  } else {
    FdArgs<T> a = fdargs<T>(h, 0.0);
    a.in = static_cast<const T*>(h->fields);
    const int pi = prof_begin(h, PROF_FD);
    const int ng = fd_launch<T>(2, h->p, a, h->stream);
    prof_end(h, pi);
    PF_TRY(check_launch("FD energy"));
    // partials: {f, grad c, grad eta, c} -> sc[0..3]; reorder below
    PF_TRY(reduce(h, ng, 4, sc, dV, 0.5 * h->kc * dV, 0.5 * h->ke * dV, dV));
  }
  double hv[4];
  if (hipMemcpyAsync(hv, sc, sizeof(hv), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return fail(PF_ERR_HIP, std::string("energy readback: ") + hipGetErrorString(hipGetLastError()));
  double chem, mass, gc, ge;
  if (scheme == 0) {
    chem = hv[0];
    mass = hv[1];
    gc = hv[2];
    ge = hv[3];
  } else {
    chem = hv[0];
    gc = hv[1];
    ge = hv[2];
    mass = hv[3];
  }
  out[0] = chem + gc + ge;
  out[1] = chem;
  out[2] = gc;
  out[3] = ge;
  out[4] = mass;
  for (int i = 0; i < 5; ++i)
    if (!std::isfinite(out[i])) return fail(PF_ERR_NONFINITE, "free energy is not finite");
  return PF_OK;
}

template <typename T>
void fill_staging(pf_handle* h) {
  h->staging.assign(h->ws_need - h->off_tw[0], 0);
  unsigned char* base = h->staging.data() - h->off_tw[0];
  for (int ax = 0; ax < 3; ++ax) {
    double* tw = reinterpret_cast<double*>(base + h->off_tw[ax]);
    for (size_t q = 0; q < h->tw[ax].size(); ++q) tw[q] = h->tw[ax][q];
    T* kt = reinterpret_cast<T*>(base + h->off_k[ax]);
    for (size_t i = 0; i < h->kt[ax].size(); ++i) kt[i] = T(h->kt[ax][i]);
  }
}

// Discrete adjoint of k FS steps (see AdjArgs for the per-point algebra).
// With e = (I - S) lambda the parameter-gradient increments of one step are
//   dJ/dM += -dt q0 - q1 / M,  dJ/dkappa_c += -q1 / kappa_c,
//   dJ/dL += -dt q2 - q3 / L,  dJ/dkappa_eta += -q3 / kappa_eta.
// The segment's states are recomputed into `store` with the forward kernels,
// then the adjoint steps run from the last step to the first:
//   R2C of lambda -> strided transforms and the multipliers D_c, D_c k2,
//   D_eta (column pass, adjoint mode) -> adjoint row pass.
template <typename T>
pf_status adjoint_run(pf_handle* h, double dt, long long k, const T* u0, T* lam, double dparams[4],
                      T* store) {
  PF_TRY(fs_run<T>(h, dt, k, u0, nullptr, store));
  const long long fsz = (long long)h->F * h->P;
  double* acc = scal(h) + SC_DPAR;
  // first transform of lambda^k
  XArgs<T> x = xargs<T>(h);
  x.u_in = lam;
  x.b_out = specB<T>(h);
  x.flags = X_LOAD_REAL | X_FWD_RAW;
  PF_TRY(row<T>(h, x, nullptr));
  for (long long n = k - 1; n >= 0; --n) {
    ColArgs<T> a = cargs<T>(h, dt);
    a.src = specB<T>(h);
    if (h->nd == 2) {
      a.dst = specS<T>(h);
      a.mode = COL_ADJ;
      PF_TRY(col<T>(h, a, 1, nullptr));
    } else {
      a.dst = specB<T>(h);
      a.mode = COL_FWD;
      PF_TRY(col<T>(h, a, 1, nullptr));
      a.dst = specS<T>(h);
      a.mode = COL_ADJ;
      PF_TRY(col<T>(h, a, 2, nullptr));
      a.src = specS<T>(h);
      a.mode = COL_INV;
      a.F = h->F + 1;
      PF_TRY(col<T>(h, a, 1, nullptr));
    }
    AdjArgs<T> r;
    std::memset(&r, 0, sizeof(r));
    r.s_in = specS<T>(h);
    r.u_n = (n == 0) ? u0 : store + (n - 1) * fsz;
    r.u_np1 = store + n * fsz;
    r.lam = lam;
    r.b_out = specB<T>(h);
    r.twx = twp<T>(h, 0);
    r.mean_c = scal(h) + SC_MEANC;
    r.partials = partials(h);
    r.fs_real = h->P;
    r.fs_spec = (long long)h->spec_field;
    r.rows = h->rows;
    r.Sx = h->Sx;
    r.nyo = h->nyo;
    r.F = h->F;
    r.do_fwd = n > 0 ? 1 : 0;
    r.fe = fe_params<T>(h);
    r.dtM = T(dt * h->M);
    r.dtL = T(dt * h->L);
    const int pi = prof_begin(h, PROF_ADJ);
    const int nb = adj_row_launch<T>(h->nx, h->p, r, h->stream);
    prof_end(h, pi);
    if (nb < 0) return fail(PF_ERR_UNSUPPORTED, "adjoint row pass: unsupported Nx");
    PF_TRY(check_launch("adjoint row pass"));
    PF_TRY(reduce(h, nb, 4, acc, 1, 1, 1, 1, n == k - 1 ? 0 : 1));
  }
  double q[4];
  if (hipMemcpyAsync(q, acc, sizeof(q), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return fail(PF_ERR_HIP, std::string("adjoint readback: ") + hipGetErrorString(hipGetLastError()));
  dparams[0] += -dt * q[0] - q[1] / h->M;
  dparams[1] += -q[1] / h->kc;
  dparams[2] += -dt * q[2] - q[3] / h->L;
  dparams[3] += -q[3] / h->ke;
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(dparams[i])) return fail(PF_ERR_NONFINITE, "parameter gradient is not finite");
  return PF_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

namespace {
template <typename T>
pf_status time_pass_run(pf_handle* h, int pass, int reps, double* avg_ms) {
  const double dt = h->last_dt > 0.0 ? h->last_dt : 0.1;
  auto launch = [&]() -> pf_status {
    if (pass == 0) {
      XArgs<T> y = xargs<T>(h);
      y.dtL = T(dt * h->L);
      y.s_in = specS<T>(h);
      y.b_out = specB<T>(h);
      y.flags = X_FWD_DERIV;
      return row<T>(h, y, nullptr);
    }
    ColArgs<T> a = cargs<T>(h, dt);
    a.src = specB<T>(h);
    a.dst = specS<T>(h);
    a.mode = COL_UPDATE;
    return col<T>(h, a, h->nd == 2 ? 1 : 2, nullptr);
  };
  PF_TRY(launch());
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(PF_ERR_HIP, "hipEventCreate failed");
  pf_status st = PF_OK;
  if (hipEventRecord(e0, h->stream) != hipSuccess) st = fail(PF_ERR_HIP, "hipEventRecord failed");
  for (int i = 0; i < reps && st == PF_OK; ++i) st = launch();
  float ms = 0.f;
  if (st == PF_OK) {
    if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      st = fail(PF_ERR_HIP, "event timing failed");
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == PF_OK) *avg_ms = double(ms) / reps;
  return st;
}
}  // namespace

extern "C" {

pf_status pf_create(const pf_config* cfg, pf_handle** out) {
  if (!out) return fail(PF_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(PF_ERR_INVALID, "cfg is NULL");
  const pf_config& c = *cfg;
  if (c.ndim != 2 && c.ndim != 3) return fail(PF_ERR_INVALID, "ndim must be 2 or 3");
  const int maxn = c.ndim == 2 ? 4096 : 1024;
  for (int d = 0; d < c.ndim; ++d) {
    if (!is_pow2(c.n[d]) || c.n[d] < 8 || c.n[d] > maxn)
      return fail(PF_ERR_INVALID, "grid sizes must be powers of two in [8, " + std::to_string(maxn) + "]");
    if (!finite_pos(c.dx[d])) return fail(PF_ERR_INVALID, "dx must be finite and > 0");
  }
  if (c.ndim == 2 && c.n[2] != 1) return fail(PF_ERR_INVALID, "n[2] must be 1 in 2D");
  if (c.p < 1 || c.p > 8) return fail(PF_ERR_INVALID, "p must be in [1, 8]");
  if (c.prec != PF_F32 && c.prec != PF_F64) return fail(PF_ERR_INVALID, "prec must be PF_F32 or PF_F64");
  if (c.fe != PF_FE_POLY && c.fe != PF_FE_PAPER) return fail(PF_ERR_INVALID, "unknown free energy");
  if (c.kmode != PF_K_SPECTRAL && c.kmode != PF_K_FD2 && c.kmode != PF_K_FD4)
    return fail(PF_ERR_INVALID, "unknown kmode");
  if (!finite_pos(c.M) || !finite_pos(c.kappa_c) || !finite_pos(c.L) || !finite_pos(c.kappa_eta))
    return fail(PF_ERR_INVALID, "M, kappa_c, L, kappa_eta must be finite and > 0");
  for (int i = 0; i < 12; ++i)
    if (!std::isfinite(c.fe_coef[i])) return fail(PF_ERR_INVALID, "fe_coef must be finite");

  pf_handle* h = new (std::nothrow) pf_handle;
  if (!h) return fail(PF_ERR_INVALID, "out of host memory");
  h->cfg = c;
  h->nd = c.ndim;
  h->nx = c.n[0];
  h->ny = c.n[1];
  h->nz = c.ndim == 3 ? c.n[2] : 1;
  h->cfg.n[2] = h->nz;
  h->p = c.p;
  h->F = c.p + 1;
  h->nxh = h->nx / 2 + 1;
  h->es = c.prec == PF_F32 ? 4 : 8;
  const int align_c = c.prec == PF_F32 ? 16 : 8;  // complex values per 128 bytes
  // x-spectrum rows hold kx = 0 .. Nx/2 - 1; the Nyquist values follow the
  // rows as one array per field.  In 2D each row carries one more 128-byte
  // segment: the column pass strides along y by the row length, and a
  // power-of-two row stride made its concurrent accesses collide (measured:
  // 1024^2 FP32 column pass 17.7 -> 16.5 us, 4096^2 FP64 1.60 -> 0.95 ms),
  // except on float rows of 4096 points, where the unpadded 16 KiB stride
  // measured faster (0.43 against 0.47 ms).  3D rows (and planes) are not
  // padded: no gain was measured there.
  h->Sx = (h->nx / 2 + align_c - 1) / align_c * align_c;
  if (c.ndim == 2 && !(c.prec == PF_F32 && h->nx == 4096)) h->Sx += align_c;
  h->rows = h->ny * h->nz;
  h->P = (long long)h->nx * h->ny * h->nz;
  h->M = c.M;
  h->kc = c.kappa_c;
  h->L = c.L;
  h->ke = c.kappa_eta;
  h->dV = c.dx[0] * c.dx[1] * (c.ndim == 3 ? c.dx[2] : 1.0);
  h->stream = static_cast<hipStream_t>(c.stream);
  const int ns[3] = {h->nx, h->ny, h->nz};
  for (int ax = 0; ax < 3; ++ax) {
    const double dx = (ax < c.ndim) ? c.dx[ax] : 1.0;
    axis_tables(ns[ax], dx, c.kmode, ax == 0, h->tw[ax], h->kt[ax]);
  }
  // workspace layout
  const size_t cbytes = 2 * h->es;
  h->nyo = (long long)h->rows * h->Sx;
  h->spec_field = size_t(h->nyo) + (size_t(h->rows) + align_c - 1) / align_c * align_c;
  size_t off = 0;
  h->off_B = off;
  off = align256(off + size_t(h->F + 1) * h->spec_field * cbytes);
  h->off_S = off;
  off = align256(off + size_t(h->F + 1) * h->spec_field * cbytes);
  h->off_C = off;
  off = align256(off + h->spec_field * cbytes);
  for (int ax = 0; ax < 3; ++ax) {  // twiddle tables are double for both precisions
    h->off_tw[ax] = off;
    off = align256(off + size_t(ns[ax]) * 2 * sizeof(double));
  }
  for (int ax = 0; ax < 3; ++ax) {
    h->off_k[ax] = off;
    off = align256(off + h->kt[ax].size() * h->es);
  }
  long long np = h->rows;
  np = std::max<long long>(np, (long long)h->nxh * std::max(h->ny, h->nz) * (h->F + 1));
  np = std::max<long long>(np, (h->P + 255) / 256);
  h->nparts = np;
  h->off_part = off;
  off = align256(off + size_t(np) * 4 * sizeof(double));
  h->off_scal = off;
  off = align256(off + 64 * sizeof(double));
  h->ws_need = off;
  if (h->es == 4) fill_staging<float>(h);
  else fill_staging<double>(h);
  *out = h;
  return PF_OK;
}

void pf_destroy(pf_handle* h) {
  if (!h) return;
  for (auto& r : h->prof_pool) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  delete h;
}

size_t pf_workspace_bytes(const pf_handle* h) { return h ? h->ws_need : 0; }

size_t pf_segment_bytes(const pf_handle* h, int64_t k) {
  if (!h || k < 0) return 0;
  return size_t(k) * size_t(h->F) * size_t(h->P) * h->es;
}

pf_status pf_bind(pf_handle* h, void* fields, void* workspace, size_t workspace_bytes) {
  if (!h) return fail(PF_ERR_INVALID, "handle is NULL");
  if (!fields || !workspace) return fail(PF_ERR_INVALID, "fields and workspace must be non-NULL");
  if ((reinterpret_cast<uintptr_t>(fields) & 255) || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return fail(PF_ERR_INVALID, "fields and workspace must be 256-byte aligned");
  if (workspace_bytes < h->ws_need)
    return fail(PF_ERR_NOMEM, "workspace too small: need " + std::to_string(h->ws_need) + " bytes");
  h->fields = fields;
  h->ws = static_cast<char*>(workspace);
  if (hipMemcpyAsync(h->ws + h->off_tw[0], h->staging.data(), h->staging.size(),
                     hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return fail(PF_ERR_HIP, std::string("table upload: ") + hipGetErrorString(hipGetLastError()));
  return PF_OK;
}

pf_status pf_set_params(pf_handle* h, double M, double kappa_c, double L, double kappa_eta) {
  if (!h) return fail(PF_ERR_INVALID, "handle is NULL");
  if (!finite_pos(M) || !finite_pos(kappa_c) || !finite_pos(L) || !finite_pos(kappa_eta))
    return fail(PF_ERR_INVALID, "M, kappa_c, L, kappa_eta must be finite and > 0");
  h->M = M;
  h->kc = kappa_c;
  h->L = L;
  h->ke = kappa_eta;
  return PF_OK;
}

pf_status pf_set_stream(pf_handle* h, void* stream) {
  if (!h) return fail(PF_ERR_INVALID, "handle is NULL");
  h->stream = static_cast<hipStream_t>(stream);
  return PF_OK;
}

static pf_status check_step(pf_handle* h, double dt, int64_t nsteps) {
  if (!h) return fail(PF_ERR_INVALID, "handle is NULL");
  if (!h->ws) return fail(PF_ERR_INVALID, "pf_bind has not been called");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(PF_ERR_INVALID, "dt must be finite and > 0");
  if (nsteps < 0) return fail(PF_ERR_INVALID, "nsteps must be >= 0");
  return PF_OK;
}

pf_status pf_step_fs(pf_handle* h, double dt, int64_t nsteps) {
  PF_TRY(check_step(h, dt, nsteps));
  h->last_dt = dt;
  if (h->es == 4) {
    float* u = static_cast<float*>(h->fields);
    return fs_run<float>(h, dt, nsteps, u, u, nullptr);
  }
  double* u = static_cast<double*>(h->fields);
  return fs_run<double>(h, dt, nsteps, u, u, nullptr);
}

pf_status pf_step_fs_static(pf_handle* h, void* fields, double dt, int64_t nsteps) {
  if (!h) return fail(PF_ERR_INVALID, "handle is NULL");
  if (!fields) return fail(PF_ERR_INVALID, "fields must be non-NULL");
  if (reinterpret_cast<uintptr_t>(fields) & 255) return fail(PF_ERR_INVALID, "fields must be 256-byte aligned");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(PF_ERR_INVALID, "dt must be finite and > 0");
  if (nsteps < 0) return fail(PF_ERR_INVALID, "nsteps must be >= 0");
  if (h->ws_need > kStaticScratchBytes)
    return fail(PF_ERR_NOMEM, "pf_step_fs_static: the step needs " + std::to_string(h->ws_need) +
                                  " bytes of workspace, above the static scratch of " +
                                  std::to_string(kStaticScratchBytes) + " bytes");
  std::string why;
  char* ws = static_cast<char*>(static_scratch_ptr(why));
  if (!ws) return fail(PF_ERR_HIP, why);
  // the tables go in on every call: an earlier call on this device may have
  // left another configuration's tables (or spectra) in the scratch
  if (hipMemcpyAsync(ws + h->off_tw[0], h->staging.data(), h->staging.size(), hipMemcpyHostToDevice,
                     h->stream) != hipSuccess)
    return fail(PF_ERR_HIP, std::string("table upload: ") + hipGetErrorString(hipGetLastError()));
  // run on the scratch, then restore the handle's own binding (if any)
  char* const ws_bound = h->ws;
  void* const fields_bound = h->fields;
  h->ws = ws;
  h->fields = fields;
  h->last_dt = dt;
  pf_status st;
  if (h->es == 4) {
    float* u = static_cast<float*>(fields);
    st = fs_run<float>(h, dt, nsteps, u, u, nullptr);
  } else {
    double* u = static_cast<double*>(fields);
    st = fs_run<double>(h, dt, nsteps, u, u, nullptr);
  }
  h->ws = ws_bound;
  h->fields = fields_bound;
  return st;
}

pf_status pf_step_fd(pf_handle* h, double dt, int64_t nsteps) {
  PF_TRY(check_step(h, dt, nsteps));
  return h->es == 4 ? fd_run<float>(h, dt, nsteps) : fd_run<double>(h, dt, nsteps);
}

pf_status pf_energy(pf_handle* h, int32_t scheme, double out[5]) {
  if (!h || !out) return fail(PF_ERR_INVALID, "handle and out must be non-NULL");
  if (!h->ws) return fail(PF_ERR_INVALID, "pf_bind has not been called");
  if (scheme != 0 && scheme != 1) return fail(PF_ERR_INVALID, "scheme must be 0 (FS) or 1 (FD)");
  return h->es == 4 ? energy_run<float>(h, scheme, out) : energy_run<double>(h, scheme, out);
}

pf_status pf_adjoint_fs(pf_handle* h, double dt, int64_t k, const void* u_ckpt, void* lambda,
                        double dparams[4], void* seg_store) {
  PF_TRY(check_step(h, dt, k));
  if (!u_ckpt || !lambda || !dparams || (k > 0 && !seg_store))
    return fail(PF_ERR_INVALID, "u_ckpt, lambda, dparams and seg_store must be non-NULL");
  if (k == 0) return PF_OK;
  return h->es == 4 ? adjoint_run<float>(h, dt, k, static_cast<const float*>(u_ckpt),
                                         static_cast<float*>(lambda), dparams,
                                         static_cast<float*>(seg_store))
                    : adjoint_run<double>(h, dt, k, static_cast<const double*>(u_ckpt),
                                          static_cast<double*>(lambda), dparams,
                                          static_cast<double*>(seg_store));
}


pf_status pf_time_pass(pf_handle* h, int32_t pass, int32_t reps, double* avg_ms) {
  if (!h || !avg_ms) return fail(PF_ERR_INVALID, "handle and avg_ms must be non-NULL");
  if (!h->ws) return fail(PF_ERR_INVALID, "pf_bind has not been called");
  if ((pass != 0 && pass != 1) || reps < 1) return fail(PF_ERR_INVALID, "pass must be 0 or 1, reps >= 1");
  return h->es == 4 ? time_pass_run<float>(h, pass, reps, avg_ms)
                    : time_pass_run<double>(h, pass, reps, avg_ms);
}

pf_status pf_profile_enable(pf_handle* h, int32_t enable) {
  if (!h) return fail(PF_ERR_INVALID, "handle is NULL");
  h->prof_on = enable != 0;
  h->prof_used = 0;
  return PF_OK;
}

pf_status pf_profile_read(pf_handle* h, int32_t kernel_class, int64_t* count, double* total_ms) {
  if (!h || !count || !total_ms) return fail(PF_ERR_INVALID, "NULL argument");
  if (kernel_class < 0 || kernel_class >= PROF_NCLS) return fail(PF_ERR_INVALID, "bad kernel class");
  if (hipStreamSynchronize(h->stream) != hipSuccess)
    return fail(PF_ERR_HIP, std::string("sync: ") + hipGetErrorString(hipGetLastError()));
  int64_t n = 0;
  double ms = 0.0;
  for (size_t i = 0; i < h->prof_used; ++i) {
    if (h->prof_pool[i].cls != kernel_class) continue;
    float e = 0.f;
    if (hipEventElapsedTime(&e, h->prof_pool[i].a, h->prof_pool[i].b) != hipSuccess)
      return fail(PF_ERR_HIP, "hipEventElapsedTime failed");
    ms += e;
    ++n;
  }
  *count = n;
  *total_ms = ms;
  return PF_OK;
}

const char* pf_status_string(pf_status s) {
  switch (s) {
    case PF_OK: return "PF_OK";
    case PF_ERR_INVALID: return "PF_ERR_INVALID";
    case PF_ERR_UNSUPPORTED: return "PF_ERR_UNSUPPORTED";
    case PF_ERR_NOMEM: return "PF_ERR_NOMEM";
    case PF_ERR_HIP: return "PF_ERR_HIP";
    case PF_ERR_NONFINITE: return "PF_ERR_NONFINITE";
  }
  return "unknown pf_status";
}

const char* pf_last_error(void) { return g_err.c_str(); }

int32_t pf_version(void) { return 100; }

}  // extern "C"
