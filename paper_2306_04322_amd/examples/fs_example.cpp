// A host program that drives libpfspec through its C ABI alone: the HIP
// runtime owns the device memory, the library does every step of the
// method.  It advances the Sec. 2.1 model (f_chem, c + 4 order parameters,
// FP64) on an n x n periodic grid by `steps` semi-implicit FS steps and
// writes the initial and final fields, then prints the free energy.
//
//   fs_example N STEPS DT OUT_FILE
//
// OUT_FILE receives 2 * 5 * N * N doubles: the initial fields, then the
// final fields, each in the library's [field][y][x] layout.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "pfspec.h"

#define HIP_OK(x)                                                             \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                   \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 2;                                                               \
    }                                                                         \
  } while (0)

#define PF_OK_OR_FAIL(x)                                                      \
  do {                                                                        \
    pf_status s_ = (x);                                                       \
    if (s_ != PF_OK) {                                                        \
      std::fprintf(stderr, "%s: %s (%s)\n", #x, pf_status_string(s_), pf_last_error()); \
      return 3;                                                               \
    }                                                                         \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 5) {
    std::fprintf(stderr, "usage: %s N STEPS DT OUT_FILE\n", argv[0]);
    return 1;
  }
  const int n = std::atoi(argv[1]);
  const long steps = std::atol(argv[2]);
  const double dt = std::atof(argv[3]);
  const int p = 4, F = p + 1;

  pf_config cfg = {};
  cfg.ndim = 2;
  cfg.n[0] = n;
  cfg.n[1] = n;
  cfg.n[2] = 1;
  cfg.dx[0] = cfg.dx[1] = cfg.dx[2] = 1.0;
  cfg.p = p;
  cfg.prec = PF_F64;
  cfg.fe = PF_FE_PAPER;
  const double coef[5] = {2.0, 0.3, 0.7, 1.0, 5.0};  // rho2, c_alpha, c_beta, w, alpha (Sec. 2.1)
  for (int i = 0; i < 5; ++i) cfg.fe_coef[i] = coef[i];
  cfg.M = 5.0;
  cfg.kappa_c = 3.0;
  cfg.L = 5.0;
  cfg.kappa_eta = 3.0;
  cfg.kmode = PF_K_SPECTRAL;
  cfg.stream = nullptr;

  pf_handle* h = nullptr;
  PF_OK_OR_FAIL(pf_create(&cfg, &h));

  // a smooth periodic state: c around 0.5, small order parameters in
  // [0, 0.1] (the range of the benchmark's random initial state)
  const size_t P = size_t(n) * n;
  std::vector<double> u(F * P);
  const double k = 2.0 * M_PI / n;
  for (int y = 0; y < n; ++y)
    for (int x = 0; x < n; ++x) {
      const size_t q = size_t(y) * n + x;
      u[q] = 0.5 + 0.05 * std::cos(k * x) * std::cos(2 * k * y);
      for (int i = 0; i < p; ++i)
        u[(1 + i) * P + q] = 0.05 + 0.05 * std::sin(k * (i + 1) * x + 0.7 * i) * std::cos(k * y + 0.3 * i);
    }

  void* fields = nullptr;
  void* ws = nullptr;
  const size_t wsb = pf_workspace_bytes(h);
  HIP_OK(hipMalloc(&fields, u.size() * sizeof(double)));
  HIP_OK(hipMalloc(&ws, wsb));
  HIP_OK(hipMemcpy(fields, u.data(), u.size() * sizeof(double), hipMemcpyHostToDevice));
  PF_OK_OR_FAIL(pf_bind(h, fields, ws, wsb));
  PF_OK_OR_FAIL(pf_step_fs(h, dt, steps));
  double e[5];
  PF_OK_OR_FAIL(pf_energy(h, 0, e));  // synchronises the stream
  std::vector<double> v(u.size());
  HIP_OK(hipMemcpy(v.data(), fields, v.size() * sizeof(double), hipMemcpyDeviceToHost));

  FILE* f = std::fopen(argv[4], "wb");
  if (!f) {
    std::fprintf(stderr, "cannot write %s\n", argv[4]);
    return 4;
  }
  std::fwrite(u.data(), sizeof(double), u.size(), f);
  std::fwrite(v.data(), sizeof(double), v.size(), f);
  std::fclose(f);
  std::printf("energy %.17g chem %.17g grad_c %.17g grad_eta %.17g mass %.17g\n", e[0], e[1], e[2],
              e[3], e[4]);
  pf_destroy(h);
  HIP_OK(hipFree(ws));
  HIP_OK(hipFree(fields));
  return 0;
}
