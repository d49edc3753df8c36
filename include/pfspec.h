/*
 * libpfspec -- semi-implicit Fourier-spectral (FS) phase-field step on one
 * AMD Instinct MI355X (gfx950), with the explicit finite-difference (FD)
 * step beside it.
 *
 * Method: Boccardo et al., "Efficiency and accuracy of GPU-parallelized
 * Fourier spectral methods for solving phase-field models" (arXiv:2306.04322).
 * A coupled Cahn-Hilliard (concentration c, Eq. (2)) / Allen-Cahn (order
 * parameters eta_1..eta_p, Eq. (3)) system with free energy Eq. (1) on a
 * periodic 2D or 3D grid.
 *
 * Conventions shared by every call
 * --------------------------------
 * Fields.  One device buffer of F = 1 + p real arrays, structure of arrays,
 *   layout [F][Nz][Ny][Nx], x fastest, c first then eta_1..eta_p (Nz = 1 in
 *   2D), element type float (PF_F32) or double (PF_F64).
 * Ownership.  Every device buffer (fields, workspace, lambda, u_ckpt,
 *   seg_store) is allocated and owned by the caller and must stay valid
 *   until the queued work has completed.  The library never allocates or
 *   frees device memory; the handle owns host-side plan state only.
 * Streams.  All GPU work is enqueued on the stream given in the config (or
 *   by pf_set_stream); calls return before the work completes except where
 *   noted (pf_energy, pf_adjoint_fs synchronise the stream).  One handle per
 *   stream; a handle is not thread safe.
 * Errors.  Every call returns a pf_status.  No C++ exception crosses the
 *   ABI.  pf_last_error() returns a thread-local message for the last
 *   failure on the calling thread.  Asynchronous GPU faults surface at the
 *   next synchronising call.
 */
#ifndef PFSPEC_H
#define PFSPEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PF_OK = 0,
  PF_ERR_INVALID = 1,     /* bad argument or configuration */
  PF_ERR_UNSUPPORTED = 2, /* valid request the library does not implement */
  PF_ERR_NOMEM = 3,       /* caller-supplied buffer too small */
  PF_ERR_HIP = 4,         /* a HIP runtime call failed */
  PF_ERR_NONFINITE = 5    /* a reduction produced NaN or Inf */
} pf_status;

typedef enum { PF_F32 = 0, PF_F64 = 1 } pf_precision;

/* Chemical free-energy density.
 * PF_FE_PAPER: f = rho2 (c-c_a)^2 (1-h) + rho2 (c_b-c)^2 h + w g (Sec. 2.1),
 *   h = sum_i eta_i^3 (6 eta_i^2 - 15 eta_i + 10),
 *   g = sum_i eta_i^2 (1-eta_i)^2 + alpha sum_i sum_{j!=i} eta_i^2 eta_j^2.
 *   fe_coef = {rho2, c_alpha, c_beta, w, alpha}.
 * PF_FE_POLY: Landau polynomial (not in the paper)
 *   f = -A/2 (c-c_m)^2 + B/4 (c-c_m)^4 + D/4 (c-c_a)^4 + D/4 (c-c_b)^4
 *       - gamma/2 (c-c_a)^2 sum eta_i^2 + delta/4 sum eta_i^4
 *       + eps/2 sum_i sum_{j!=i} eta_i^2 eta_j^2.
 *   fe_coef = {c_alpha, c_beta, c_m, A, B, D, gamma, delta, eps}. */
typedef enum { PF_FE_POLY = 0, PF_FE_PAPER = 1 } pf_fe_kind;

/* Squared frequency |xi|^2 used by the FS step (Sec. 2.2):
 * PF_K_SPECTRAL Eq. (16)/(19); PF_K_FD2 Eq. (17)/(20); PF_K_FD4 Eq. (18)/(21).
 * |xi|^4 is the square of the chosen |xi|^2. */
typedef enum { PF_K_SPECTRAL = 0, PF_K_FD2 = 1, PF_K_FD4 = 2 } pf_k_kind;

typedef struct {
  int32_t ndim;        /* 2 or 3 */
  int32_t n[3];        /* Nx, Ny, Nz: powers of two, 8..4096 (2D), 8..1024 (3D); Nz = 1 in 2D */
  double dx[3];        /* grid spacing per axis, > 0 (dx[2] ignored in 2D) */
  int32_t p;           /* number of order parameters, 1..8 */
  int32_t prec;        /* pf_precision */
  int32_t fe;          /* pf_fe_kind */
  double fe_coef[12];  /* see pf_fe_kind */
  double M, kappa_c;   /* Cahn-Hilliard mobility and gradient coefficient, > 0 */
  double L, kappa_eta; /* Allen-Cahn kinetic and gradient coefficient, > 0 */
  int32_t kmode;       /* pf_k_kind */
  void* stream;        /* hipStream_t; NULL = default stream */
} pf_config;

typedef struct pf_handle pf_handle;

/* Validate `cfg` and build the host-side plan: the variables Algorithm 1
 * initialises before its time loop (the grid x_j = j dx on a periodic box of
 * N dx per axis, the frequency index vectors and |xi|^2 of Eq. (16)/(19), or
 * the FS-FD symbols of Eq. (17)/(18)/(20)/(21)), the DFT twiddles, and the
 * constants of Sec. 2.1 (the free-energy coefficients of f_chem and the
 * kinetic coefficients M, kappa_c, L, kappa_eta of Eq. (2), (3)).  The
 * tables are computed in double precision on the host.  Makes no HIP call,
 * so a bad configuration is reported without touching the GPU.
 * Returns PF_ERR_INVALID for a malformed config and *out = NULL; on success
 * the caller owns *out and releases it with pf_destroy. */
pf_status pf_create(const pf_config* cfg, pf_handle** out);

/* Release host plan state.  Does not touch caller buffers.  NULL is ignored. */
void pf_destroy(pf_handle* h);

/* Bytes of device workspace pf_bind needs (FFT intermediates, tables,
 * FD ping-pong buffer, reduction scratch), 256-byte aligned pieces. */
size_t pf_workspace_bytes(const pf_handle* h);

/* Bytes of the seg_store pf_adjoint_fs needs for a segment of k steps:
 * k field sets (k * F * Nx*Ny*Nz elements). */
size_t pf_segment_bytes(const pf_handle* h, int64_t k);

/* Attach the caller's field buffer and workspace (device pointers,
 * 256-byte aligned) and upload the tables into the workspace (enqueued on
 * the stream).  PF_ERR_NOMEM if workspace_bytes < pf_workspace_bytes(h). */
pf_status pf_bind(pf_handle* h, void* fields, void* workspace, size_t workspace_bytes);

/* Replace the kinetic coefficients (M, kappa_c, L, kappa_eta), all > 0. */
pf_status pf_set_params(pf_handle* h, double M, double kappa_c, double L, double kappa_eta);

/* Change the stream later calls enqueue on. */
pf_status pf_set_stream(pf_handle* h, void* stream);

/* Advance the bound fields by nsteps semi-implicit FS steps of size dt
 * (Algorithm 1; Eq. (10)-(15)), in place.  Per step: the free-energy
 * derivatives at time t, forward transforms, the diagonal k-space solve,
 * inverse transforms.  The mean of c (the k = 0 mode) is held in double
 * precision for the whole call.  dt > 0 and nsteps >= 0, else
 * PF_ERR_INVALID.  Asynchronous. */
pf_status pf_step_fs(pf_handle* h, double dt, int64_t nsteps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * FS steps as pf_step_fs, on the field buffer `fields` (device, 256-byte
 * aligned, layout and precision of the handle's config), with the step's
 * workspace taken from a static device array of the library
 * (PF_STATIC_SCRATCH_BYTES = 64 MiB, one copy per GPU, held from the
 * library's load until the process exits) instead of a caller buffer.
 * Needs no pf_bind and leaves the handle's binding untouched.  Allocates
 * nothing: no hipMalloc, hipFree or allocating library call.  Runs on the
 * current device; the first call on a device looks up the array's device
 * address.  The tables are re-uploaded (hipMemcpyAsync from host memory
 * the handle holds) on every call, and every workspace value the step
 * reads is written earlier in the same call, so nothing carries over
 * between calls.  All calls on one GPU share the one array: calls that overlap in
 * time on one GPU (other streams, other threads) race and give wrong
 * results.  PF_ERR_NOMEM if pf_workspace_bytes(h) exceeds the array;
 * PF_ERR_INVALID for a NULL or unaligned `fields`, dt <= 0 or nsteps < 0.
 * Asynchronous, like pf_step_fs. */
#define PF_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
pf_status pf_step_fs_static(pf_handle* h, void* fields, double dt, int64_t nsteps);

/* Advance the bound fields by nsteps explicit FD steps (Sec. 2.2: forward
 * Euler, 5-point (2D) / 7-point (3D) periodic Laplacian; every right-hand
 * side at time t), in place.  dt > 0 and nsteps >= 0, else PF_ERR_INVALID.
 * Asynchronous. */
pf_status pf_step_fd(pf_handle* h, double dt, int64_t nsteps);

/* Free energy of the bound fields (Eq. (1)), accumulated in double:
 * out = {E_total, E_chem, E_grad_c, E_grad_eta, mass}, mass = dV * sum c.
 * scheme 0: gradient terms in the FS spectral form with the handle's
 * |xi|^2; scheme 1: forward-difference squares (FD form).
 * Synchronises the stream.  PF_ERR_NONFINITE if any output is not finite. */
pf_status pf_energy(pf_handle* h, int32_t scheme, double out[5]);

/* Discrete adjoint of k FS steps of size dt starting from the field set
 * u_ckpt (device, same layout as the fields).
 * In:  lambda (device, F field layout) = dJ/du^k.
 * Out: lambda = dJ/du^0 of the segment; dparams[0..3] (host, double) +=
 *      dJ/d(M, kappa_c, L, kappa_eta).
 * seg_store (device, pf_segment_bytes(h, k) bytes) receives the recomputed
 * states u^1..u^k.  The recomputation uses the same kernels as pf_step_fs,
 * so it reproduces the forward trajectory bit for bit.  The bound fields
 * are not modified.  Synchronises the stream. */
pf_status pf_adjoint_fs(pf_handle* h, double dt, int64_t k, const void* u_ckpt,
                        void* lambda, double dparams[4], void* seg_store);

/* Per-kernel-class timing with HIP events recorded around each launch on
 * the handle's stream.  enable != 0 starts a fresh record. */
pf_status pf_profile_enable(pf_handle* h, int32_t enable);

/* Synchronise and report the launches recorded for `kernel_class`
 * (0 = row pass, 1 = column pass, 2 = FD stencil, 3 = reduction,
 *  4 = adjoint row pass): count and summed milliseconds. */
pf_status pf_profile_read(pf_handle* h, int32_t kernel_class, int64_t* count, double* total_ms);

/* Time one pass of the steady-state FS step on its own: `pass` 0 = the row
 * pass (inverse x transform, free-energy derivative, forward x transform),
 * 1 = the k-space update pass (the column pass in 2D; the z-update pass in
 * 3D).  Launches it `reps` times back to back on the handle's stream
 * between two events, after one untimed launch, and returns the average
 * milliseconds per launch in *avg_ms (synchronises).  Reads and rewrites
 * the step's intermediate buffers in the workspace, so call it after
 * pf_step_fs; the bound fields are not touched.  reps >= 1. */
pf_status pf_time_pass(pf_handle* h, int32_t pass, int32_t reps, double* avg_ms);

const char* pf_status_string(pf_status s);
const char* pf_last_error(void);
int32_t pf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PFSPEC_H */
