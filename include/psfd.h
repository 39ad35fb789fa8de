/*
 * psfd.h -- C ABI of the MI355X background-field PSFD / Lippmann-Schwinger solver.
 *
 * The library solves the EUV mask scattering problem of the paper "Pseudo-spectral
 * frequency-domain method with background field decomposition and Green's function
 * preconditioner": the absorber field E_mask on a periodic clip above a planar
 * multilayer, from
 *   - the discrete Lippmann-Schwinger system of eq. (18),
 *       x - IFFT(F[G_L] . FFT(V x)) = IFFT(F[G_L] . FFT(V (E_inc + E_layer))),
 *     V = k0^2 delta_eps, with the windowed dyadic Green's function of eqs. (13)-(17)
 *     (windowed in z over the absorber thickness, exact per transverse order in x, y),
 *   - the outer fixed point of eqs. (8)-(9): E_layer is the multilayer reflection
 *     T_R (per transverse Fourier order, generalized reflection coefficients) of the
 *     downgoing field at the multilayer surface, propagated up per order.
 *
 * Conventions
 *   - lengths in nm; time dependence exp(-i w t); absorbing media have Im(eps) > 0.
 *   - grid: nx, ny, nz powers of two, 4 <= nx, ny <= 256, 2 <= nz <= 128; x, y periodic
 *     with period lx, ly (Floquet phase of the incidence); z covers the absorber
 *     [0, t] with cell-centred planes z_k = (k + 1/2) t / nz; z = 0 is the multilayer.
 *   - complex arrays are interleaved (re, im). Fields are ENVELOPES
 *     u = E exp(-i (kx0 x + ky0 y)) laid out [3][nz][ny][nx] (component, z, y, x) with
 *     sample (k, j, i) at x = i lx/nx, y = j ly/ny, z = z_k.
 *   - the contrast delta_eps = eps - eps_bg is [nz][ny][nx].
 *   - order amplitudes are [ny][nx][3] in FFT order: index (j, i) is the order
 *     (n, m) = (fftfreq index of j, of i) with kx = kx0 + 2 pi m / lx.
 *   - every device pointer is owned by the caller, must stay valid until the call
 *     returns, and must not alias another argument unless stated.
 *   - `stream` is a hipStream_t (0 = default stream); calls are ordered on it.
 *   - every call returns PSFD_OK (0), PSFD_NOT_CONVERGED (> 0, outputs written and
 *     info filled) or a negative error; psfd_last_error() gives a thread-local
 *     message for the last failing call of the calling thread.
 */
#ifndef PSFD_H
#define PSFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PSFD_OK = 0,
  PSFD_NOT_CONVERGED = 1,
  PSFD_ERR_INVALID_ARG = -1,
  PSFD_ERR_UNSUPPORTED_SIZE = -2,
  PSFD_ERR_OOM = -3,
  PSFD_ERR_SINGULAR = -4, /* an order grazes the surface (beta = 0, Wood anomaly) */
  PSFD_ERR_NONFINITE = -5,
  PSFD_ERR_HIP = -6
};

enum { PSFD_TE = 0, PSFD_TM = 1 };
enum { PSFD_FP64 = 0, PSFD_MIXED = 1 };             /* psfd_opts.precision */
enum { PSFD_C64 = 0, PSFD_C128 = 1 };               /* dtype of psfd_apply */
enum { PSFD_APPLY_TRANSPOSE = 1, PSFD_APPLY_K_ONLY = 2, PSFD_APPLY_REFLECT = 4 }; /* psfd_apply flags */
enum { PSFD_COUPLING_OUTER = 0, PSFD_COUPLING_MONO = 1 };  /* psfd_opts.coupling */

typedef struct { double eps_re, eps_im, thickness_nm; } psfd_layer; /* top to bottom */

/* Problem statement (Sec. 2 and the experiment set-ups of Sec. 3). */
typedef struct {
  int32_t nx, ny, nz;
  double lx_nm, ly_nm, t_nm;      /* clip period (x, y) and absorber thickness */
  double wavelength_nm, eps_bg;   /* eps_bg real and positive (vacuum: 1) */
  double theta_deg, phi_deg;      /* incidence polar angle and azimuth */
  int32_t pol;                    /* PSFD_TE: E along s = (-sin phi, cos phi, 0); PSFD_TM: E along p- */
  int32_t n_layers;
  const psfd_layer* layers;       /* host array of n_layers layers, copied at plan creation */
  double eps_sub_re, eps_sub_im;  /* substrate half-space */
} psfd_problem;

/* Solver options. rtol: relative residual of eq. (18) (GMRES, Saad & Schultz);
 * outer_rtol: relative change of the reflected spectrum that ends the outer loop
 * of eqs. (8)-(9) (<= 0: use rtol); restart: GMRES(m), 1 <= m <= 32;
 * max_iters: Arnoldi steps per linear solve; max_outer: outer iterations;
 * precision: PSFD_FP64, or PSFD_MIXED (FP32 Arnoldi cycles, FP64 residual and
 * solution: each restart recomputes the residual in FP64); inner_eta: relative
 * reduction asked of one FP32 cycle (<= 0: 1e-4); coupling: PSFD_COUPLING_OUTER
 * runs the outer fixed point of eqs. (8)-(9) (each step a GMRES solve of eq. (18),
 * rtol tightened to 0.1 rtol as the reflection settles), PSFD_COUPLING_MONO runs
 * GMRES once on (I - (K + R_vol T_R K_top) V) u = e_bg, whose solution is that
 * fixed point (default). */
typedef struct {
  double rtol, outer_rtol;
  int32_t restart, max_iters, max_outer, precision;
  double inner_eta;
  int32_t coupling;
} psfd_opts;

typedef struct {
  int32_t iters;          /* Arnoldi steps, all outer iterations */
  int32_t outer_iters;
  int32_t cycles;         /* GMRES cycles (FP64 residual evaluations) */
  int32_t status;
  double rel_residual;    /* last FP64 relative residual of eq. (18) */
  double outer_change;    /* last relative change of the reflected spectrum */
  double mono_residual;   /* FP64 ||e_bg - (I - (K + R K_top) V) u|| / ||e_bg|| of the total field */
} psfd_info;

typedef struct psfd_plan psfd_plan;
typedef struct psfd_server psfd_server;

/* Build the FP64 tables of a problem (orders, reflection matrices T_R from the
 * recursive generalized reflection of the stack, kernel scalars, FFT twiddles)
 * on the current HIP device (the plan's device; blocks until they are there). opts may be NULL (defaults: rtol 1e-6, restart 30,
 * max_iters 5000, max_outer 100, PSFD_MIXED). Errors: INVALID_ARG,
 * UNSUPPORTED_SIZE, SINGULAR, OOM, HIP. */
int psfd_plan_create(const psfd_problem* prob, const psfd_opts* opts, psfd_plan** out);
void psfd_plan_destroy(psfd_plan* plan);
/* Device bytes a solve with this plan allocates (tables + Krylov workspace). */
int psfd_plan_footprint(const psfd_plan* plan, size_t* device_bytes);

/* One operator apply (eq. (18)): y = x - K(V x), or y = K(V x) with
 * PSFD_APPLY_K_ONLY; with PSFD_APPLY_TRANSPOSE the bilinear transpose (kernel at
 * the negated wavevector); with PSFD_APPLY_REFLECT, K is replaced by the coupled
 * M = K + R_vol T_R K_top (free space plus the multilayer response of eq. (9)). d_deps [nz][ny][nx], d_x and d_y [3][nz][ny][nx], all of
 * `dtype` (complex64 or complex128), device memory; d_y must not alias d_x.
 * Uses a plan-owned scratch field (allocated on first use). On 128 x 128 planes
 * with nz 32 or 64 the transverse transforms run split four ways over y (rows
 * y = 4 r + q) and the z pencil combines the quarter spectra; the environment
 * variable PSFD_QUARTER_PLANES=0 selects the one-block-per-plane (FP32) or
 * strip (FP64) transforms instead (same results to rounding). */
int psfd_apply(psfd_plan* plan, const void* d_deps, const void* d_x, void* d_y, int dtype, int flags,
               void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): psfd_apply with the same
 * arguments, kernels and results, that allocates nothing. Its workspace (3 nx ny nz
 * values of `dtype`) lives in a static device array of PSFD_NOALLOC_SCRATCH_BYTES
 * per device, held until the process ends; the plan's device tables come from
 * psfd_plan_create. The plan's device must be current. A grid whose workspace
 * exceeds the array (e.g. 256 x 256 x 64 in complex128) is refused with
 * UNSUPPORTED_SIZE. Every call on a device shares that device's array: calls
 * that overlap on one device (on different streams or threads) race; calls
 * ordered on one stream do not. Asynchronous on `stream`. */
#define PSFD_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int psfd_apply_noalloc(psfd_plan* plan, const void* d_deps, const void* d_x, void* d_y, int dtype, int flags,
                       void* stream);

/* Full solve (Sec. 2, eqs. (8)-(9); Sec. 3, eq. (18)): the background source,
 * GMRES on eq. (18) with the monolithic or outer coupling of the multilayer
 * response, and the readouts. d_deps complex128 [nz][ny][nx] (device); outputs
 * (complex128, device): d_emask [3][nz][ny][nx] = E_mask envelope, d_orders
 * [ny][nx][3] = reflected order amplitudes a_q at z = t (may be NULL), d_u
 * [3][nz][ny][nx] = the total field u = E_inc + E_layer + E_mask in the slab
 * (may be NULL; what psfd_solve_adjoint takes: E_mask alone does not determine
 * the layered part, which follows from the downgoing readout of V u). Blocks
 * until done. Returns NOT_CONVERGED when an iteration limit stops it. */
int psfd_solve(psfd_plan* plan, const void* d_deps, void* d_emask, void* d_orders, void* d_u, psfd_info* info,
               void* stream);

/* Adjoint solve: the vector-Jacobian product of the reflected orders with
 * respect to the contrast, for any real loss L of the orders. The orders
 * a = c0 + W V u are holomorphic in delta_eps, u being the total field of
 * (I - M V) u = e_bg (M = K + R_vol T_R K_top, eqs. (3), (8)-(9), (18)); with
 * lambda = (I - M^T V)^-1 W^T conj(G) (the transposed coupled system, kernel
 * at the negated wavevector), dL = Re sum_r k0^2 d(delta_eps) sum_c lambda_c u_c.
 * Inputs (device, complex128): d_deps [nz][ny][nx]; d_u [3][nz][ny][nx], the
 * forward total field (psfd_solve's d_u with the same plan and contrast);
 * d_grad_orders [ny][nx][3], G = dL/dRe a + i dL/dIm a (PyTorch's convention
 * for complex tensors, twice dL/d conj(a)). Output d_grad [nz][ny][nx]
 * (device, complex128, must not alias an input) = dL/dRe delta_eps + i dL/dIm
 * delta_eps. The transposed GMRES runs with the plan's options (tolerance,
 * restart, precision); info (may be NULL) receives its counters. Blocks until
 * done. Errors: INVALID_ARG, NONFINITE, OOM, HIP; NOT_CONVERGED with d_grad
 * written when the iteration limit stops the solve. */
int psfd_solve_adjoint(psfd_plan* plan, const void* d_deps, const void* d_u, const void* d_grad_orders,
                       void* d_grad, psfd_info* info, void* stream);

/* Batched solves of instances of one grid shape (same nx, ny, nz, lx, ly, t,
 * wavelength and stack; angles, polarisation and contrast per instance) in
 * lock-step batched launches. probs[i] / d_deps[i] / d_emask[i] / d_orders[i]
 * per instance (device pointers, complex128). info array of n. */
int psfd_solve_batch(int32_t n, const psfd_problem* probs, const psfd_opts* opts, const void* const* d_deps,
                     void* const* d_emask, void* const* d_orders, psfd_info* info, void* stream);

/* psfd_solve_batch keeps the device workspace of its last calls (at most 4, per
 * device, shape, batch size, restart length and precision; least recently used
 * freed first) and reuses it for the next call of the same kind. This frees
 * every kept workspace; calls running in other threads keep theirs. */
int psfd_release_cached_workspaces(void);

/* Serving: continuous batching of solve requests admitted by device-memory
 * footprint. Requests of one kind (grid shape, restart length, precision,
 * inner_eta) share a slot group; tolerance and iteration limit are per
 * request. A group of min(max_slots, free budget / slot bytes) slots is
 * created when a request of its kind arrives and one slot fits what is left
 * of hbm_budget (bytes of device workspace the server may allocate; a slot is
 * psfd_plan_footprint's bytes). Otherwise the request waits, first come first
 * served: idle groups are released and the oldest busy groups drained (they
 * finish their slots, then free their memory) until it fits. A group idle for
 * 5 s frees its memory. Only a request that does not fit even an empty budget
 * completes at once with PSFD_ERR_OOM. Every group has its own worker thread
 * and HIP stream, so groups run concurrently; a group issues its Arnoldi steps
 * as plain launches (no stream capture, which other threads' work could
 * invalidate). Served solves use the monolithic coupling;
 * a served result equals the lone psfd_solve of the same problem and options
 * (same kernels, reductions in a fixed order per instance).
 * create: opts (may be NULL: library defaults) are the defaults of requests
 * submitted without options. submit copies the problem and options (opts may
 * be NULL: the server's; the coupling field is ignored); the caller's buffers
 * must stay valid until poll reports done. destroy finishes every submitted
 * request, then frees the workspaces. submit / poll are thread-safe. */
int psfd_server_create(size_t hbm_budget, int32_t max_slots, const psfd_opts* opts, psfd_server** out);
int psfd_server_submit(psfd_server* srv, const psfd_problem* prob, const psfd_opts* opts, const void* d_deps,
                       void* d_emask, void* d_orders, uint64_t* ticket);
/* done = 1 once finished; info filled then. latency_s (may be NULL): submit to
 * completion wall time. */
int psfd_server_poll(psfd_server* srv, uint64_t ticket, int32_t* done, psfd_info* info, double* latency_s);
int psfd_server_destroy(psfd_server* srv);

/* Diagnostics: run stage `stage` of psfd_apply (0: transverse forward FFT with
 * the contrast multiply, 1: z-pencil FFT / dyadic kernel / inverse, 2: transverse
 * inverse FFT with the axpy) `reps` times back to back between two HIP events on
 * `stream` and store the mean time per launch in *ms. Same buffers as psfd_apply
 * (d_y receives stage 2's output; the plan scratch holds stages 0-1), with the
 * kernels psfd_apply takes for the shape. For throughput measurements; results of
 * a lone stage are not an operator apply. */
int psfd_bench_stage(psfd_plan* plan, int stage, const void* d_deps, const void* d_x, void* d_y, int dtype,
                     int reps, float* ms, void* stream);

/* Diagnostics: time one classical Gram-Schmidt pass of the Arnoldi step at
 * column j (0 <= j < 32), on the plan's grid: pass 0 the projections <v_i, w>
 * (i <= j) and ||w||^2 of GMRES (Saad & Schultz; Sec. 3), pass 1 the update
 * w -= sum_i h_i v_i with the ||w||^2 partials, pass 2 the step's inverse
 * transverse FFT kernel that writes w (stage 2 of the operator apply, eq. (18)),
 * which on FP32 64 x 64 and 128 x 128 planes also forms the projections of pass 0 (then
 * no separate pass 0 runs in a step), pass 3 the forward transverse FFT kernel
 * of step j + 1 (stage 0, contrast from the first nz*ny*nx values of d_x),
 * which on FP32 64 x 64 and 128 x 128 planes in lock-step solves also does the update of
 * pass 1 for column j (then pass 1 runs only at the last column of a cycle).
 * A basis of j + 2 vectors of
 * `dtype`, each a copy of d_x (complex64 or complex128 [3][nz][ny][nx], device),
 * is allocated for the call and freed after it; the pass runs once untimed,
 * then `reps` times back to back between two HIP events on `stream`, and *ms
 * receives the mean time per launch. Blocks until done. For throughput
 * measurements only (the passes run on copies, not on an orthogonal basis). */
int psfd_bench_gram_schmidt(psfd_plan* plan, int pass, int j, const void* d_x, int dtype, int reps, float* ms,
                            void* stream);

/* ------------------------------------------------------------------------
 * Isolated-domain mode: a scatterer in free space (no periodicity, no
 * multilayer), with the dyadic Green's function truncated to a ball of radius R
 * (the windowed kernel of eqs. (13) and (15)-(17), with h(k; R) carrying R^2
 * and A(0) the factor 4 pi) and the convolution of eq. (18) zero-padded to twice
 * the grid on all three axes. The kernel table is precomputed once per plan in
 * FP64 from the closed form F[G_R] = A(k) I + B(k) k^ k^: sampled on a grid
 * oversampled per axis (factor o_a, the smallest power of two >= max(4, 1 + R /
 * L_a), L_a = n_a h_a; Nyquist planes zeroed), inverse DFT, restricted to the
 * offsets [-n, n) per axis, forward DFT on the 2n grid.
 *
 * Grid: nx, ny, nz powers of two in [2, 128] with o_a n_a <= 1024; voxel sizes
 * dx, dy, dz in nm; sample (k, j, i) at (i dx, j dy, k dz). Fields are
 * [3][nz][ny][nx] (component x, y, z), the contrast delta_eps = eps - eps_bg is
 * [nz][ny][nx], V = k0^2 delta_eps, k0 = 2 pi / wavelength, k_bg = k0 sqrt(eps_bg).
 */
typedef struct psfd_iso_plan psfd_iso_plan;

typedef struct {
  int32_t nx, ny, nz;
  double dx_nm, dy_nm, dz_nm;   /* voxel size */
  double wavelength_nm;
  double eps_bg_re, eps_bg_im;  /* background permittivity: Re > 0, Im >= 0 */
  double radius_nm;             /* window radius R; <= 0: the box diagonal sqrt(sum L_a^2) */
} psfd_iso_problem;

/* Validate the problem and precompute the kernel table on the current device
 * (blocks until done; the precompute holds 96 prod(o_a n_a) bytes of device
 * memory while it runs; the plan keeps the natural FP64 table, 768 nx ny nz
 * bytes, and the tables in the order of the z pass, 576 (nz + 1) nx ny bytes
 * for FP64 and FP32 together). *out receives the plan, owned by the caller and
 * released with psfd_iso_plan_destroy. Errors: INVALID_ARG, UNSUPPORTED_SIZE
 * (a size, or a radius that needs o_a n_a > 1024), OOM / HIP. */
int psfd_iso_plan_create(const psfd_iso_problem* prob, psfd_iso_plan** out);
void psfd_iso_plan_destroy(psfd_iso_plan* plan);

/* y = x - P IFFT(table . FFT(Z V x)) (eq. (18) for the isolated scatterer; Z
 * pads every axis to twice its length, P restricts back). d_deps, d_x, d_y:
 * device arrays of `dtype` (PSFD_C64: complex64, FP32 arithmetic on the FP32
 * rounding of the table; PSFD_C128: complex128, FP64); d_y must not alias d_x.
 * A workspace of 96 nx ny nz (C64) or 192 nx ny nz (C128) bytes is allocated at
 * the first call of each dtype and kept with the plan. Asynchronous on
 * `stream`; calls on one plan must not overlap. */
int psfd_iso_apply(psfd_iso_plan* plan, const void* d_deps, const void* d_x, void* d_y, int dtype, void* stream);

/* Solve u - P IFFT(table . FFT(Z V u)) = b (eq. (18) for the isolated scatterer,
 * b e.g. the incident field sampled on the grid) by GMRES(restart) (Saad &
 * Schultz) from u = 0: classical Gram-Schmidt (a second pass where the update
 * leaves less than 1/sqrt(2) of the norm), every restart
 * from the FP64 residual b - A u, u accumulated in FP64. precision: PSFD_FP64,
 * or PSFD_MIXED (FP32 basis and applies; a cycle also ends after reducing the
 * residual 1e4-fold). d_deps, d_b, d_u: complex128 device
 * arrays ([nz][ny][nx], [3][nz][ny][nx] twice); d_u must not alias d_b. Stops
 * when ||b - A u|| <= rtol ||b|| (info->rel_residual) or after max_iters
 * Arnoldi steps (then PSFD_NOT_CONVERGED, u written). 1 <= restart <= 64. The
 * basis ((restart + 1) 48 nx ny nz bytes in FP64, half in mixed), two FP64
 * vectors and, in mixed precision, an FP32 copy of the contrast (8 nx ny nz
 * bytes) are allocated for the call. Blocks
 * until done; calls on one plan must not overlap. */
int psfd_iso_solve(psfd_iso_plan* plan, const void* d_deps, const void* d_b, void* d_u, double rtol, int32_t restart,
                   int32_t max_iters, int32_t precision, psfd_info* info, void* stream);

/* The precomputed table (may be NULL): complex128 [6][2nz][2ny][2nx], the
 * entries xx, yy, zz, xy, xz, yz of the symmetric 3 x 3 kernel per wavevector
 * of the padded grid in FFT order, copied to the device array d_table on
 * `stream`. over (may be NULL): the 3 oversampling factors (z, y, x) of the
 * precompute; radius_nm (may be NULL): R. */
int psfd_iso_table(psfd_iso_plan* plan, void* d_table, int32_t* over, double* radius_nm, void* stream);

/* Diagnostics: run pass `stage` of psfd_iso_apply (-1: all of it; 0: x rows
 * times V, FFT; 1: y columns FFT; 2: z FFT, table product, inverse z FFT; 3:
 * inverse y columns; 4: inverse x rows with y = x - w) `reps` times back to back
 * between two HIP events on `stream`; *ms receives the mean time per launch.
 * Same buffers as psfd_iso_apply. Blocks until done. */
int psfd_iso_bench_stage(psfd_iso_plan* plan, int stage, const void* d_deps, const void* d_x, void* d_y, int dtype,
                         int reps, float* ms, void* stream);

/* ------------------------------------------------------------------------
 * Differential PSFD operator with a z-PML: the comparison solver of the
 * preconditioner study (Sec. 3). The curl-curl equation of the mask field on
 * the homogeneous background (eq. (8)),
 *     A E = curl curl E - k_bg^2 E - V E = V e_src,   V = k0^2 delta_eps,
 * discretised pseudo-spectrally (every derivative a Fourier derivative along
 * its axis, eq. (6)); the clip is periodic in x and y (Floquet envelopes, as on
 * the main path) and z covers an extended grid of nz_ext planes of spacing
 * t_nm / nz, with perfectly matched layers at both ends where the z derivative
 * is stretched by 1 / (1 + i s(z)) (eq. (7)); s(z) = s_max (d / L)^p at the depth
 * d of the plane centre into a layer of L = pml_cells planes, s_max =
 * (p + 1) ln(1 / R0) / (2 k_bg L) for a target round-trip reflection R0. The
 * z derivative zeroes the z-Nyquist wavenumber. Preconditioning on the left:
 * PSFD_PRECOND_NONE (A x = b) or PSFD_PRECOND_DAMPING (D A x = D b with the
 * spectral damping D(k) = min(1, k_bg^2 / |k|^2) of the full wavevector).
 * Forms: PSFD_DIFF_BACKGROUND, the background-field method: the contrast planes
 * are the absorber, e_src = E_inc + E_layer with E_layer from the multilayer
 * reflection T_R of the downgoing field at z = 0, read on the plane below the
 * absorber, in an outer fixed point (eqs. (8)-(9)); PSFD_DIFF_FULL_DOMAIN, the
 * full-domain method: the multilayer is on the grid as contrast (the caller
 * builds it into the contrast planes below the absorber), e_src = E_inc, and
 * the background medium continues below the stack (no reflection operator).
 * Planes z_k = (k - z0 + 1/2) dz with z0 the absorber's first plane; the
 * absorber is the top nz of the ncz contrast planes starting at zc0. Fields
 * [3][nz_ext][ny][nx], contrast [ncz][ny][nx]. */
typedef struct psfd_diff_plan psfd_diff_plan;
enum { PSFD_DIFF_BACKGROUND = 0, PSFD_DIFF_FULL_DOMAIN = 1 };
enum { PSFD_PRECOND_NONE = 0, PSFD_PRECOND_DAMPING = 1 };

typedef struct {
  psfd_problem base;       /* clip, incidence, multilayer, absorber grid (nz planes over t_nm) */
  int32_t nz_ext;          /* planes of the extended z grid: a power of two in [16, 1024] */
  int32_t zc0, ncz;        /* contrast planes [zc0, zc0 + ncz); background form: ncz = base.nz */
  int32_t pml_cells;       /* PML planes at each end (0: none, the z axis stays periodic) */
  int32_t pml_order;       /* grading p (<= 0: 3) */
  double pml_reflection;   /* R0 (outside (0, 1): 1e-8) */
  int32_t form;            /* PSFD_DIFF_BACKGROUND or PSFD_DIFF_FULL_DOMAIN */
} psfd_diff_problem;

/* Validates (pml_cells + 1 <= zc0, zc0 + ncz + 1 <= nz_ext - pml_cells: a readout
 * plane on each side of the contrast planes outside the PML) and builds the
 * tables on the current device (blocks). Errors: INVALID_ARG, UNSUPPORTED_SIZE,
 * SINGULAR, OOM, HIP. */
int psfd_diff_plan_create(const psfd_diff_problem* prob, psfd_diff_plan** out);
void psfd_diff_plan_destroy(psfd_diff_plan* plan);
/* y = A x or D A x (precond); d_deps [ncz][ny][nx], d_x, d_y [3][nz_ext][ny][nx],
 * all of dtype (PSFD_C64: FP32 arithmetic, PSFD_C128: FP64), device; d_y must not
 * alias d_x. A workspace of one field of dtype is allocated at the first call of
 * each dtype and kept with the plan. Asynchronous on stream. */
int psfd_diff_apply(psfd_diff_plan* plan, const void* d_deps, const void* d_x, void* d_y, int dtype, int precond,
                    void* stream);
/* Solve of the form: GMRES(restart) (host-driven, restarts from the FP64
 * residual; opts->precision PSFD_MIXED: FP32 basis and applies) on the
 * (preconditioned) system to opts->rtol, inside the outer fixed point of the
 * background form until the reflected spectrum changes by at most outer_rtol
 * (<= 0: rtol) or max_outer steps. d_deps complex128 [ncz][ny][nx]; d_e
 * (complex128 [3][nz_ext][ny][nx]) receives the mask field (background form) or
 * the scattered field (full domain) on the extended grid; d_orders (may be
 * NULL; complex128 [ny][nx][3]) the reflected order amplitudes at z = t (the
 * top of the absorber), the same quantity psfd_solve returns. opts may be NULL
 * (defaults of psfd_plan_create; restart <= 64). Blocks; NOT_CONVERGED when a
 * limit stops it. */
int psfd_diff_solve(psfd_diff_plan* plan, const void* d_deps, void* d_e, void* d_orders, const psfd_opts* opts,
                    int precond, psfd_info* info, void* stream);

const char* psfd_status_string(int status);
const char* psfd_last_error(void);
const char* psfd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PSFD_H */
