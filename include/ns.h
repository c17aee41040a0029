/*
 * ns.h -- C ABI of libns.so: the dealiased nonlinear term of 3D periodic
 * incompressible Navier-Stokes and the Runge-Kutta schemes built on it, on one
 * AMD Instinct MI355X (gfx950).  Method: Lambert, Reneuve & Augier,
 * "Aliasing and phase shifting in pseudo-spectral simulations of the
 * incompressible Navier-Stokes equations" (arXiv 2603.08892).
 *
 * Problem (Eq. base-eq): dS/dt = sigma S + N(S), S = u_hat the spectral velocity,
 * sigma(k) = -nu |k|^2, N(S) the divergence-free projection of the advective term,
 * evaluated pseudo-spectrally in rotational form, N = M P FFT(u x omega).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Box 2*pi, N points per direction, integer wavenumbers.  Forward transform
 * u_hat(k) = N^-3 sum_x u(x) exp(-i k.x), inverse unnormalised (Eqs. u_fft_1d,
 * u_expansion_1d and supplementary Eq. dft_def).
 *
 * Spectral field layout ("state layout"): 3 components, each [N][N][N/2+1]
 * complex in C order, interleaved (re, im); component stride N*N*(N/2+1)
 * complex.  Axis 0 is k_x, axis 1 is k_y, both in FFT index order (index i < N/2
 * holds k = i, else k = i - N); axis 2 is k_z = 0..N/2, contiguous.  Element type
 * is float2 for NS_FP32 and double2 for NS_FP64 (cfg.precision).
 *
 * Truncation (Sec. "Standard dealiasing with truncation", Fig. 1): with
 * k_max = ct*N/2, the sphere keeps integer |k|^2 <= K2max, K2max the largest
 * integer strictly below k_max^2; the cube keeps max_i |k_i| <= Kmax, Kmax the
 * largest integer strictly below k_max.  A real value within a relative 1e-9 of
 * an integer is taken as that integer (so C_t = 2/3 at N = 192 keeps K2max = 4095).
 * States live in the retained set: on input every mode outside it is ignored
 * (treated as zero); on output every mode outside it is zero.
 *
 * Shifts are in grid-spacing units: s = (sx, sy, sz) means Delta = s*2*pi/N and the
 * phase factor exp(2 pi i k.s / N) (Eqs. shift_operator, shift_operator_3d).
 *
 * Memory and streams: every field pointer of the 3D calls is a device pointer,
 * 256-byte aligned, owned by the caller; the library allocates no device memory
 * (only a few KB of pinned host memory per context for the spectra results).
 * The caller provides one workspace of ns_workspace_bytes() bytes at ns_init;
 * the context borrows it and must not outlive it.  Work is enqueued on
 * cfg.stream (a hipStream_t; NULL = the null stream) and the calls return
 * without waiting, except ns_spectra and ns_spectra_wait, which wait for their
 * few-KB result, ns_budget_read and ns_timing_read.  A context is not thread safe; calls that
 * overlap on one context race.
 *
 * Errors: every call returns ns_status.  Arguments are checked on the host before
 * any HIP call.  Asynchronous device faults surface at a later call as
 * NS_ERR_HIP.  ns_last_error gives a message for the last failure on a context
 * (or, for ctx == NULL, for the last failure of a call without a context --
 * ns_init, ns_workspace_bytes, the 1D model -- on the calling thread).
 */
#ifndef NS_H_
#define NS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ns_ctx ns_ctx;

typedef enum {
  NS_OK = 0,
  NS_ERR_ARG = 1,       /* invalid argument (null/misaligned pointer, bad size or value) */
  NS_ERR_SIZE = 2,      /* workspace too small */
  NS_ERR_HIP = 3,       /* a HIP runtime call failed (possibly an earlier async fault) */
  NS_ERR_STATE = 4,     /* out of host memory at ns_init, or ns_spectra_wait with nothing in flight */
  NS_ERR_NONFINITE = 5  /* ns_spectra found a NaN or Inf in its input */
} ns_status;

typedef enum { NS_FP32 = 0, NS_FP64 = 1 } ns_precision;
/* Truncation masks (Sec. "Standard dealiasing with truncation", Figs. 1, 5 and 7):
 * SPHERE keeps |k| < C_t N/2, i.e. |k|^2 <= K2max (the largest integer below
 * (C_t N/2)^2); CUBE keeps every |k_i| < C_t N/2; NO_MULTIPLE_ALIASES keeps the
 * modes of the sphere with |k_i| + |k_j| < 2N/3 for every pair of axes, so that
 * no double (or triple) alias of a state held in it reaches a kept mode
 * (identical to SPHERE for C_t <= 2 sqrt(2)/3; Fig. 7b at C_t = 1); ROGALLO
 * applies the same pair rule to the cube: Rogallo's truncation, the cube less
 * thin prisms along its edges (Fig. 5). */
typedef enum {
  NS_MASK_SPHERE = 0,
  NS_MASK_CUBE = 1,
  NS_MASK_NO_MULTIPLE_ALIASES = 2,
  NS_MASK_ROGALLO = 3
} ns_mask;

/* Step variants of ns_step_rk2_phaseshift.  The phase-shift RK2 schemes of Sec.
 * "Extension to the multidimensional case" (0-2), the schemes without shifts they
 * are compared against (Sec. "Time advancement", Euler and midpoint RK2: 3, 4),
 * the Euler phase-shift scheme (Eq. sum_ps_non_ps in 3D: 5), and the fully exact
 * scheme averaging every evaluation over the eight shifts in {0, 1/2}^3, which
 * removes every alias class for any truncation (6; eight evaluations per stage). */
typedef enum {
  NS_PS_EXACT = 0,  /* midpoint RK2, every evaluation the average over shifts 0 and (1/2,1/2,1/2) */
  NS_PS_APPROX = 1, /* Heun/Rogallo with alpha = 0, beta = (1/2,1/2,1/2) */
  NS_PS_RANDOM = 2, /* Heun/Rogallo with alpha ~ U[0,1)^3 per step, beta = alpha + 1/2 (mod 1) */
  NS_RK2 = 3,       /* midpoint RK2 without shifts (truncation only) */
  NS_EULER = 4,     /* forward Euler in integrating-factor form, without shifts */
  NS_EULER_PS = 5,  /* Euler with the average over shifts 0 and (1/2,1/2,1/2) */
  NS_PS_EXACT8 = 6  /* midpoint RK2, every evaluation the average over the 8 shifts {0,1/2}^3 */
} ns_ps_variant;

typedef struct {
  int32_t n;          /* grid points per direction: 2^a 3^b 5^c, a >= 1, 8 <= n <= 1024 */
  int32_t precision;  /* ns_precision of every field */
  int32_t mask;       /* ns_mask */
  int32_t flags;      /* 0, or NS_CFG_GENERIC_PASSES */
  double nu;          /* kinematic viscosity, >= 0 */
  double ct;          /* truncation coefficient, 0 < ct <= 1 */
  uint64_t seed;      /* seed of the per-step random shifts (NS_PS_RANDOM, alphas == NULL) */
  void* stream;       /* hipStream_t on which all work is enqueued */
} ns_config;

/* Config flag: always use the size-generic passes (runtime radix plan) instead of
 * the compile-time specialised FP32 passes for N = 64, 128, 144, 160, 192, 216, 240,
 * 256, 270, 324, 360, 384, 512.  Results agree to FP32 round-off; meant for testing
 * and comparison. */
#define NS_CFG_GENERIC_PASSES 1

/* Forcing of the "split" phase-shift scheme (Eq. forcing-eq) and of the RK4
 * baseline: a divergence-free random field on the shell k2_lo <= |k|^2 <= k2_hi
 * (only 4..9 supported, the 96 modes of 2 <= |k| <= 3), redrawn every step from
 * SplitMix64(seed, step) and scaled so that the step injects energy at rate
 * `injection`: a sum w Re(conj(u0).g) + a^2 dt/2 sum w |g|^2 = injection, O = a g.
 * The Heun schemes add O to both stages (O0 = O1 = O), RK4 to all four slopes. */
typedef struct {
  int32_t k2_lo, k2_hi;  /* must be 4 and 9 */
  double injection;      /* energy injection rate, > 0 */
  uint64_t seed;
} ns_forcing;

/* Host-side outputs of ns_spectra; every pointer may be NULL (not written).
 * n_shell = ns_num_shells(n).  FP64 throughout. */
typedef struct {
  double* e_shell;  /* [n_shell] E(n) = 1/2 sum_{shell n} w |u|^2, shell: n(n-1) < |k|^2 <= n(n+1) */
  double* d_shell;  /* [n_shell] D(n) = nu sum_{shell n} w |k|^2 |u|^2 (dissipation spectrum) */
  double* t_shell;  /* [n_shell] T(n) = sum_{shell n} w Re(conj(u).N) (zero if n_hat is NULL) */
  double* e_1d;     /* [3][n/2+1] E_i(m) = 1/2 sum_{|k_i| = m} w |u|^2 */
  double* totals;   /* [5] E, eps = nu sum w |k|^2 |u|^2, H = 1/2 sum w Re(conj(u).omega), T, #nonfinite */
} ns_spectra_out;

/* Flags of ns_nonlinear. */
#define NS_NL_PS_AVG 1  /* return 1/2 [N(u; 0) + N(u; (1/2,1/2,1/2))] (Eq. sum_ps_non_ps, 3D shift); `shift` ignored */

/* Bytes of device workspace needed for cfg (0 if cfg is invalid). */
size_t ns_workspace_bytes(const ns_config* cfg);

/* Number of shells of the spectra for grid size n. */
int32_t ns_num_shells(int32_t n);

/* Largest retained |k|^2 (SPHERE, NO_MULTIPLE_ALIASES: of the sphere) or |k_i|
 * (CUBE, ROGALLO: of the cube) for cfg, -1 if cfg is invalid. */
int64_t ns_retained_bound(const ns_config* cfg);

/* Create a context on `workspace` (device memory, >= ns_workspace_bytes(cfg)
 * bytes, 256-byte aligned).  Builds FFT plans and uploads FP64-generated
 * twiddles; synchronous.  *out is set only on NS_OK. */
ns_status ns_init(const ns_config* cfg, void* workspace, size_t ws_bytes, ns_ctx** out);

/* Release a context (host memory only; the workspace stays the caller's). */
ns_status ns_destroy(ns_ctx* ctx);

const char* ns_last_error(const ns_ctx* ctx);

/* Change the stream later calls enqueue on.  The context's workspace (scratch
 * fields, stage buffers, tables, spectra partials, budget) is shared by every
 * call, so the caller must order the new stream after the work already enqueued
 * on the old one (an event recorded on the old stream and waited for on the new
 * one); otherwise a later call can overwrite buffers that earlier work still
 * reads. */
ns_status ns_set_stream(ns_ctx* ctx, void* stream);

/* One evaluation of the nonlinear term (Sec. "Aliasing description" for the
 * pseudo-spectral product, Eqs. shift_operator_3d and sum_ps_non_ps for the shift):
 *   n_hat = M conj(phi) P FFT( IFFT(phi M u_hat) x IFFT(i k x phi M u_hat) ),
 * phi = exp(2 pi i k.shift/N); shift NULL = unshifted.  u_hat and n_hat are
 * state-layout device arrays and must not overlap.  n_hat is fully written
 * (zero outside the retained set and at k = 0). */
ns_status ns_nonlinear(ns_ctx* ctx, const void* u_hat, void* n_hat, const double shift[3],
                       int32_t flags);

/* nsteps steps of classical RK4 in integrating-factor (Lawson) form, unshifted
 * (the 2/3-truncation baseline of Tables I-V when cfg.ct = 2/3), in place on the
 * state u_hat.  dt > 0, nsteps >= 0.  forcing (nullable): the large-scale forcing
 * of ns_forcing, drawn for step step0 + s from that step's start state exactly as
 * in ns_step_rk2_phaseshift, and added to the slope of every stage (N_i + O; the
 * forced runs of Table V force both schemes).  As for ns_step_rk2_phaseshift, the
 * intermediate states of one call stay in the workspace; nsteps steps in one call
 * are bit-identical to nsteps calls of one step. */
ns_status ns_step_rk4_trunc(ns_ctx* ctx, void* u_hat, double dt, int32_t nsteps, const ns_forcing* forcing,
                            int64_t step0);

/* nsteps steps of phase-shift RK2 (Eqs. Rogallo1981 and its 3D form; split
 * forcing of Eq. forcing-eq when forcing != NULL, Heun variants only), or of
 * one of the other ns_ps_variant schemes, in place on u_hat.  variant:
 * an ns_ps_variant value, NS_ERR_ARG outside 0..6.  alphas: host array [nsteps][3] of
 * first-stage shifts for NS_PS_RANDOM, or NULL to draw them as
 * alpha_i = SplitMix64 uniform (cfg.seed, step0 + s, i); ignored by the other
 * variants.  step0 keys the random draws (shifts and forcing) of the first step,
 * so that runs can be split and resumed exactly: nsteps steps in one call give
 * bit-identical results to nsteps calls of one step.  In one call every variant
 * keeps the intermediate states in the workspace (compact, aligned rows of the
 * retained planes), so steps after the first read, and steps before the last
 * write, less than a step of its own.
 *   exact:  S_h = E_{dt/2}(S0 + dt/2 A(S0)), S = E_dt S0 + dt E_{dt/2} A(S_h),
 *           A = 1/2 [N(.;0) + N(.;1/2)]
 *   heun:   S1 = E_dt(S0 + dt (N(S0;alpha) + O)),
 *           S = E_dt S0 + dt/2 E_{dt/2} (N(S0;alpha) + N(S1;beta) + 2 O)
 *   rk2:    the exact formula with A = N(.;0); exact8: with A the 8-shift average
 *   euler:  S = E_dt (S0 + dt A(S0)), A = N(.;0) or (euler_ps) the two-shift average
 * with E_tau = exp(-nu |k|^2 tau).
 * stage1 (nullable; Heun variants with nsteps == 1): a state-layout device array,
 * distinct from u_hat, that receives the step's first-stage state S1 on the
 * retained modes (other entries are not written), for ns_vjp_rk2_phaseshift; the
 * result in u_hat is the same bit for bit. */
ns_status ns_step_rk2_phaseshift(ns_ctx* ctx, void* u_hat, double dt, int32_t nsteps,
                                 int32_t variant, const double* alphas,
                                 const ns_forcing* forcing, int64_t step0, void* stage1);

/* FP64 spectra and totals of the state u_hat (and the transfer with n_hat when
 * non-NULL), Sec. "3D flow: Taylor-Green vortices".  Every bin is summed in a
 * fixed order, so the result is reproducible bit for bit.  Waits for the result.
 * Returns NS_ERR_NONFINITE (outputs still written) if any entry of u_hat or
 * n_hat is NaN or Inf. */
ns_status ns_spectra(ns_ctx* ctx, const void* u_hat, const void* n_hat, ns_spectra_out* out);

/* For callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the spectra of ns_spectra without a
 * context and without any allocation, device or host.  The FP64 partials and bins
 * live in a file-scope device array of the library, about 4.3 MB on each GPU it
 * runs on (held until the process ends; its address is looked up once per device,
 * at the first call on that device).  n: 2^a 3^b 5^c, 8 <= n <= NS_SPECTRA_STATIC_MAX_N
 * (NS_ERR_SIZE above it); precision: ns_precision of u_hat and n_hat (state
 * layout, 256-byte aligned device pointers; n_hat may be NULL); nu >= 0 for the
 * dissipation.  Enqueued on `stream` and waited for; outputs and errors as
 * ns_spectra, with the same bit-for-bit results.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other host threads, other streams)
 * race. */
#define NS_SPECTRA_STATIC_MAX_N 512
ns_status ns_spectra_static(int32_t n, int32_t precision, double nu, const void* u_hat, const void* n_hat,
                            void* stream, ns_spectra_out* out);

/* The same in two halves, so that a time loop keeps the GPU busy while the host
 * waits: ns_spectra_async enqueues the reduction of u_hat (and n_hat) as they are
 * at that point of the stream, with its copy into pinned host memory the library
 * allocates on first use; ns_spectra_wait waits for that reduction only (not for
 * work enqueued after it) and fills out like ns_spectra.  One reduction is in
 * flight per context: a later ns_spectra_async or ns_spectra replaces one not yet
 * waited for.  ns_spectra_wait with nothing in flight returns NS_ERR_STATE. */
ns_status ns_spectra_async(ns_ctx* ctx, const void* u_hat, const void* n_hat);
ns_status ns_spectra_wait(ns_ctx* ctx, ns_spectra_out* out);

/* Transpose of the linearised phase-shift RK2 step at state u_hat0:
 * lam holds dJ/dS_{n+1} on entry and dJ/dS_n on return, both with respect to the
 * Parseval inner product <a,b> = sum_k w Re(conj(a).b) (w = 1 on the k_z = 0 and
 * N/2 planes, 2 elsewhere); multiply by w for the gradient of the real and
 * imaginary parts taken as independent variables.  alpha: the first-stage shift
 * used by the forward step (NS_PS_RANDOM; NULL for the other variants).
 * forcing (nullable; Heun variants): the forward step was forced (Eq. forcing-eq)
 * with the draw of step `step`; it is redrawn from u_hat0, and the adjoint also
 * carries the dependence of the forcing amplitude on u_hat0 (a B + a^2 dt/2 G =
 * injection with B = <u_hat0, g>, so da/dB = -a / sqrt(B^2 + 2 dt G injection)).
 * stage1 (nullable; Heun variants): the first-stage state S1 of the forward step,
 * as ns_step_rk2_phaseshift kept it; the adjoint then uses it instead of
 * evaluating it again (one nonlinear-term evaluation less), with the same result
 * bit for bit. */
ns_status ns_vjp_rk2_phaseshift(ns_ctx* ctx, const void* u_hat0, void* lam, double dt,
                                int32_t variant, const double alpha[3], const ns_forcing* forcing,
                                int64_t step, const void* stage1);

/* FP64 time-integrated energy budget on the GPU (Sec. "3D flow: Taylor-Green
 * vortices": dE/dt = -eps for the free flow; Sec. "Numerical methods": the forced
 * runs inject energy at a given rate).  ns_budget_start enqueues a reduction of
 * E = 1/2 sum w |u|^2 and eps = nu sum w |k|^2 |u|^2 over the retained modes of
 * u_hat and starts the record there; while the budget is on, every step of
 * ns_step_rk4_trunc and ns_step_rk2_phaseshift enqueues the same reduction of the
 * state after it (summed in a fixed order, so reproducible bit for bit) and
 * updates the record on the device: t += dt, int eps dt by the trapezoid rule
 * step by step, int P dt += the energy the step's forcing injects,
 * dt (a B + a^2 dt/2 G) = E(u0 + dt O) - E(u0).  ns_budget_read waits for the
 * stream and writes NS_BUDGET_LEN doubles: t, E, eps, E0, int eps dt, int P dt,
 * P of the last step (0 if unforced), and the residual
 * E - E0 + int eps dt - int P dt.  ns_budget_stop ends the per-step updates (the
 * record is kept).  The reductions read the state once per step (3 retained
 * components), a few percent of a step's traffic. */
#define NS_BUDGET_LEN 8
ns_status ns_budget_start(ns_ctx* ctx, const void* u_hat);
ns_status ns_budget_stop(ns_ctx* ctx);
ns_status ns_budget_read(ns_ctx* ctx, double* out);

/* Per-pass timing, the GPU counterpart of the per-task time shares of the
 * paper's profiles (Figs. 10 and 14).  While enabled, every launch of the five
 * passes of a nonlinear-term evaluation is bracketed by HIP events recorded on
 * the context's stream (this adds a little overhead per launch).  Passes:
 * 0 x-inverse (shift, curl), 1 y-inverse, 2 fused z (c2r, u x omega, r2c),
 * 3 y-forward, 4 x-forward (projection, mask, Runge-Kutta stage), 5 x-forward
 * that also runs the next evaluation's x-inverse pass on the stage output it
 * computes (the step sequences chain their evaluations this way with the
 * specialised FP32 passes).
 * ns_timing_read waits for the stream, writes per pass the summed event-to-event
 * milliseconds and the number of launches since the previous read (host arrays
 * of NS_NUM_PASSES entries; either may be NULL) and clears the record. */
#define NS_NUM_PASSES 6
ns_status ns_timing_enable(ns_ctx* ctx, int32_t enable);
ns_status ns_timing_read(ns_ctx* ctx, double* ms, int64_t* launches);

/* ---- The 1D model dS/dt = -S^2 (Sec. "Phase shifting for one-dimensional
 * problems", Eqs. model-1d-2 and 1d_initial; the scheme comparison of Fig. 8).
 * A batch of independent real signals of n points on [0, 2 pi), each held as its
 * spectrum s_hat[b][k], k = 0..n/2 (FP64 complex, interleaved re/im, rows of
 * n/2 + 1 entries; forward transform normalised by 1/n, inverse unnormalised).
 * Truncation keeps k < ct n/2 (the strict reading of the 3D masks), in and out;
 * there is no viscosity, so no integrating factor.  N(S; s) is the product
 * evaluated on the grid shifted by s cells and shifted back:
 *   N(S; s)_k = M_k conj(phi_k) FFT(-(IFFT(phi M S))^2)_k,  phi_k = exp(2 pi i k s / n).
 * Device pointers, 16-byte aligned (may be NULL when batch is 0), owned by the
 * caller; work is enqueued on
 * `stream` (a hipStream_t, NULL for the default stream) and not waited for.
 * Host checks (NS_ERR_ARG, message from ns_last_error(NULL)): n even with
 * 4 <= n <= 1024, 0 < ct <= 1 with at least one mode k >= 1 kept, batch >= 0.
 * Launch failures return NS_ERR_HIP. */
typedef enum {
  NS1D_EULER = 0,     /* S = S0 + dt N(S0; 0) */
  NS1D_EULER_PS = 1,  /* S = S0 + dt A(S0), A = 1/2 [N(.; 0) + N(.; 1/2)] (Eq. sum_ps_non_ps) */
  NS1D_RK2 = 2,       /* midpoint: S_h = S0 + dt/2 N(S0; 0), S = S0 + dt N(S_h; 0) */
  NS1D_PS_EXACT = 3,  /* the midpoint formula with A in place of N at both stages */
  NS1D_PS_APPROX = 4, /* Heun: S1 = S0 + dt N(S0; 0), S = S0 + dt/2 [N(S0; 0) + N(S1; 1/2)] (Eq. Rogallo1981) */
  NS1D_RK4 = 5        /* classical four-stage Runge-Kutta, unshifted */
} ns1d_scheme;

/* n_hat[b] = N(s_hat[b]; shift) for every signal (n_hat may alias s_hat). */
ns_status ns1d_nonlinear(const void* s_hat, void* n_hat, int32_t n, double ct, int32_t batch,
                         double shift, void* stream);

/* nsteps steps of an ns1d_scheme value on every signal, in place; one block per
 * signal keeps all stages on chip.  Also NS_ERR_ARG for dt not finite and > 0,
 * nsteps < 0 or an unknown scheme. */
ns_status ns1d_step(void* s_hat, int32_t n, double ct, int32_t batch, double dt, int32_t nsteps,
                    int32_t scheme, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NS_H_ */
