/*
 * fdemri.h -- C ABI of the frequency-domain EMRI mode-summation library
 * (MI355X / gfx950, HIP).
 *
 * The library evaluates the frequency-domain waveform of Speri et al., "Fast
 * and Fourier: Extreme Mass Ratio Inspiral Waveforms in the Frequency
 * Domain" (arXiv 2307.12585), Sec. 2.2: for every harmonic voice (l,m,n) of
 * Eq. main_wave it inverts the voice frequency F(t) = (m Omega_phi +
 * n Omega_r)/(2 pi M) on each cubic-spline segment of the sparse trajectory
 * (Eq. cubic_equation), evaluates the third-order stationary-phase term of
 * Eq. extendedspa1 at every root, and sums all voices into h_+(f) and
 * h_x(f) on an arbitrary ascending frequency array.
 *
 * Conventions
 *  - Every array argument is a DEVICE pointer (memory of the context's HIP
 *    device), unless stated otherwise.  The caller allocates and owns every
 *    input and output; the library keeps no caller pointer after a call
 *    returns.  Scratch memory is owned by the context.
 *  - Calls are asynchronous on the given stream: once argument validation
 *    passes, all work is enqueued on `stream` and the call returns.  On
 *    FDEMRI_EINVAL nothing is enqueued and outputs are untouched.
 *  - Every function returns a status code and never throws.  The text of the
 *    last error is per context (fdemri_last_error).
 *  - Device-side conditions that the host cannot see without a
 *    synchronisation (more monotonic pieces in one voice than the table
 *    holds, mode rows outside the supported range) are recorded in a
 *    per-context flag word; fdemri_sync_flags synchronises the stream,
 *    returns the word and clears it.
 *  - One context per host thread (contexts are not internally locked).  All
 *    calls on one context use its workspace: issue them on one stream, or
 *    order their streams (events); calls on a context that overlap in time on
 *    different streams race on its scratch tables and give wrong results.
 *  - Transform convention of Eq. singlevoiceFT: h(f) = int h(t) e^{+2 pi i f t} dt,
 *    with h = h_+ - i h_x (Eq. main_wave).
 */
#ifndef FDEMRI_H
#define FDEMRI_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdemri_ctx fdemri_ctx;

typedef enum {
  FDEMRI_OK = 0,
  FDEMRI_EINVAL = 1,   /* invalid argument; nothing enqueued */
  FDEMRI_ENOMEM = 2,   /* device allocation failed */
  FDEMRI_EDEVICE = 3,  /* HIP runtime error */
  FDEMRI_ENOTSUP = 4   /* valid but unsupported request (e.g. K above the limit) */
} fdemri_status;

typedef enum {
  FDEMRI_FP64 = 0,     /* everything in FP64; output complex128 (2 x double per bin) */
  FDEMRI_MIXED = 1,    /* FP64 root, phase and range reduction; FP32 special function,
                          sincos and amplitude spline, contributions summed in FP64;
                          output complex64 (2 x float per bin) */
  /* range markers, not precisions: the enumeration spans int32, so that any
     value a caller passes is a value of the type; every entry point rejects
     values other than the two above with FDEMRI_EINVAL */
  FDEMRI_PREC_RANGE_LO_ = -2147483647 - 1,
  FDEMRI_PREC_RANGE_HI_ = 2147483647
} fdemri_prec;

/* flags of fdemri_waveform_desc.flags */
#define FDEMRI_NO_PARTNERS 0x1u  /* treat every row as a single voice (l,m,n) with any
                                    sign of m; do not add the (l,-m,-n) partner */
#define FDEMRI_COEFFS_GIVEN 0x2u /* A holds the amplitude spline coefficients of every
                                    segment instead of knot values (layout below); they
                                    are used as given, without a spline solve */

/* Flag bits reported by fdemri_sync_flags */
#define FDEMRI_FLAG_PIECE_OVERFLOW 0x1u  /* a voice had more monotonic pieces than
                                            FDEMRI_MAX_PIECES; extra pieces dropped */
#define FDEMRI_FLAG_BAD_MODE 0x2u        /* a row had l outside [2, FDEMRI_MAX_L], |m| > l,
                                            or m < 0 without FDEMRI_NO_PARTNERS; such rows
                                            contribute nothing */
#define FDEMRI_FLAG_TRAJ_STEPS 0x4u      /* fdemri_trajectory: a waveform needed more than
                                            the step bound of its integrator; its knots
                                            past that point repeat the last state */
#define FDEMRI_FLAG_BAD_INPUT 0x8u       /* a waveform's device data failed the input checks
                                            (t not finite or not strictly increasing; a
                                            trajectory or amplitude value not finite; f not
                                            finite, negative or descending; FDEMRI_LL_HANN on
                                            a grid other than f_k = k f_1): its outputs are
                                            zeros (waveform, adjoint; the likelihood of a
                                            zero model) */
#define FDEMRI_MAX_PIECES 16
#define FDEMRI_MAX_KNOTS 512
#define FDEMRI_MAX_L 40

/*
 * One waveform (Sec. 2.1-2.2).  Sparse trajectory knots (Sec. 2.1: the
 * adiabatic trajectory is ~100 points), the complex amplitude knot values of
 * each (l,m,n) voice (Sec. 2.1: amplitudes interpolated with not-a-knot cubic
 * splines), the source-frame viewing angles and mu/d_L of Eq. main_wave, and
 * the frequency array (Eq. innerprod grid f_i = i/T, or any ascending grid,
 * Sec. 3.3).
 *
 * Layouts (all device pointers, read only):
 *   t, Fphi, Fr, Phiphi, Phir : [K] double.  t strictly increasing (s);
 *       Fphi = Omega_phi/(2 pi M), Fr = Omega_r/(2 pi M) in Hz; Phiphi,
 *       Phir in rad including the initial phases.
 *   l, m, n : [Nm] int32 mode numbers.  Without FDEMRI_NO_PARTNERS,
 *       2 <= l <= FDEMRI_MAX_L and 0 <= m <= l; each row with m > 0 stands for
 *       the voices (l,m,n) and (l,-m,-n), the latter with amplitude
 *       (-1)^l conj(A) (the equatorial-symmetry relation of the Schwarzschild
 *       amplitudes); m = 0 rows are single voices.
 *   A : [Nm][K][2] double, complex amplitude knot values (re, im); with
 *       FDEMRI_COEFFS_GIVEN instead [Nm][K-1][4][2] double, the coefficients
 *       a_k of A(t_i + tau) = sum_k a_k tau^k on segment i (ascending k, re, im).
 *   f : [Nf] double, ascending, f >= 0 (Hz).  Bins with f == 0 are set to 0.
 * Host scalars: theta, phi (source-frame polar/azimuthal viewing angles),
 *   scale = mu/d_L (dimensionless strain scale of Eq. main_wave).
 * Limits: 4 <= K <= FDEMRI_MAX_KNOTS, 1 <= Nm, 1 <= Nf < 2^31.
 * Data-dependent conditions are checked on the device, since the host does
 * not read device data (the device-side form of FDEMRI_EINVAL): t finite and
 * strictly increasing; Fphi, Fr, Phiphi, Phir and A finite; f finite, >= 0
 * and ascending.  A waveform that fails them gets zero outputs and raises
 * FDEMRI_FLAG_BAD_INPUT (fdemri_sync_flags); the kernels stay in bounds.
 * (fdemri_td_waveform and fdemri_signal_band raise the flag too; their
 * outputs are then unspecified.)
 */
typedef struct {
  int32_t K;
  const double *t, *Fphi, *Fr, *Phiphi, *Phir;
  int32_t Nm;
  const int32_t *l, *m, *n;
  const double *A;
  double theta, phi, scale;
  int32_t Nf;
  const double *f;
  uint32_t flags;
} fdemri_waveform_desc;

/* Context flags */
#define FDEMRI_CTX_BATCH_GRAPHS 0x1u  /* capture each distinct batch (same descriptors,
                                         pointers and precision) into a hipGraph on first
                                         use and replay it on later calls */

/* Create a context on HIP device `hip_device` (0-based) with FDEMRI_CTX_* flags.
 * On success *out receives the context.  Test hook: with the environment
 * variable FDEMRI_TEST_FAIL_ALLOC=n (n >= 1) set at creation, the n-th growth
 * of the context's workspace fails as a failed device allocation would
 * (FDEMRI_ENOMEM, nothing enqueued, outputs untouched, the context usable). */
fdemri_status fdemri_create(fdemri_ctx **out, int hip_device, uint32_t flags);

/* Release the context and its scratch memory (synchronises the device). */
void fdemri_destroy(fdemri_ctx *ctx);

/* Text of the last error on this context ("" if none).  Owned by the context. */
const char *fdemri_last_error(const fdemri_ctx *ctx);

/* Synchronise `stream` and return (and clear) the device flag word. */
fdemri_status fdemri_sync_flags(fdemri_ctx *ctx, hipStream_t stream, uint32_t *flags_out);

/*
 * Frequency-domain waveform h_+(f), h_x(f) (Sec. 2.2, Eqs. cubic_equation,
 * SPAintegral2, extendedspa1; polarizations from Eq. main_wave).
 * hp, hc : [Nf] complex outputs (interleaved re, im) of the precision's type
 * (double for FDEMRI_FP64, float for FDEMRI_MIXED).  Fully overwritten.
 * Returns FDEMRI_OK once the work is enqueued on `stream`.
 * The call enqueues kernel launches only (no copies, no memsets), so a
 * caller may capture it into a HIP graph after one eager call of the same
 * shape and precision on the same context (that call sizes the context's
 * workspace).  The graph reads the inputs and the workspace at replay; a
 * later call on the context that needs a larger workspace reallocates it and
 * invalidates such graphs, so other work should use its own context.  (The
 * old workspace is released once the work enqueued before that call has
 * completed, without synchronising the device.)
 */
fdemri_status fdemri_waveform(fdemri_ctx *ctx, const fdemri_waveform_desc *desc,
                              fdemri_prec prec, void *hp, void *hc, hipStream_t stream);

/*
 * fdemri_waveform without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results as
 * fdemri_waveform (bit for bit), but the scratch tables (spline
 * coefficients, piece tables, mode constants) live in a fixed device array
 * of FDEMRI_NOALLOC_SCRATCH_BYTES that the library holds on every device it
 * runs on until the process ends; the call makes no hipMalloc, hipFree or
 * other allocating call and leaves the context's own workspace alone.
 * Scratch needed: about 64 B per mode and spline segment (FP64; 96 B mixed)
 * plus 1.6 KB per mode, i.e. up to 3843 modes at K = 200 in either
 * precision; larger requests return FDEMRI_ENOTSUP with nothing enqueued.
 * Every call on one device shares that device's array, and each call
 * rewrites whatever it reads: calls that overlap in time on one device (two
 * streams, two contexts, two host threads) race and give wrong results;
 * serialise them (one stream, or events).  Kernel profiling
 * (fdemri_profile_enable) does not bracket these launches.
 */
#define FDEMRI_NOALLOC_SCRATCH_BYTES (96u << 20)
fdemri_status fdemri_waveform_noalloc(fdemri_ctx *ctx, const fdemri_waveform_desc *desc,
                                      fdemri_prec prec, void *hp, void *hc, hipStream_t stream);

/*
 * Several waveforms in one persistent launch (Sec. 3.2 timing studies
 * evaluate many parameter draws; the batch amortises launches).
 * descs : HOST array of B descriptors (device pointers inside).
 * hp, hc : HOST arrays of B device output pointers.
 * Results equal B calls of fdemri_waveform with the same precision, bit for
 * bit.  With FDEMRI_CTX_BATCH_GRAPHS the whole sequence (record upload,
 * batched preparation kernels, persistent gather) is captured once per
 * distinct batch and replayed; the caller must keep the input contents it
 * wants evaluated in the same buffers (the graph reads them at replay).
 */
fdemri_status fdemri_waveform_batch(fdemri_ctx *ctx, int32_t B, const fdemri_waveform_desc *descs,
                                    fdemri_prec prec, void *const *hp, void *const *hc,
                                    hipStream_t stream);

/*
 * Vector-Jacobian product of the waveform: the gradient of a real loss L of
 * h_+ and h_x, such as the Whittle log-likelihood of Eq. likelihood, with
 * respect to the amplitude and phase splines, the viewing angles, the scale
 * and the initial phases.  The forward terms of Eq. extendedspa1 are
 * recomputed (not stored); the frequency splines, and hence the root times
 * t(f) of Eq. cubic_equation, are held fixed.
 * g_hp, g_hc : [Nf] complex cotangents dL/dRe h + i dL/dIm h, interleaved,
 *   of the precision's type (double for FDEMRI_FP64, float for FDEMRI_MIXED).
 * Outputs (device, fully overwritten; each may be NULL to skip):
 *   gA        : [Nm][K-1][4][2] double, dL/d(amplitude spline coefficients)
 *               a_k of A(t_i + tau) = sum_k a_k tau^k, same complex convention.
 *   gPhi      : [2][K-1][4] double, dL/d(Phi_phi and Phi_r spline coefficients),
 *               ascending powers of tau.
 *   gA_knots  : [Nm][K][2] double, dL/d(amplitude knot values A of the desc),
 *               through the transposed not-a-knot spline (must be NULL with
 *               FDEMRI_COEFFS_GIVEN: the amplitudes then have no knots;
 *               FDEMRI_EINVAL otherwise).
 *   gPhi_knots: [2][K] double, dL/d(Phi_phi and Phi_r knot values).
 *   g_scalars : [5] double: dL/dtheta, dL/dphi, dL/dscale, dL/dPhi_phi0,
 *               dL/dPhi_r0 (the last two: a common offset of all Phi knots).
 * The result is deterministic: the bins are cut into chunks that the waves
 * take from a device counter, which decides only which wave evaluates a
 * chunk; every sum runs in a fixed order.  The context's workspace grows to
 * hold the chunk plan: about 370 B per (row, segment) plus 120 MB.
 */
fdemri_status fdemri_vjp(fdemri_ctx *ctx, const fdemri_waveform_desc *desc, fdemri_prec prec,
                         const void *g_hp, const void *g_hc, double *gA, double *gPhi,
                         double *gA_knots, double *gPhi_knots, double *g_scalars,
                         hipStream_t stream);

/* flags of fdemri_loglike */
#define FDEMRI_LL_HANN 0x1u  /* compare the data with the model convolved with the
                                3-tap Hann kernel h_w(f_k) = h(f_k)/2 - h(f_{k+1})/4
                                - h(f_{k-1})/4 (the frequency-domain form of a Hann
                                window on the DFT grid; h = 0 past the last bin and
                                h(f_{-1}) = conj h(f_1) before the first).  Only on
                                a grid f_k = k f_1 (f_0 = 0, uniform to 1e-12), the
                                grid on which it is the transform of the windowed
                                series; other grids raise FDEMRI_FLAG_BAD_INPUT.
                                Past the last bin the model is taken as 0 also when
                                that bin is the Nyquist bin (whose neighbour would
                                be the conjugate reflection): the signal band is
                                expected to end below Nyquist */

/*
 * Whittle log-likelihood of data against the waveform of `desc` (Eq. likelihood
 * with the inner product of Eq. innerprod), with the mode sum fused: the
 * model is reduced bin by bin where it is formed and never written to memory.
 *   d_p, d_c : [Nf] complex data per channel (interleaved re, im) of the
 *              precision's type (double for FDEMRI_FP64, float for FDEMRI_MIXED).
 *   wS       : [Nf] double, the weight of each bin in the inner product,
 *              4 w_k / S_n(f_k) with w_k the quadrature weight of the grid
 *              (1/T on the DFT grid); 0 excludes a bin (the DC bin, f = 0,
 *              is outside the sum of Eq. innerprod).
 *   ll_flags : FDEMRI_LL_* flags.
 *   out      : [3] double, DEVICE: out[0] = log L = -1/2 sum_{+,x} sum_k wS_k
 *              |d_k - h_k|^2, out[1] = sum wS |h|^2 (<h|h> summed over the two
 *              channels), out[2] = sum wS Re(conj(d) h) (<d|h>), with h the
 *              (windowed) model; on the mixed path the model is rounded to FP32
 *              first, as fdemri_waveform would store it, and the sums are FP64.
 * The result is deterministic (fixed reduction order, no atomics).  Errors as
 * fdemri_waveform; FDEMRI_EINVAL for NULL data, weights or output.
 */
fdemri_status fdemri_loglike(fdemri_ctx *ctx, const fdemri_waveform_desc *desc, fdemri_prec prec,
                             const void *d_p, const void *d_c, const double *wS, uint32_t ll_flags,
                             double *out, hipStream_t stream);

/*
 * fdemri_loglike for B waveforms in one persistent launch (the batch path of
 * fdemri_waveform_batch with the model reduced where it is formed, so that
 * no waveform of the batch is written to memory).
 *   descs          : HOST array of B descriptors.
 *   d_p, d_c, wS   : HOST arrays of B device pointers (data and weights per
 *                    waveform, as for fdemri_loglike).
 *   out            : [B][3] double, DEVICE.
 * Each out[b] equals fdemri_loglike of waveform b with the same precision and
 * flags, bit for bit.  Not captured into graphs (enqueued eagerly).
 */
fdemri_status fdemri_loglike_batch(fdemri_ctx *ctx, int32_t B, const fdemri_waveform_desc *descs,
                                   fdemri_prec prec, const void *const *d_p, const void *const *d_c,
                                   const double *const *wS, uint32_t ll_flags, double *out,
                                   hipStream_t stream);

/*
 * Time-domain waveform on a uniform grid, the comparison model of the
 * paper's FD/TD study (Sec. 3.2): h(t) = sum over voices of H_V(t)
 * e^{-i Phi_V(t)} (Eq. wave_voice) from the same splines, angles and partner
 * convention as fdemri_waveform, with h_+ = Re h and h_x = -Im h
 * (Eq. main_wave; h = h_+ - i h_x).
 *   t0, dt, Nt : samples t_k = t0 + k dt (k*dt rounded, then added), k < Nt;
 *                dt > 0, Nt >= 0.
 *   hp_t, hc_t : [Nt] double, DEVICE, h_+(t_k) and h_x(t_k); 0 for samples
 *                outside [t_0, t_{K-1}] of the trajectory.  Fully overwritten.
 * The frequency array of desc is validated but not used.  The transform of
 * the result with the sign of Eq. singlevoiceFT, x~(f_k) = dt conj(rfft(x))[k]
 * for real x, is what the FD sum approximates.
 */
fdemri_status fdemri_td_waveform(fdemri_ctx *ctx, const fdemri_waveform_desc *desc, double t0, double dt,
                                 int32_t Nt, double *hp_t, double *hc_t, hipStream_t stream);

/*
 * Sparse trajectories on the device (Sec. 2.1: the adiabatic orbit is
 * integrated to ~100 points before the mode sum), for the toy orbit-averaged
 * fluxes of the synthetic workloads, one waveform per thread:
 *   dp/dt = -(64/5) q (1-e^2)^{3/2} p^-3 (1 + 7e^2/8) / M_s,
 *   de/dt = -(304/15) q e (1-e^2)^{3/2} p^-4 (1 + 121e^2/304) / M_s,
 *   dPhi_phi/dt = Omega_phi / M_s, dPhi_r/dt = Omega_r / M_s,
 *   Omega_phi = p^{-3/2} (1-e^2)^{3/2}, Omega_r = Omega_phi sqrt(1 - 6/p),
 * q = mu/M, M_s = M G M_sun / c^3, from t = 0 to T or to the plunge
 * p = 6 + 2e + 0.1; K knots uniform in [0, t_end].  Dormand-Prince 5(4)
 * with relative tolerance 1e-12 (absolute 1e-12, 1e-14, 1e-9, 1e-9 for p, e
 * and the two phases).
 *   params : HOST array of B fdemri_traj_params (M in solar masses, mu in
 *            solar masses, T in s, phases in rad); M, mu, T > 0,
 *            0 <= e0 < 1, p0 > 6 + 2 e0 + 0.1.
 *   out    : [B][7][K] double, DEVICE: per waveform the rows t, F_phi, F_r
 *            (Hz), Phi_phi, Phi_r (rad), p, e - the first five are the
 *            trajectory fields of fdemri_waveform_desc.
 * 4 <= K <= FDEMRI_MAX_KNOTS.  FDEMRI_FLAG_TRAJ_STEPS (fdemri_sync_flags)
 * reports a waveform that reached the integrator's step bound.
 */
typedef struct {
  double M, mu, p0, e0, T, Phiphi0, Phir0;
} fdemri_traj_params;
fdemri_status fdemri_trajectory(fdemri_ctx *ctx, int32_t B, const fdemri_traj_params *params, int32_t K,
                                double *out, hipStream_t stream);

/*
 * Frequency band occupied by the waveform of `desc` (Sec. 3.3: a downsampled
 * grid spans only [0, f_max] of the signal): band[0], band[1] (DEVICE
 * doubles) = the smallest and largest |F_V| at the ends of the monotonic
 * pieces of all voices (0, 0 without voices).  The frequency array of desc
 * is validated but not used.
 */
fdemri_status fdemri_signal_band(fdemri_ctx *ctx, const fdemri_waveform_desc *desc, double *band,
                                 hipStream_t stream);

/*
 * Mode selection by power (Sec. 2.1: modes are kept by their share of the
 * total power; the share is taken at every knot and the union kept):
 * row mu of A is kept when |A_mu(t_i)|^2 > eps * sum_nu |A_nu(t_i)|^2 at one
 * knot i at least, |A|^2 = re*re + im*im rounded term by term.
 *   A      : [Nm][K][2] double, DEVICE, complex amplitude knot values (the
 *            layout of fdemri_waveform_desc.A).
 *   eps    : threshold, finite and >= 0.
 *   idx    : [Nm] int32, DEVICE: the kept rows, in table order, in
 *            idx[0 .. *n_keep); the rest is left as it was.
 *   n_keep : int32, DEVICE.
 * 1 <= K, 0 <= Nm.  Deterministic (fixed summation order).  FDEMRI_EINVAL for
 * invalid sizes, eps or NULL pointers (nothing enqueued).
 */
fdemri_status fdemri_select_modes(fdemri_ctx *ctx, int32_t K, int32_t Nm, const double *A, double eps,
                                  int32_t *idx, int32_t *n_keep, hipStream_t stream);

/*
 * Autotuner of the gather's block shape (1, 2 or 4 consecutive 64-bin tiles
 * per wavefront, i.e. 256, 512 or 1024 contiguous bins per 4-wave workgroup
 * sharing one active-mode list; the result does not depend on the choice,
 * only the time does).  Runs the given batch (B = 1:
 * a single waveform) once per candidate, timed with HIP events on `stream`,
 * keeps the fastest for this precision and workload class (log2 of the
 * total bin count; single or batch) on the context, and, if the environment
 * variable FDEMRI_TUNE_CACHE names a file, appends the choice there
 * (keyed by device name and architecture; read back by fdemri_create).
 * Outputs hp/hc are overwritten.  *bpl_out (host) receives the choice.
 */
fdemri_status fdemri_autotune(fdemri_ctx *ctx, int32_t B, const fdemri_waveform_desc *descs,
                              fdemri_prec prec, void *const *hp, void *const *hc,
                              hipStream_t stream, int32_t *bpl_out);

/*
 * The per-root factor of Eq. extendedspa1,
 *   G = |Fd|^{-1/2} e^{-i pi/4 sgn Fd} W(X),  X = 2 pi Fd^3 / (3 Fdd^2),
 * W(X) = sqrt(2|X|/pi) e^{-i pi/4 sgn X} e^{-iX} K_{1/3}(-iX) (the printed
 * constant taken with the opposite sign, the reading under which the factor
 * reduces to the standard stationary-phase one as Fdd -> 0), for n pairs
 * (Fd, Fdd) = (dF/dt, d2F/dt2) at a root, evaluated by the device code of the
 * mode sum.  As there, the length of the large-argument series is chosen per
 * 64 consecutive elements (one wavefront) from the largest |1/X| among them.
 *   gd, gdd : [n] double, DEVICE; dir : [n] int32, DEVICE, the direction (+1 or
 *             -1) of the monotonic piece, used only where Fd == 0 (then
 *             G = pi (pi |Fdd|)^{-1/3} [Ai(0) - i dir Bi(0)]).
 *   G       : [n] complex (interleaved re, im) of the precision's type.
 * Fdd == 0 gives the standard factor (W = 1); Fd == Fdd == 0 gives 0.
 * FDEMRI_EINVAL for n < 0 or NULL pointers (nothing enqueued).
 */
fdemri_status fdemri_spa_factor(fdemri_ctx *ctx, fdemri_prec prec, int32_t n, const double *gd,
                                const double *gdd, const int32_t *dir, void *G, hipStream_t stream);

/*
 * Count of mode-bin evaluations of the last fdemri_waveform call on this
 * context: the number of (monotonic piece of |F_V|, bin) pairs with the bin
 * inside the piece's frequency range.  Synchronises `stream`.
 */
fdemri_status fdemri_last_eval_count(fdemri_ctx *ctx, hipStream_t stream, int64_t *count_out);

/*
 * Count of the evaluations of the last fdemri_waveform (or batch) call whose
 * root was solved.  Rows with the same (m, n) have the same voice frequency
 * m Omega_phi + n Omega_r (Eq. main_wave), hence the same pieces, roots
 * (Eq. cubic_equation) and per-root factors of Eq. extendedspa1 up to the
 * amplitude A_lmn and the harmonics; a table of more than 256 and at most
 * 4096 rows is evaluated by voice groups of such rows, each (piece of a
 * group, bin) pair once, and this counts those pairs.  Equals
 * fdemri_last_eval_count when the rows were not grouped.  Synchronises
 * `stream`.
 */
fdemri_status fdemri_last_group_eval_count(fdemri_ctx *ctx, hipStream_t stream, int64_t *count_out);

/*
 * Per-kernel timing for measurement.  While enabled, every kernel launch of
 * this context is bracketed by HIP events recorded on its launch stream.
 * fdemri_profile_read synchronises `stream`, returns the accumulated
 * milliseconds and launch counts per kernel class (FDEMRI_KERNEL_*; arrays of
 * FDEMRI_KERNEL_COUNT entries, host memory) and resets the accumulators.
 */
#define FDEMRI_KERNEL_SPLINE 0  /* the trajectory splines (none when the set-up is fused) */
#define FDEMRI_KERNEL_PIECES 1  /* the set-up: piece tables, amplitude splines, input checks;
                                   for at most 256 modes and 256 knots one fused launch that
                                   also solves the trajectory splines */
#define FDEMRI_KERNEL_GATHER 2
#define FDEMRI_KERNEL_VJP 3      /* the adjoint's per-(mode, segment) kernel (its reductions
                                    and the transposed spline are not bracketed) */
#define FDEMRI_KERNEL_COUNT 4
fdemri_status fdemri_profile_enable(fdemri_ctx *ctx, int enable);
fdemri_status fdemri_profile_read(fdemri_ctx *ctx, hipStream_t stream, double *ms_out, int64_t *launches_out);
/*
 * The kernel classes bracketed while profiling is enabled: bit FDEMRI_KERNEL_x
 * of class_mask (all classes after fdemri_create).  Each bracket is an event
 * pair on the launch stream between consecutive kernels, so a measurement
 * that needs one kernel's duration should record that class only.  Bits at
 * or above FDEMRI_KERNEL_COUNT: FDEMRI_EINVAL, mask unchanged.
 */
fdemri_status fdemri_profile_classes(fdemri_ctx *ctx, uint32_t class_mask);

#ifdef __cplusplus
}
#endif

#endif /* FDEMRI_H */
