/*
 * recon.h -- C ABI of the MI355X (gfx950) iterative Fourier-space reconstruction
 * with wide-angle redshift-space distortions of Burden, Percival & Howlett,
 * "Reconstruction in Fourier space" (arXiv:1504.02591).
 *
 * Method, as implemented (section / equation names refer to the paper):
 *   paint    -- galaxies and randoms are binned onto an N^3 mesh (Sec. 3.1, Sec. 3.2);
 *               here with a deterministic integer fixed-point cloud-in-cell stencil.
 *   solve    -- Gaussian smoothing S(k) = exp(-k^2 R^2/2) in Fourier space (Sec. 3.1),
 *               galaxy and random densities smoothed separately, overdensity
 *               delta = (rho - rho_bar)/rho_bar (Sec. 2) formed against the randoms and
 *               zeroed outside a binary survey mask (Sec. 3.2), then the starting
 *               displacement: the Zel'dovich solve Psi(k) = i k delta(k)/(b k^2)
 *               (Sec. 2, eq. Zeldovich) or the approximate RSD-corrected starts of
 *               eq. (approx1) / eq. (approx2).
 *   iterate  -- the iterative removal of the non-parallel RSD term (Sec. 5.1,
 *               eq. iterative): D_{n+1} = D_s + f div[(Psi_n . r) r] with r the unit
 *               vector from the observer to each cell, Psi_{n+1} = i k D_{n+1}/(b k^2);
 *               the fixed point solves eq. (Nusser) with the RSD term scaled by
 *               beta = f/b.
 *   shift    -- galaxies and randoms are moved back along the displacement
 *               (Sec. 1): -Psi - f (Psi . r) r for galaxies, -Psi for randoms.
 *
 * Conventions: grid node (ix,iy,iz) sits at box_origin + (L/N)(ix,iy,iz); real fields
 * are [iz][iy][ix] float32 (x fastest); the box is periodic.  Positions are float32
 * [n][3] (x,y,z); weights float32 [n] with 0 <= w < 64 (NULL means 1).
 *
 * Ownership: every pointer argument named "device" is device memory owned by the
 * caller, who keeps it alive until the plan's stream has completed the call.  The
 * workspace passed to recon_plan is caller-owned device memory that the plan uses
 * exclusively until recon_destroy.  The plan owns only host-side metadata.
 *
 * Ordering: calls are asynchronous on the plan's stream except where noted (the
 * solve reads totals back once; iterate reads one convergence norm per pass).
 * The state machine is paint(GAL) [, paint(RAN)] -> solve -> iterate (repeatable)
 * -> shift / get_psi; recon_set_delta replaces the paint steps.
 *
 * Errors: every call returns RECON_OK (0), a positive warning, or a negative error
 * code; recon_strerror names the code and recon_last_error returns the plan's last
 * message.  No C++ exception crosses this interface.
 */
#ifndef RECON_H
#define RECON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define RECON_OK 0
#define RECON_NOTCONVERGED 1   /* warning: max_iter reached before the tolerance */
#define RECON_RESTARTED 2      /* warning: a learned start was rejected and its realisation restarted
                                  from the plain start (converged otherwise); see recon_iterate   */
#define RECON_EINVAL (-1)      /* invalid argument or invalid input data (NaN position, bad weight, ...) */
#define RECON_ENOMEM (-2)      /* workspace too small */
#define RECON_EDEVICE (-3)     /* a HIP runtime call or kernel launch failed */
#define RECON_ESTATE (-4)      /* call out of order */
#define RECON_EDIVERGED (-5)   /* eps non-finite, rising on two consecutive passes to above 1e-5, or
                                  ||Psi_n|| > 100 ||Psi_1|| */

/* catalogue selector */
#define RECON_GAL 0
#define RECON_RAN 1
/* recon_shift: or-ed into the catalogue selector when pos, n and offsets are the catalogue painted last
   through the brick-binned deposit and pos has not changed since that paint */
#define RECON_SHIFT_AS_PAINTED 256

/* starting displacement */
#define RECON_START_PLAIN 0    /* Psi_0 from the redshift-space overdensity (Sec. 5.2, first start) */
#define RECON_START_FFTA1 1    /* eq. (approx1):  Psi_p - beta/(1+beta) (Psi_p . r) r            */
#define RECON_START_FFTA2 2    /* eq. (approx2):  Psi_p - 3 beta/(7+3 beta) (Psi_p . r) r        */
#define RECON_START_LEARNED 3  /* Psi_p + Delta r with Delta predicted by a small 3D CNN        */

/* plan flags */
#define RECON_NO_RANDOMS 1u        /* mean-density mode: delta = rho/rho_bar - 1, no randoms, no mask */
#define RECON_KEEP_DELTA 2u        /* keep the smoothed overdensity delta_s in configuration space     */
#define RECON_START_BUFFERS 4u     /* allocate the start-correction field (needed by FFTA / learned)   */
#define RECON_PASS_GRAPHS 32u      /* replay the steady-state correction pass as one HIP graph (captured
                                      on first use on a private stream; eager while profiling)         */
#define RECON_LOGNORMAL 64u        /* Sec. 6, eq. (logdelta): start from ln(max(1 + delta_s, 1e-3)) + C,
                                      C = -<ln(max(1 + delta_s, 1e-3))> over all cells (the kept
                                      delta_s of RECON_KEEP_DELTA is the transformed field); not applied
                                      to a field given to recon_set_delta                               */
#define RECON_FFT_SPLITBF16 128u   /* precision study: the last radix-8 stage of every transform of the steady
                                      correction pass's z step runs on the matrix cores as an 8-point DFT
                                      GEMM with split-bfloat16 operands (2 terms, 3 products, about
                                      2^-16 relative per product); n >= 64, other steps stay FP32      */
#define RECON_FFT_SPLITBF16_X3 256u  /* as RECON_FFT_SPLITBF16 with 3 terms (6 products, about 2^-24)  */
#define RECON_RELAXED 1024u        /* relaxed correction pass (not in the paper): D_{n+1} = (1 - w) D_n +
                                      w (D_s + f div[(Psi_n . r) r]) with w = 2/(2 + beta), beta = f/b.
                                      The pass of Sec. 5.1 has real eigenvalues in [-beta, 0] (the RSD
                                      term is -beta times a projection seen through k'/|k|), so this w
                                      shrinks the error by beta/(2 + beta) per pass instead of up to
                                      beta; the fixed point (eq. Nusser) is the same.  The first pass
                                      after an FFTA or learned start is the plain pass.                */

/* paint flags */
#define RECON_PAINT_ACCUMULATE 1u  /* add to the grid instead of replacing it */
#define RECON_PAINT_NGP 2u         /* nearest-grid-point deposit (the paper's binning, Sec. 3.1): the whole
                                      quantised weight on the nearest node (node i + 1 when the FP32
                                      fraction is >= 1/2); per-object atomics; the shift stays CIC   */

typedef struct recon_plan_s recon_plan_t;

typedef struct {
  int32_t n;               /* cells per side, power of two in [8, 1024]                                  */
  int32_t batch;           /* independent realisations sharing this geometry (>= 1)                      */
  double box_len;          /* L > 0 [Mpc/h]                                                              */
  double box_origin[3];    /* lower corner of the periodic box                                           */
  double observer[3];      /* observer position, same frame (Sec. 3.1: r points away from the observer)  */
  double bias;             /* b > 0 (Sec. 3.2: delta_g = b delta)                                         */
  double growth;           /* f >= 0 (eq. Nusser)                                                        */
  double smooth_r;         /* R >= 0 [Mpc/h] (Sec. 3.1 smoothing)                                        */
  double mask_tau;         /* mask threshold as a fraction of the mean 27-cell random sum (>= 0)          */
  uint32_t flags;          /* RECON_NO_RANDOMS | RECON_KEEP_DELTA | RECON_START_BUFFERS | RECON_PASS_GRAPHS |
                              RECON_LOGNORMAL | RECON_FFT_SPLITBF16[_X3] | RECON_RELAXED
                              (| RECON_CNN_BUFFERS | RECON_CNN_HALF, recon_cnn.h)                        */
  int64_t max_objects;     /* largest catalogue painted in one call that uses the brick-binned deposit
                              (workspace holds 36 B per object for it: the brick-ordered copy, each
                              object's slot, the brick-order shift's staging); larger calls fall back
                              to per-object atomics.  0 disables binning.  Must be < 2^32.             */
} recon_params_t;

/* Device bytes the workspace must provide for these parameters (0 if the parameters are invalid). */
size_t recon_workspace_bytes(const recon_params_t* params);

/* Create a plan.  workspace: device memory of at least recon_workspace_bytes bytes, 256-byte aligned,
 * caller-owned.  stream: a hipStream_t (NULL = default stream).  Returns EINVAL for invalid parameters,
 * ENOMEM when workspace_bytes is too small. */
int recon_plan(recon_plan_t** out, const recon_params_t* params, void* workspace, size_t workspace_bytes,
               void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): a plan whose workspace is the library's own device scratch, a
 * fixed array of recon_noalloc_limit() bytes (64 MiB) per GPU that each GPU the library runs on holds
 * until the process ends.  The call allocates no device or pinned memory (it calls no hipMalloc,
 * hipHostMalloc or hipFree; the plan's host-side record and its read-back buffers are ordinary host
 * memory).  It takes the scratch of the device current on the calling thread; stream must belong to
 * that device.  Every no-allocation plan on one GPU shares that GPU's scratch: creating one makes any
 * earlier one on the same device stale (its calls then return RECON_ESTATE), and calls of two such
 * plans that overlap in time race on the same memory.  The scratch keeps the last plan's contents;
 * the plan clears what it needs as a plan on a caller workspace does.  RECON_ENOMEM when the
 * parameters need more than recon_noalloc_limit() bytes (recon_workspace_bytes tells), RECON_EINVAL for
 * invalid parameters or RECON_PASS_GRAPHS (graph instantiation may allocate), RECON_EDEVICE when the
 * scratch address cannot be taken.  Otherwise the plan behaves as one from recon_plan. */
int recon_plan_noalloc(recon_plan_t** out, const recon_params_t* params, void* stream);
size_t recon_noalloc_limit(void);

/* Deposit a catalogue (Sec. 3.1 / 3.2 binning; cloud-in-cell in integer fixed point, units 2^-32 of
 * weight, periodic wrap).  pos: device float32 [n][3]; w: device float32 [n] or NULL; offsets: device
 * int64 [batch+1] giving each realisation's object range (NULL when batch == 1).  Objects with a
 * non-finite position, a position more than 2^30 cells from the box, or a weight outside [0, 64) are
 * skipped and make the next recon_solve return EINVAL.  The grid is bit-identical for any object order. */
int recon_paint(recon_plan_t* plan, int which, const float* pos, const float* w, int64_t n,
                const int64_t* offsets, uint32_t flags);

/* Totals, smoothing, mask, overdensity and its spectrum D_s, and the starting displacement (a
 * synchronisation point: error flags are read back).  start: RECON_START_*; net: device pointer to
 * the learned-start network parameters (RECON_START_LEARNED only, layout in recon_cnn.h; the plan
 * needs RECON_KEEP_DELTA | RECON_START_BUFFERS | RECON_CNN_BUFFERS), else NULL.
 * EINVAL when a painted object was invalid, or the total galaxy weight or the total random weight
 * of a realisation is zero (the overdensity is then undefined). */
int recon_solve(recon_plan_t* plan, int start, const void* net);

/* Run correction passes (Sec. 5.1) until eps_n = ||Psi_n - Psi_{n-1}|| / ||Psi_n|| <= tol for every
 * realisation, or max_iter passes in this call.  tol <= 0 runs exactly max_iter passes.  Synchronises
 * once per pass; the transform of the final Psi is left queued on the plan's stream.  iters_out: host int32 [batch], total passes of each realisation (may be NULL);
 * eps_out: host double [batch * max_iter], eps of each pass of this call, NaN-padded (may be NULL).
 * The plain iteration judges a learned start: a realisation whose learned start gives a non-finite
 * eps_1, an eps_1 above an upper bound of the plain start's eps_1 (beta/(1 - beta), and a bound from
 * the same pass's sums: the start is then provably worse than the plain one), or a diverging
 * iteration restarts once from the plain start (D_0 = D_s) within this call's pass budget; its pass
 * count and eps history then count from that restart (recon_start_restarts counts restarts).
 * Returns OK, NOTCONVERGED, RESTARTED (converged after a restart) or EDIVERGED.  May be called again
 * to continue. */
int recon_iterate(recon_plan_t* plan, int max_iter, double tol, int32_t* iters_out, double* eps_out);

/* Restarts from the plain start since the last recon_solve: host int32 [batch]. */
int recon_start_restarts(const recon_plan_t* plan, int32_t* out);

/* Sparsity of the last recon_solve's transforms (Sec. 3.2: the survey occupies part of the box), for
 * byte accounting: the setup transforms work on z tiles (one y row, a few consecutive x, every z) and
 * skip tiles with nothing to transform.  out: host int64 [batch][4] = {tiles of the galaxy grid that
 * hold data, the same for the random grid (0 without randoms), tiles with any cell inside the survey
 * mask (all tiles without randoms), tiles per realisation}.  ESTATE before a solve; synchronises. */
int recon_tile_counts(recon_plan_t* plan, int64_t* out);

/* Move a catalogue back along the displacement (Sec. 1).  disp_out: device float32 [n][3]
 * (galaxies: -Psi - f (Psi.r) r, randoms: -Psi, Psi interpolated with the deposit's stencil);
 * pos_out: device float32 [n][3] receiving pos + disp, or NULL.  which: RECON_GAL or RECON_RAN,
 * optionally or-ed with RECON_SHIFT_AS_PAINTED.  With that flag the caller states that pos, n and
 * offsets are the catalogue painted last through the brick-binned deposit (the plan has
 * max_objects >= n and the paint had no RECON_PAINT_NGP flag) and that pos is unchanged since: the
 * shift then runs on the deposit's brick-ordered copy of the positions and puts the results back in
 * input order, bit-identical to the direct shift; EINVAL when which, pos, n or offsets differ from
 * that paint's.  Without the flag the positions are read from pos.  Objects the deposit rejected get
 * a zero displacement. */
int recon_shift(recon_plan_t* plan, int which, const float* pos, int64_t n, const int64_t* offsets,
                float* disp_out, float* pos_out);

/* Copy the current displacement Psi (device float32 [batch][3][N^3], [iz][iy][ix]). */
int recon_get_psi(recon_plan_t* plan, float* psi_out);

/* Copy a deposit grid (device int64 [batch][N^3], units 2^-32 of weight). */
int recon_get_grid(recon_plan_t* plan, int which, int64_t* out);

/* Diagnostic of Sec. 4 (Table 1): over the grid points of each realisation, the ratio
 * q = (Psi_ref . r) / (Psi . r) of a reference displacement (e.g. the real-space one) to the current
 * Psi, both projected on the line of sight; points with Psi . r = 0 or q outside [lo, hi] (the
 * paper cuts q > 3 and q < -1) are outliers.  psi_ref: device float32 [batch][3][N^3];
 * stats_out: host double [batch][4] = {mean q, standard deviation, outlier fraction, kept count}.
 * Needs a computed Psi; synchronises once. */
int recon_radial_ratio(recon_plan_t* plan, const float* psi_ref, double lo, double hi, double* stats_out);

/* Diagnostic of Sec. 4.1 (eq. irrotational, eq. solenoidal): split the plane-parallel RSD field
 * (Psi.x) x of a real field psi_x = Psi.x (device float32 [batch][N^3]) into its irrotational part,
 * IFFT[k_x k_j / k^2 FFT(psi_x)] (derivative wavenumbers, zero at each axis's Nyquist index; the
 * k = 0 mode to the solenoidal part), and the solenoidal remainder psi_x x - irrotational.
 * irr_out, sol_out: device float32 [batch][3][N^3] (sol_out may be NULL).  Uses the plan's transform
 * buffers: afterwards the plan must be painted (or given delta_s) and solved again. */
int recon_helmholtz(recon_plan_t* plan, const float* psi_x, float* irr_out, float* sol_out);

/* Copy the smoothed masked overdensity delta_s (device float32 [batch][N^3]); needs RECON_KEEP_DELTA. */
int recon_get_delta(recon_plan_t* plan, float* out);

/* Test hook: supply delta_s directly (device float32 [batch][N^3]), replacing paint and smoothing. */
int recon_set_delta(recon_plan_t* plan, const float* delta_s);

/* Instrumentation (not part of the method): while enabled, every kernel launched by the plan is
 * bracketed by HIP events on the plan's stream.  recon_profile_stop synchronises the stream, writes the
 * launch count and summed duration (ms) of each kernel kind into counts[k] / total_ms[k] for
 * k < min(cap, kinds), clears the record and returns the number of kernel kinds; names come from
 * recon_profile_kernel_name(k). */
int recon_profile_start(recon_plan_t* plan);
/* Debug build only (the library compiled with -DRECON_DEBUG, librecon_debug.so): the number of array
 * indices the device code found outside their array (each such access is skipped), on the current
 * device since the last reset; synchronises the device; reset != 0 clears the count.  The release
 * build has no checks and returns -1; -2 on a HIP error. */
int64_t recon_debug_violations(int reset);
int recon_profile_stop(recon_plan_t* plan, int32_t* counts, double* total_ms, int cap);
const char* recon_profile_kernel_name(int kind);

void recon_destroy(recon_plan_t* plan);
const char* recon_strerror(int code);
const char* recon_last_error(const recon_plan_t* plan);

#ifdef __cplusplus
}
#endif

#endif /* RECON_H */
