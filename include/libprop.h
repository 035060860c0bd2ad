/*
 * libprop -- scalar and vectorial light propagation with exact adjoints on
 * one MI355X (gfx950) GPU.
 *
 * What is computed (paper: Methods, "Features and performance"; Software
 * section).  The simulator propagates complex fields between planes by two
 * methods, each scalar and vectorial: the FFT-based numerical integration of
 * the Rayleigh-Sommerfeld (RS) diffraction integral, and the chirped
 * z-transform (CZT), which samples an arbitrary output region.  A high-NA
 * objective is evaluated with CZT methods.  Gradients with respect to the
 * optical parameters (SLM phases, wave-plate retardance and angle) come from
 * the adjoint of every linear operator (the paper uses reverse-mode
 * autodiff, of which the adjoint method is a special case).
 *
 * Conventions (the paper states none; readings of this library):
 *  - grid: row-major [ny][nx], x fastest; sample (i, j) sits at
 *    (cx + (j - nx/2) dx, cy + (i - ny/2) dy) (integer division); metres.
 *  - time dependence exp(-i w t): outgoing waves exp(+i k r), k = 2 pi / lambda.
 *  - fields are interleaved complex: PROP_C64 = float (re, im) pairs
 *    (torch.complex64), PROP_C128 = double pairs (torch.complex128); real
 *    parameter arrays (phases, phase gradients) are float resp. double.
 *  - batch: `batch` independent fields stored back to back; every field
 *    pointer addresses batch * ny * nx contiguous elements.
 *  - adjoints: each *_adjoint applies the exact adjoint A^H of its forward
 *    operator A; with the gradient convention g = dL/dRe + i dL/dIm this
 *    maps output gradients to input gradients.
 *
 * Memory: every field pointer is DEVICE memory owned by the caller (e.g. a
 * torch tensor); the library neither retains nor frees it.  Inputs and
 * outputs must not overlap (PROP_EALIAS).  All calls are asynchronous on
 * `stream` (a hipStream_t; NULL = the legacy default stream).  Kernel
 * spectra, chirp vectors and twiddle tables are computed on first use, on
 * the caller's stream, and cached per geometry; a call on another stream
 * waits for them on the device.  Spectra and chirp vectors live in a
 * least-recently-used cache with a byte budget (prop_cache_set_limit);
 * workspace is cached per stream.  Calls on one stream are ordered; calls
 * on different streams may run concurrently.  A one-shot call may be
 * captured into a hipGraph once the same geometry has been computed
 * outside the capture.
 *
 * Status: 0 on success, > 0 success with a warning, < 0 error (nothing was
 * launched; outputs untouched).  Device-side numeric problems are not
 * checked: NaN/Inf in the input propagate to the output.
 */
#ifndef LIBPROP_H
#define LIBPROP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PROP_OK = 0,
  PROP_WUNDERSAMPLED = 1, /* RS/VRS: exp(ikr) under-sampled at the largest offset (result still computed) */
  PROP_ENULL = -1,        /* a required pointer is NULL */
  PROP_ESHAPE = -2,       /* n < 1, batch < 0, or a transform length above 8192 */
  PROP_EPARAM = -3,       /* bad dtype, lambda <= 0, z <= 0, pitch <= 0, NA not in (0,1), f <= 0, non-finite */
  PROP_EALIAS = -4,       /* an output overlaps an input */
  PROP_ENOMEM = -5,       /* device allocation failed */
  PROP_EDEVICE = -6,      /* a HIP call failed; prop_last_device_error() has the code */
  PROP_ELIMIT = -7        /* beyond the fixed scratch of an allocation-free entry point */
};

/* The two sentinels give the enum the value range of int32_t, so that an
 * out-of-range value from a C caller stays defined in C++ and is rejected
 * with PROP_EPARAM instead of being assumed away by the compiler. */
typedef enum {
  PROP_C64 = 0,
  PROP_C128 = 1,
  PROP_DTYPE_MIN_ENUM_ = -0x7fffffff - 1,
  PROP_DTYPE_MAX_ENUM_ = 0x7fffffff
} prop_dtype;

/* Sampling grid: nx, ny samples with pitch dx, dy, centred at (cx, cy). */
typedef struct {
  int32_t nx, ny;
  double dx, dy;
  double cx, cy;
} prop_grid;

/* Aplanatic objective for the focusing mode of VCZT. */
typedef struct {
  double na; /* numerical aperture, 0 < na < 1 */
  double f;  /* focal length (m); the pupil is the input grid, aperture radius f*na */
} prop_lens;

/* ---------------------------------------------------------------- RS --
 * Scalar Rayleigh-Sommerfeld (first kind) propagation over distance z > 0
 * onto the input grid (paper: Methods, RS propagation; Software section,
 * "a general FFT-based light propagation algorithm"):
 *   U(x_m, y_l) = dx dy sum_{i,j} U0(x_j, y_i) H(x_m - x_j, y_l - y_i; z),
 *   H = (1/2pi)(z/r^2)(1/r - i k) exp(i k r),  r = sqrt(X^2 + Y^2 + z^2),
 * evaluated exactly (up to rounding) as a zero-padded FFT convolution of
 * length M = prop_fft_length(2n - 1) per axis (the smallest supported
 * length >= 2n - 1).  Requires M <= 8192, i.e. nx, ny <= 4096.
 * u_in/u_out: [batch][ny][nx].
 * Returns PROP_WUNDERSAMPLED when, along some axis with 2 d > lambda,
 * z < sqrt((2 L d / lambda)^2 - L^2) (L = n d), after launching.
 */
int rs_propagate(prop_dtype t, const void* u_in, void* u_out, const prop_grid* g, double wavelength,
                 double z, int32_t batch, void* stream);
/* g_in = A^H g_out for A = rs_propagate (same geometry and layout). */
int rs_adjoint(prop_dtype t, const void* g_out, void* g_in, const prop_grid* g, double wavelength,
               double z, int32_t batch, void* stream);

/* --------------------------------------------------------------- CZT --
 * Fresnel propagation over z > 0 onto an arbitrary output window `win`
 * (position and pitch free; paper: Methods, "CZT ... allows arbitrary
 * selection and sampling of the region of interest"):
 *   U(X_p, Y_q) = K P(X_p, Y_q) sum_{i,j} U0(x_j, y_i) Q(x_j, y_i)
 *                 exp(-i 2pi (X_p x_j + Y_q y_i) / (lambda z)),
 *   K = exp(ikz) dx dy / (i lambda z), Q = exp(ik(x^2+y^2)/2z),
 *   P = exp(ik(X^2+Y^2)/2z),
 * evaluated by separable Bluestein transforms of length
 * L = prop_fft_length(n_in + n_out - 1) per axis (L <= 8192).
 * u_in: [batch][g_in.ny][g_in.nx]; u_out: [batch][win.ny][win.nx].
 */
int czt_propagate(prop_dtype t, const void* u_in, void* u_out, const prop_grid* g_in,
                  const prop_grid* win, double wavelength, double z, int32_t batch, void* stream);
/* g_in = A^H g_out for A = czt_propagate (window -> input grid). */
int czt_adjoint(prop_dtype t, const void* g_out, void* g_in, const prop_grid* g_in_grid,
                const prop_grid* win, double wavelength, double z, int32_t batch, void* stream);

/* --------------------------------------------------------------- VRS --
 * Vectorial RS (paper: Methods, vectorial RS): E_x, E_y propagate as scalar
 * RS; E_z follows from div E = 0:
 *   E_z = -dx dy sum [E_x0 (x - x')/z + E_y0 (y - y')/z] H.
 * ex, ey, ox, oy, oz: [batch][ny][nx].  Same limits and warning as RS.
 */
int vrs_propagate(prop_dtype t, const void* ex, const void* ey, void* ox, void* oy, void* oz,
                  const prop_grid* g, double wavelength, double z, int32_t batch, void* stream);
/* (g_ex, g_ey) = A^H (g_x, g_y, g_z) for A = vrs_propagate. */
int vrs_adjoint(prop_dtype t, const void* gx, const void* gy, const void* gz, void* gex, void* gey,
                const prop_grid* g, double wavelength, double z, int32_t batch, void* stream);

/* -------------------------------------------------------------- VCZT --
 * Vectorial CZT (paper: Methods, vectorial CZT; high-NA objective "with CZT
 * methods").  lens == NULL: free space over z > 0 with C the CZT operator,
 *   E_x = C[E_x0], E_y = C[E_y0],
 *   E_z = -(1/z) (X C[E_x0] + Y C[E_y0] - C[x E_x0 + y E_y0]).
 * lens != NULL: focal field of an aplanatic objective (Richards-Wolf/Debye
 * integral; z is ignored but must be finite):
 *   E(X,Y) = (i k f e^{-ikf} / 2pi) (dx dy / f^2)
 *            sum_pupil (E_inf / s_z) exp(i k (s_x X + s_y Y)),
 *   s_perp = (x, y)/f, s_z = sqrt(1 - |s_perp|^2), aperture x^2+y^2 <= (f na)^2,
 *   E_inf = sqrt(s_z) [(E0.n_phi) n_phi + (E0.n_rho) n_theta].
 * ex, ey: [batch][g_in.ny][g_in.nx]; ox, oy, oz: [batch][win.ny][win.nx].
 */
int vczt_propagate(prop_dtype t, const void* ex, const void* ey, void* ox, void* oy, void* oz,
                   const prop_grid* g_in, const prop_grid* win, double wavelength, double z,
                   const prop_lens* lens, int32_t batch, void* stream);
/* (g_ex, g_ey) = A^H (g_x, g_y, g_z) for A = vczt_propagate. */
int vczt_adjoint(prop_dtype t, const void* gx, const void* gy, const void* gz, void* gex, void* gey,
                 const prop_grid* g_in, const prop_grid* win, double wavelength, double z,
                 const prop_lens* lens, int32_t batch, void* stream);

/* Adjoint fused with the SLM phase gradient (the last pass of the adjoint
 * writes it directly; paper: Methods, one free phase per SLM pixel, and the
 * gradients of the loss with respect to it).  For U = V exp(i phi) entering
 * the propagator, g_U = A^H g_out and dL/dphi = Im(g_U conj U):
 * grad (real, [batch][ny][nx] of the input grid) receives Im(g_U conj u),
 * added to its contents when accumulate != 0.  g_u (may be NULL) receives
 * g_U itself.  u: the modulated field that entered the propagator.  Same
 * geometry, limits and warnings as rs_adjoint / czt_adjoint.
 */
int rs_adjoint_phase_grad(prop_dtype t, const void* g_out, const void* u, void* g_u, void* grad,
                          int32_t accumulate, const prop_grid* g, double wavelength, double z,
                          int32_t batch, void* stream);
int czt_adjoint_phase_grad(prop_dtype t, const void* g_out, const void* u, void* g_u, void* grad,
                           int32_t accumulate, const prop_grid* g_in, const prop_grid* win,
                           double wavelength, double z, int32_t batch, void* stream);

/* ------------------------------------------------- distance gradients --
 * Derivative of L with respect to the propagation distance z, for a loss
 * whose gradient seed on the output is g_out (g = dL/dRe + i dL/dIm, the
 * adjoints' convention).  Every experiment of the paper optimises
 * distances along with the phase masks (Results; Methods, parameter
 * spaces include the distances z_i).  dz: device double [batch], one value
 * per batch item, dL/dz = Re sum conj(g_out) dU/dz (FP64 fixed-order
 * reduction).
 * rs_grad_z: dU/dz = dx dy sum U0 dH/dz with the RS-I kernel derivative
 *   dH/dz = (1/2pi) e^{ikr} [1/r^3 - ik/r^2 + z^2 (k^2/r^3 + 3ik/r^4 - 3/r^5)]
 *   (one RS pass with that kernel's spectrum, cached like H).  Same limits
 *   and sampling warning as rs_propagate.
 * czt_grad_z: differentiating every z-dependent factor of the CZT sum,
 *   dU/dz = (ik - 1/z - ik|X|^2/(2z^2)) U - (ik/(2z^2)) C[|x|^2 U0]
 *           + (2 pi i/(lambda z^2)) (X C[x U0] + Y C[y U0]),
 *   C = czt_propagate; u_out = C[u_in] if the caller has it, else NULL
 *   (computed internally).
 */
int rs_grad_z(prop_dtype t, const void* u_in, const void* g_out, double* dz, const prop_grid* g,
              double wavelength, double z, int32_t batch, void* stream);
/* rs_adjoint_grad_z: rs_adjoint and rs_grad_z of one RS step in one call,
 * for a backward pass that needs both: g_in = RS^H g_out (the same passes
 * as rs_adjoint) and dz as rs_grad_z gives it, up to rounding.  The sum is
 * taken in the row-spectrum domain (Parseval along x), where the adjoint's
 * first pass already holds the transformed g_out, so the distance gradient
 * costs one row pass, one column pass and a dot product instead of a full
 * propagation and a dot product.  u_in: the step's forward input, g_out:
 * the output seed, both [batch][ny][nx]; g_in (same layout) and dz (device
 * double [batch]) may not overlap the inputs or each other (PROP_EALIAS).
 * Same limits and sampling warning as rs_propagate. */
int rs_adjoint_grad_z(prop_dtype t, const void* g_out, const void* u_in, void* g_in, double* dz,
                      const prop_grid* g, double wavelength, double z, int32_t batch, void* stream);
int czt_grad_z(prop_dtype t, const void* u_in, const void* u_out, const void* g_out, double* dz,
               const prop_grid* g_in, const prop_grid* win, double wavelength, double z, int32_t batch,
               void* stream);

/* ------------------------------------------------- sources and elements --
 * Gaussian source (paper: Methods, light sources of any wavelength and
 * power): out = amplitude exp(-r^2/w0^2) [exp(-i k r^2 / 2 lens_f) if
 * lens_f > 0], r measured from the origin; phases in FP64.  out:
 * [batch][ny][nx], every batch item identical.
 */
int prop_source_gaussian(prop_dtype t, void* out, const prop_grid* g, double w0, double amplitude,
                         double lens_f, double wavelength, int32_t batch, void* stream);
/* Radially polarised source: (E_x, E_y) = (x, y) exp(-r^2/w0^2) /
 * (w0 exp(-1/2) / sqrt 2), so that max |E_perp| = 1. */
int prop_source_radial(prop_dtype t, void* ex, void* ey, const prop_grid* g, double w0, int32_t batch,
                       void* stream);
/* SLM (paper: Methods, one free phase per pixel): u_out = u_in exp(i phase).
 * phase: real [phase_batch][npix] with phase_batch = batch or 1 (shared). */
int prop_modulate(prop_dtype t, const void* u_in, const void* phase, void* u_out, int64_t npix,
                  int32_t batch, int32_t phase_batch, void* stream);
/* SLM adjoint: g_in = g_out exp(-i phase) (same layout and rules as
 * prop_modulate). */
int prop_modulate_adjoint(prop_dtype t, const void* g_out, const void* phase, void* g_in, int64_t npix,
                          int32_t batch, int32_t phase_batch, void* stream);
/* SLM gradient: grad = Im(g_u conj(u)) (u = the modulated field), real
 * [batch][npix]; accumulate != 0 adds to grad. */
int prop_phase_grad(prop_dtype t, const void* g_u, const void* u, void* grad, int64_t npix,
                    int32_t batch, int32_t accumulate, void* stream);
/* SLM gradient of a phase shared by the whole batch (phase_batch 1 in
 * prop_modulate): grad[pix] = sum_b Im(g_u[b][pix] conj(u[b][pix])), the
 * batch summed per pixel in a fixed order in FP64; real [npix];
 * accumulate != 0 adds to grad. */
int prop_phase_grad_sum(prop_dtype t, const void* g_u, const void* u, void* grad, int64_t npix,
                        int32_t batch, int32_t accumulate, void* stream);
/* out[k][b][.] = in[k][b][.] * scale[b] for k < nplanes (1..3), scale a
 * device double [batch] (e.g. an upstream gradient applied to per-item
 * gradient seeds).  in, out: host arrays of device pointers; out[k] may be
 * in[k] (in place), other overlaps are rejected (PROP_EALIAS). */
int prop_scale_items(prop_dtype t, const void* const* in, void* const* out, int32_t nplanes,
                     const double* scale, int64_t npix, int32_t batch, void* stream);
/* Wave plate / variable retarder (paper: Methods, variable retarders with
 * retardance eta and angle theta): (ox, oy) = J (ex, ey),
 * J = R(-theta) diag(1, e^{i eta}) R(theta). */
int prop_waveplate(prop_dtype t, const void* ex, const void* ey, void* ox, void* oy, double eta,
                   double theta, int64_t npix, int32_t batch, void* stream);
/* Adjoint: (g_ex, g_ey) = J^H (g_x, g_y); dparams (device double
 * [batch][2]) receives dL/deta, dL/dtheta per batch item (deterministic
 * fixed-order reduction). ex, ey: the wave plate's inputs. */
int prop_waveplate_adjoint(prop_dtype t, const void* gx, const void* gy, const void* ex,
                           const void* ey, void* gex, void* gey, double eta, double theta,
                           double* dparams, int64_t npix, int32_t batch, void* stream);
/* Wave plates with one parameter pair per batch item, read from device
 * memory: params = device double [batch][2] = (eta, theta), so that
 * optimised parameters stay on the GPU.  Same matrix as prop_waveplate. */
int prop_waveplate_batched(prop_dtype t, const void* ex, const void* ey, void* ox, void* oy,
                           const double* params, int64_t npix, int32_t batch, void* stream);
/* Adjoint: (g_ex, g_ey) = J_b^H (g_x, g_y) per item.  gey may be NULL when
 * both input components were one field (a wave plate fed (A, A)): gex then
 * receives g_A = (J^H g)_x + (J^H g)_y.  If dparams (device double
 * [batch][2]) is non-NULL it receives (dL/deta, dL/dtheta) per item
 * (fixed-order FP64 reduction) and ex, ey (the forward inputs) are
 * required; otherwise they may be NULL. */
int prop_waveplate_batched_adjoint(prop_dtype t, const void* gx, const void* gy, const void* ex,
                                   const void* ey, void* gex, void* gey, const double* params,
                                   double* dparams, int64_t npix, int32_t batch, void* stream);

/* Beam splitter (paper: Methods, large-scale search space; Results,
 * large-scale ansatz with beam-splitter ratios [T, R]).  Lossless,
 * symmetric and polarisation independent, with mixing angle alpha per batch
 * item (T = cos^2 alpha, R = sin^2 alpha), on each of ncomp (1..3)
 * components k:
 *   c_k = cos(alpha) a_k + i sin(alpha) b_k,  d_k = i sin(alpha) a_k + cos(alpha) b_k.
 * a, b, c, d: host arrays of ncomp device pointers, each a [batch][npix]
 * plane.  a or b may be NULL: a dark input port (zero field).  alpha:
 * device double [batch].  Outputs may not overlap inputs or each other
 * (PROP_EALIAS). */
int prop_beam_splitter(prop_dtype t, const void* const* a, const void* const* b, void* const* c,
                       void* const* d, int32_t ncomp, const double* alpha, int64_t npix,
                       int32_t batch, void* stream);
/* Adjoint: g_a = cos g_c - i sin g_d, g_b = -i sin g_c + cos g_d (ga or gb
 * NULL: not wanted).  If dalpha (device double [batch]) is non-NULL it
 * receives dL/dalpha = Re sum conj(g_c) dc/dalpha + conj(g_d) dd/dalpha per
 * item (fixed-order FP64 reduction) from the forward inputs a, b (NULL =
 * dark port). */
int prop_beam_splitter_adjoint(prop_dtype t, const void* const* gc, const void* const* gd,
                               const void* const* a, const void* const* b, void* const* ga,
                               void* const* gb, int32_t ncomp, const double* alpha, double* dalpha,
                               int64_t npix, int32_t batch, void* stream);

/* -------------------------------------------------------------- losses --
 * Detector loss on window `win`: I = |E_x|^2 + |E_y|^2 + |E_z|^2,
 * sigma^2 = sum I |X - Xbar|^2 / P about the intensity centroid,
 * F_z = sum |E_z|^2 / P, loss = sigma^2 / lambda^2 + w_fz F_z.
 * ez may be NULL (two components).  result: device double [batch][8] =
 * (loss, sigma^2, F_z, P, Xbar - cx, Ybar - cy, 0, 0).  If gx and gy are
 * non-NULL the gradient seeds g_c = 2 E_c dL/dI_c are written (gz too when
 * ez and gz are non-NULL).  Reductions use FP64 in a fixed order.
 */
int prop_spot_loss(prop_dtype t, const void* ex, const void* ey, const void* ez, const prop_grid* win,
                   double wavelength, double w_fz, double* result, void* gx, void* gy, void* gz,
                   int32_t batch, void* stream);
/* Allocation-free variant of prop_spot_loss, for callers that cannot
 * allocate device memory: code under hipGraph stream capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, results and
 * errors; it calls no hipMalloc, hipFree or allocating routine.  Its FP64
 * partial sums live in a fixed device array of the library (2.5 MiB per
 * GPU, kept until the process ends) instead of per-stream workspace, so
 * batch is limited to 256 (PROP_ELIMIT above).  All calls on one GPU share
 * that array: calls that overlap in time on one GPU (e.g. on two streams)
 * race and must be ordered by the caller.  Results equal prop_spot_loss's
 * bit for bit (same kernels, same reduction order). */
int prop_spot_loss_noalloc(prop_dtype t, const void* ex, const void* ey, const void* ez, const prop_grid* win,
                           double wavelength, double w_fz, double* result, void* gx, void* gy, void* gz,
                           int32_t batch, void* stream);

/* The paper's detector side (Methods: STED microscopy; loss function;
 * exploration of optical topologies).
 * prop_density_loss: threshold-density loss L = Area / I_eps of the
 *   detected intensity I, with i_eps = I where I > eps * max I (0 <= eps <= 1),
 *   I_eps = sum i_eps, Area = number of such pixels.  I is the intensity of
 *   the ncomp (1..3) field components comps[k] (e.g. E_x, E_y for the radial
 *   component, E_z alone for the longitudinal one), formed in FP64 as
 *   sum_k (Re^2 + Im^2) in the order given.  With ndep > 0 it is the STED
 *   effective intensity I_eff = I_ex [1 - beta (1 - exp(-I_dep / I_ex))]
 *   (0 where I_ex = 0) of that excitation intensity and the depletion
 *   intensity of the fields dep[k], quenching efficiency 0 <= beta <= 1.
 *   Every field: device [batch][npix] of dtype t.  result: device double
 *   [batch][4] = (L, Area, I_eps, max I).  seeds / dep_seeds (optional
 *   arrays of ncomp / ndep device pointers, entries may be NULL): gradient
 *   seeds g_c = 2 E_c dL/dI_c, where dL/dI = -Area / I_eps^2 on the
 *   selected pixels and 0 elsewhere (the selection itself carries no
 *   gradient), chained through dI_eff/dI_ex = 1 - beta + beta e^{-r}(1 + r)
 *   and dI_eff/dI_dep = -beta e^{-r}, r = I_dep / I_ex.
 * prop_softmin: smooth minimum over ndet detector losses per batch item,
 *   value = -log(sum exp(-beta l)) / beta (beta > 0), weights (optional,
 *   [batch][ndet]) = d value / d l.  All pointers are device doubles.
 */
int prop_density_loss(prop_dtype t, const void* const* comps, int32_t ncomp, const void* const* dep,
                      int32_t ndep, double beta, int64_t npix, double eps, double* result,
                      void* const* seeds, void* const* dep_seeds, int32_t batch, void* stream);
int prop_softmin(const double* losses, int32_t ndet, double beta, double* value, double* weights,
                 int32_t batch, void* stream);

/* Optimiser step on the device (the paper optimises with Adam, comparing
 * AdamW among others; Methods).  One Adam step with bias correction over n
 * real parameters: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr wd p + lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps);
 * weight_decay (wd) > 0 is the decoupled AdamW decay.  t selects the
 * precision of param, grad, m, v: PROP_C64 -> float, PROP_C128 -> double
 * (device arrays of n; m and v start at zero, step counts from 1).
 */
int prop_adam_step(prop_dtype t, void* param, const void* grad, void* m, void* v, int64_t n, double lr,
                   double beta1, double beta2, double eps, double weight_decay, int32_t step, void* stream);

/* Stopping rule of the optimisation (Methods, discovery experiments: a run
 * ends once its best loss has stood for 500 steps, looked at every 100
 * steps).  Per batch item b: if loss[b] < best[b] then
 * best[b] = loss[b], since[b] = 0, else since[b] += 1 (a NaN loss never
 * improves).  Device arrays of batch entries, owned by the caller: loss
 * (float64, read), best (float64, start at +inf) and since (int64, start at
 * 0), both updated in place.  The caller reads `since` back at its checks
 * and stops an item once since >= patience.  best and since must not
 * overlap loss or each other (PROP_EALIAS); batch 0 is a no-op.
 */
int prop_track_best(const double* loss, double* best, int64_t* since, int32_t batch, void* stream);

/* Gradient of a parameter shared by a batch (a distance, a wave plate):
 * out[j] = sum over items i < n of in[i * m + j], summed in item order in
 * FP64.  in: device double [n][m]; out: device double [m], not overlapping
 * in (PROP_EALIAS); n, m >= 1 (PROP_ESHAPE). */
int prop_sum_items(const double* in, double* out, int32_t n, int32_t m, void* stream);

/* ------------------------------------------------------------- utility -- */
/* Host-only sampling check of RS/VRS: PROP_OK or PROP_WUNDERSAMPLED. */
int prop_sampling_check(const prop_grid* g, double wavelength, double z);
/* Smallest supported transform length >= n, or -1 above 8192.  Supported
 * lengths: powers of two 1..8192 and 3 * 2^k for 96 <= 3 * 2^k <= 6144. */
int32_t prop_fft_length(int32_t n);
/* Autotuner.  The column passes (RS column convolution, vectorial mixing,
 * Bluestein columns) and the Bluestein row passes have launch variants:
 * lines per workgroup on the built-in radix schedule (bit-identical
 * results) and, for complex64 transforms of length 768, 1024, 1536 and 3072,
 * the same on an alternative schedule whose first and last radices are
 * equal (8x12x8, 8x16x8, 16x6x16, 16x12x16; the product of a convolution
 * then stays in registers) -- different rounding, so a tuned choice is kept
 * for the shape (and by a plan for its lifetime) and recorded.  With
 * LIBPROP_AUTOTUNE=1 in the environment (or during the first execution of a
 * PROP_PLAN_AUTOTUNE plan) the first launch of each new shape takes its
 * choice from the tuning cache file when that holds a valid record for this
 * GPU architecture and shape, and otherwise times every candidate on
 * scratch buffers (allocating them and synchronising the stream), keeps the
 * fastest and appends it to the file; without tuning, and under stream
 * capture, the built-in variant is used and the file is not read.
 * prop_autotune_report writes one text line per tuned shape (chosen
 * variant, schedule, lines per workgroup, whether timed or read from the
 * file, and the measured ms of each candidate) into buf (cap bytes,
 * NUL-terminated) and returns the size needed including the NUL. */
int32_t prop_autotune_report(char* buf, int32_t cap);
/* Tuning cache file: one text line per shape, "libprop-tune 1 <arch>
 * <element bytes> <pass kind> <n> <lines> <n_in> <n_out> <batch> <variant>".
 * Its path is `path`, or with path NULL LIBPROP_TUNE_CACHE, else
 * $XDG_CACHE_HOME/libprop/tune.txt or $HOME/.cache/libprop/tune.txt ("":
 * none).  A missing or unreadable file reads as empty; a malformed line, or
 * one whose variant is not a candidate of its shape, is skipped (those
 * shapes are timed anew); the last line of a shape wins.  prop_tune_cache_path
 * sets the path, reads the file and returns the number of usable records;
 * prop_tune_cache_rejected returns the number of lines skipped.  Choices
 * already made in this process are kept. */
int32_t prop_tune_cache_path(const char* path);
int32_t prop_tune_cache_rejected(void);
/* Free cached spectra, chirps, twiddles, workspaces and autotuner choices
 * (synchronises the device).  Tables pinned by live plans are kept: their
 * kernels and captured graphs address them until prop_plan_destroy. */
void prop_cache_clear(void);
/* Byte budget of the cached kernel spectra and zoom chirp vectors (default
 * 8 GiB, or LIBPROP_CACHE_MB from the environment; bytes <= 0 restores the
 * default).  Distances are optimised in every experiment of the paper
 * (Results; Methods, the large-scale search space), and each new distance
 * needs new tables; once the cached tables exceed the budget, the least
 * recently used ones that no plan pins and no call in progress uses are
 * freed, down to 3/4 of the budget.  Each such eviction round first
 * synchronises the device once (enqueued kernels may still read a
 * victim).  Pinned tables never count against eviction. */
void prop_cache_set_limit(int64_t bytes);
typedef struct {
  int64_t table_bytes;    /* bytes of cached spectra and zoom vectors */
  int64_t limit;          /* current budget */
  int64_t spectra, zooms, twiddles; /* cached entries */
  int64_t pinned;         /* entries pinned by live plans */
  int64_t evictions;      /* entries evicted so far */
  int64_t eviction_syncs; /* device synchronisations of eviction rounds */
} prop_cache_stats;
/* Snapshot of the cache (host struct owned by the caller; NULL: no-op). */
void prop_cache_info(prop_cache_stats* out);
/* Text for a status code. */
const char* prop_status_string(int status);
/* hipError_t of the last PROP_EDEVICE on this thread (0 if none). */
int prop_last_device_error(void);

/* ---------------------------------------------------------------- plans --
 * Batches of independent setups of uneven sizes and parameters (the paper
 * evaluates many candidate setups per optimisation step: Results, batches
 * of setups sharing parameters; Methods, compile-once-per-shape reuse).
 * prop_plan_create validates every setup, computes all kernel spectra, chirp
 * vectors and twiddle tables (pinned in the cache for the plan's lifetime:
 * neither eviction nor prop_cache_clear frees them), and allocates all
 * workspace, so that
 * prop_plan_forward / prop_plan_adjoint / prop_plan_step only enqueue
 * kernels: they neither allocate nor synchronise, and may be captured into a
 * caller's hipGraph.  prop_plan_step is prop_plan_forward followed by
 * prop_plan_adjoint (the same kernels in the same order, so the same bits),
 * for callers whose output gradients gout are fixed before the step (the
 * paper's batches evaluate forward and gradient of every setup in one
 * step).  With PROP_PLAN_GRAPH the plan captures its own forward, adjoint
 * and step once each, on first use (setups spread over up to 4 parallel
 * branches; in the step every forward branch joins before the adjoint
 * branches start), and afterwards replays each as a single hipGraphLaunch
 * on the caller's stream.
 *
 * Per setup (one propagator call, or one RS -> lens -> CZT chain, on
 * `batch` fields), with the stage factor f = exp(i phase) exp(-i k r^2 /
 * (2 lens_f)) (each factor optional):
 *   scalar ops (RS, CZT): forward out = op(in * f); adjoint g_u = op^H(gout),
 *     gin = g_u conj(f) (if gin != NULL), grad_phase = Im(g_u conj(in * f))
 *     (if grad_phase != NULL).  The stage runs inside the transforms: the
 *     phase multiplies the loads of the first pass, and the last pass of the
 *     adjoint writes gin and grad_phase; a CZT folds its lens into the input
 *     chirp exactly, RS applies it as separable factors.  The adjoint reads
 *     in[0] again, which must therefore still hold the forward's input;
 *   PROP_OP_RS_CZT (the chain of one setup of the paper's batched searches:
 *     SLM, free space, lens, focal plane): forward out = CZT_z2(L RS_z(in *
 *     exp(i phase))), L = exp(-i k r^2 / (2 lens_f)) (lens_f 0: none) on the
 *     input grid, CZT over z2 onto `win`; adjoint gin and grad_phase of
 *     in and phase as above.  The lens folds into the CZT chirp; the RS -> CZT
 *     intermediate lives in the plan's workspace;
 *   vector ops (VRS, VCZT): forward u = in * f (a pass of its own; the plan
 *     keeps u), out = op(u); adjoint g_u = op^H(gout), gin = g_u conj(f),
 *     grad_phase = sum over both components Im(g_u conj(u)).
 * Adjoints require a preceding forward.  Scalar ops use in[0], out[0],
 * gout[0], gin[0]; vector ops use two inputs and three outputs.  phase /
 * grad_phase: real [batch][g_in.ny][g_in.nx] (float for PROP_C64, double
 * for PROP_C128).  All pointers are device memory owned by the caller and
 * must stay valid for the plan's lifetime.
 * Errors: as the single calls, reported by prop_plan_create with *plan set
 * to NULL; PROP_ESHAPE for an unknown op.
 */
enum { PROP_OP_RS = 0, PROP_OP_CZT = 1, PROP_OP_VRS = 2, PROP_OP_VCZT = 3, PROP_OP_RS_CZT = 4 };
#define PROP_PLAN_GRAPH 1u
/* PROP_PLAN_AUTOTUNE: the first forward and the first adjoint (through
 * prop_plan_forward, prop_plan_adjoint or prop_plan_step) run eagerly with
 * the autotuner on (see
 * prop_autotune_report); they allocate scratch memory and synchronise the
 * stream.  Later calls (and the captured graph) use the chosen variants. */
#define PROP_PLAN_AUTOTUNE 2u
/* PROP_PLAN_FAULT_NOMEM (fault injection, for testing callers' error paths):
 * prop_plan_create fails as if its workspace allocation had failed on an
 * exhausted device: it returns PROP_ENOMEM, sets *plan to NULL, frees
 * everything it allocated and launches nothing on the caller's buffers. */
#define PROP_PLAN_FAULT_NOMEM 0x100u

typedef struct {
  int32_t op;           /* PROP_OP_* */
  int32_t batch;        /* fields in this setup (>= 1) */
  prop_grid g_in, win;  /* win: output window of CZT / VCZT / RS_CZT (ignored for RS / VRS) */
  double wavelength, z; /* z ignored by focusing VCZT; the RS distance of RS_CZT */
  int32_t has_lens;     /* VCZT: focusing mode with `lens` */
  prop_lens lens;
  double lens_f;        /* > 0: thin-lens phase on the input (RS_CZT: between RS and CZT) */
  const void* phase;    /* optional SLM phase applied to the input */
  const void* in[2];
  void* out[3];
  const void* gout[3];
  void* gin[2];
  void* grad_phase;     /* optional: dL/dphase */
  double z2;            /* RS_CZT: the CZT distance (> 0); ignored otherwise */
} prop_setup;

typedef struct prop_plan prop_plan;
int prop_plan_create(prop_dtype t, const prop_setup* setups, int32_t n, uint32_t flags, prop_plan** plan);
int prop_plan_forward(prop_plan* plan, void* stream);
int prop_plan_adjoint(prop_plan* plan, void* stream);
int prop_plan_step(prop_plan* plan, void* stream);
void prop_plan_destroy(prop_plan* plan);

/* ------------------------------------------------------------- tracing --
 * Kernel-level timing for benchmarks and profiling.  prop_trace_enable(1)
 * clears the trace and brackets every subsequent hot-path launch with a
 * pair of hipEvents recorded on the caller's stream; prop_trace_enable(0)
 * stops.  prop_trace_read() waits for the recorded events, aggregates them
 * per pass name (launch count, summed kernel milliseconds, summed
 * algorithmic bytes = compulsory reads + writes of each launch), writes at
 * most `max` entries to `out` (caller-owned host memory), clears the trace
 * and returns the number of passes, or PROP_EDEVICE.
 */
typedef struct {
  char name[32];
  int32_t launches;
  double total_ms;
  double bytes;
} prop_trace_stat;
void prop_trace_enable(int32_t on);
int32_t prop_trace_read(prop_trace_stat* out, int32_t max);
/* Restrict tracing to the launches of one pass (its name as reported by
 * prop_trace_read; the string is copied), or trace every pass again with
 * NULL.  Each traced launch records two events on its stream, which adds a
 * few microseconds between dependent kernels, so a timed run can trace just
 * the pass it reports on. */
void prop_trace_only(const char* name);

#ifdef __cplusplus
}
#endif

#endif /* LIBPROP_H */
