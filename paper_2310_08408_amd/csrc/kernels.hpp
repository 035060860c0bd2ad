// Host-side launch interface of the libprop HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_engine.hpp"

namespace lp {

// Lines of a batch of 2-D arrays.  Row mode: line l of batch item b starts
// at b*bstride + l*pitch and its elements are contiguous.  Column mode: line
// l is column l, element i at b*bstride + i*pitch + l.  (complex elements)
struct Lines {
  int64_t bstride, pitch;
};

// Plain transform of length n (a supported length) of nlines lines: inputs
// beyond n_in are zero, the first n_out outputs are kept and scaled.  In
// place is allowed.
template <typename T, int DIR>
hipError_t launch_fft_lines(int n, bool col, const cx<T>* in, cx<T>* out, Lines li, Lines lo, int nlines, int n_in,
                            int n_out, T scale, int batch, const cx<T>* tw, hipStream_t s);

// RS workspace layout.  The row-transformed plane of one field (rows y <
// ny, spectral columns kx < Mx) is stored in tiles of kTile adjacent
// columns: element (y, kx) at (kx / kTile) * ny * kTile + y * kTile +
// kx % kTile.  A column pass then reads and writes each tile as one
// contiguous block, and the row passes touch whole cache lines across
// kTile neighbouring rows.
constexpr int kTileShift = 2;
constexpr int kTile = 1 << kTileShift;
inline int64_t rs_plane_elems(int ny, int Mx) { return (int64_t)((Mx + kTile - 1) / kTile) * kTile * ny; }

// SLM / thin-lens stage of a plan setup, U = V exp(i phase) lx[col] ly[row]
// (each factor optional), fused into a transform pass instead of running as
// a pass of its own.  Forward: the first pass multiplies each loaded input
// by the factor.  Adjoint: the last pass stores g_V = g_U conj(factor) and,
// with a phase gradient requested, grad (+)= Im(g_V conj V) (which equals
// Im(g_U conj U)); V is then the PhaseGrad field u.
template <typename T>
struct Slm {
  const T* phase = nullptr;   // real [batch][ny][nx], item b at b * pbs (pbs 0: shared)
  int64_t pbs = 0;
  const cx<T>* lx = nullptr;  // exp(-i q x_col^2) [nx] and exp(-i q y_row^2) [ny], or NULL
  const cx<T>* ly = nullptr;
  int nx = 0;
  bool adjoint = false;       // Bluestein passes: stores of an adjoint (true) or loads of a forward
  bool active() const { return phase != nullptr || lx != nullptr; }
};

// RS row passes between contiguous fields [batch][nrows][n_io] and the tiled
// workspace (bstride w_bstride elements per batch item).  DIR = -1: forward
// transform of length n of each zero-padded input row into the workspace;
// DIR = +1: inverse transform of each workspace row, first n_io outputs
// kept and scaled.
// With pg_grad non-NULL the inverse pass also writes the SLM phase gradient
// pg_grad = Im(out conj pg_u) (added when pg_acc) of its output; out may
// then be NULL.
// slm (optional): the fused SLM stage -- applied to the loads of the forward
// pass, to the stores of the inverse pass (see Slm).
template <typename T, int DIR>
hipError_t launch_rs_rows(int n, const cx<T>* in, cx<T>* out, int64_t w_bstride, int nrows, int n_io, T scale,
                          int batch, const cx<T>* tw, hipStream_t s, const cx<T>* pg_u = nullptr,
                          T* pg_grad = nullptr, int pg_acc = 0, const Slm<T>* slm = nullptr);

// RS middle pass, in place on columns kx < ncols of the tiled workspace
// (bstride elements per batch item, n_valid rows): transform of length My
// of the zero-padded column, multiply by the even/even kernel spectrum Sq
// (half table, conjugated for the adjoint), inverse transform, keep the
// first n_valid rows.
template <typename T>
hipError_t launch_rs_cols(int My, cx<T>* W, int64_t bstride, int ncols, int n_valid, const cx<T>* Sq, int Mx,
                          bool conj_spec, int batch, const cx<T>* tw, hipStream_t s, int variant = 0);

// Vectorial RS middle pass on tiled workspaces: out column = IFFT(ca Sa
// FFT(a) + cb Sb FFT(b)) with half-table spectra of parity kind 0
// (even/even), 1 (odd in kx) or 2 (odd in ky); conj_spec conjugates both
// spectra.  out may equal a.
template <typename T>
hipError_t launch_mix2_cols(int My, const cx<T>* a, const cx<T>* b, cx<T>* out, int64_t bstride, int ncols,
                            int n_valid, const cx<T>* Sa, int kind_a, T ca, const cx<T>* Sb, int kind_b, T cb,
                            bool conj_spec, int Mx, int batch, const cx<T>* tw, hipStream_t s, int variant = 0);

// Bluestein zoom transform of each line: out[p] = post[p] *
// IFFT_L(FFT_L(pad(pre .* in)) .* chat)[p], p < n_out.
// slm (optional): the fused SLM stage on the loads (the first pass of a
// forward transform) or on the stores (the last pass of an adjoint), with
// rows and columns of the field grid taken from the line mode.
template <typename T>
hipError_t launch_bluestein(int L, bool col, const cx<T>* in, cx<T>* out, Lines li, Lines lo, int nlines, int n_in,
                            int n_out, const cx<T>* pre, const cx<T>* chat, const cx<T>* post, int batch,
                            const cx<T>* tw, hipStream_t s, int variant = 0, const cx<T>* pg_u = nullptr,
                            T* pg_grad = nullptr, int pg_acc = 0, const Slm<T>* slm = nullptr);

constexpr int kColVariants = 3;
constexpr int kSchedVariants = 2;
// Launch variants of the column and Bluestein passes (the `variant`
// argument above): variant v < kColVariants runs the built-in schedule with
// (C >> v) lines per workgroup -- bit-identical results for every v; v +
// kColVariants runs the length's alternative schedule (LP_ALT_LENGTHS, FP32
// only; RS columns and Bluestein passes), whose results differ in rounding.
// col_pass_lines gives the lines per workgroup of a candidate for kind 0
// (RS column pass), 1 (vectorial mixing), 2 (Bluestein columns) or 3
// (Bluestein rows) at length n, 0 if unsupported.
template <typename T>
int col_pass_lines(int kind, int n, int variant);
// Variant of an RS column pass (length My, ncols columns of n_valid rows)
// when nothing is tuned: bit-identical to variant 0, with fewer lines per
// workgroup where the pass would otherwise leave CUs idle.
template <typename T>
int rs_cols_fill_variant(int My, int ncols, int n_valid, int batch);
// The schedule a variant runs: 0 built-in, 1 alternative.
inline int variant_sched(int variant) { return variant / kColVariants; }

// ---- FP64 generators (setup work) ----
// Wrapped RS kernel on an My x Mx grid (complex128), kind 0: H, 1: (X/z) H,
// 2: (Y/z) H, 3: dH/dz.  Offsets d in [-(n-1), n-1] sit at index d mod M,
// the rest 0.
hipError_t launch_rs_kernel_wrapped(cx<double>* out, int Mx, int My, int nx, int ny, double dx,
                                    double dy, double k, double z, int kind, hipStream_t s);
// Kernel-spectrum table: rows ky = 0..My/2 of the full spectrum (the rest
// follows from its parity in ky), all columns, stored in 4-column tiles
// like the RS workspace: (ky, kx) at (kx / 4) (My/2+1) 4 + ky 4 + kx % 4, so
// a column pass reads its tile's spectrum as one contiguous block.
// Distance gradients.  scale * Re sum conj(a) b per batch item (npix
// elements each) into out[batch] (FP64, fixed order; partial: batch * nblk
// doubles).
template <typename T>
hipError_t launch_redot(const cx<T>* a, const cx<T>* b, double* out, double* partial, int nblk, int64_t npix,
                        int batch, hipStream_t s, double scale = 1.0);
// Threshold-density detector loss of the intensity of ncomp field
// components (optionally STED-modulated by ndep depletion components with
// quenching efficiency beta): res[batch][4] = (Area / I_eps, Area, I_eps,
// i_max); seeds (optional, per component) g_c = 2 E_c dL/dI_c.  scratch:
// 3 * batch * nblk doubles.
template <typename T>
hipError_t launch_density_loss(const void* const* comps, int ncomp, const void* const* dep, int ndep, double beta,
                               int64_t npix, double eps, double* res, double* scratch, int nblk, void* const* seeds,
                               void* const* dep_seeds, int batch, hipStream_t s);
// One Adam (AdamW when wd > 0) step over n real parameters, step >= 1.
template <typename T>
hipError_t launch_adam(T* p, const T* g, T* m, T* v, int64_t n, double lr, double b1, double b2, double eps,
                       double wd, int step, hipStream_t s);
// Soft minimum of ndet losses per batch item and its weights (d value / d l).
hipError_t launch_softmin(const double* l, int ndet, double beta, double* val, double* w, int batch, hipStream_t s);
hipError_t launch_track_best(const double* loss, double* best, int64_t* since, int batch, hipStream_t s);
// out[j] = sum over i < n of in[i * m + j], in order (FP64).
hipError_t launch_sum_items(const double* in, double* out, int n, int m, hipStream_t s);
// o = [(x^2+y^2) u | x u | y u] on the input grid (three [batch][ny][nx] planes).
template <typename T>
hipError_t launch_czt_dz_prep(const cx<T>* u, cx<T>* o, int nx, int ny, double dx, double dy, double cx0, double cy0,
                              int batch, hipStream_t s);
// out[b] = Re sum conj(g) dU/dz from U = C[u] and Tt = [C[(x^2+y^2)u] | C[xu] |
// C[yu]] on the window grid (nx, ny, dX, dY, cX, cY).
template <typename T>
hipError_t launch_czt_dz_reduce(const cx<T>* g, const cx<T>* U, const cx<T>* Tt, int nx, int ny, double dX, double dY,
                                double cX, double cY, double k, double z, double wl, double* out, double* partial,
                                int nblk, int batch, hipStream_t s);
template <typename T>
hipError_t launch_extract_half(const cx<double>* full, cx<T>* q, int Mx, int My, hipStream_t s);

// 1-D zoom-DFT vectors: sum_j a_j exp(i sigma 2 pi beta X_p x_j) with
// x_j = x0 + j dx (n_in), X_p = X0 + p dX (n_out):
//   pre[j]  = exp(i (sigma 2pi beta X0 dx j + sigma pi alpha j^2 + qin x_j^2))
//   post[p] = K/L exp(i (sigma 2pi beta (X0 x0 + x0 dX p) + sigma pi alpha p^2 + qout X_p^2))
//   chirp[m mod L] = exp(-i sigma pi alpha m^2), m in [-(n_in-1), n_out-1]
// with alpha = beta dx dX.  chirp is written in complex128 (to be
// transformed in FP64), pre/post in T.
struct ZoomSpec {
  int sigma;
  double beta, x0, dx, X0, dX, qin, qout;
  double Kre, Kim;
  int n_in, n_out, L;
};
template <typename T>
hipError_t launch_zoom_vectors(const ZoomSpec& zs, cx<T>* pre, cx<T>* post, cx<double>* chirp,
                               hipStream_t s);
template <typename T>
hipError_t launch_convert(const cx<double>* in, cx<T>* out, int64_t n, hipStream_t s);

// ---- elementwise ----
template <typename T>
hipError_t launch_modulate(const cx<T>* in, const T* phase, cx<T>* out, int64_t npix, int batch,
                           int64_t phase_bstride, hipStream_t s, bool conj = false);
template <typename T>
hipError_t launch_phase_grad(const cx<T>* g, const cx<T>* u, T* grad, int64_t npix, int batch,
                             int accumulate, hipStream_t s);
template <typename T>
hipError_t launch_source_gaussian(cx<T>* out, int nx, int ny, double dx, double dy, double cx0,
                                  double cy0, double w0, double amp, double f, double k, int batch,
                                  hipStream_t s);
template <typename T>
hipError_t launch_source_radial(cx<T>* ex, cx<T>* ey, int nx, int ny, double dx, double dy,
                                double cx0, double cy0, double w0, int batch, hipStream_t s);
// out_c = sum_d J[c][d] in_d (J: 2x2 complex, row-major, as complex128)
template <typename T>
hipError_t launch_jones(const cx<T>* ex, const cx<T>* ey, cx<T>* ox, cx<T>* oy, const double* J,
                        int64_t npix, int batch, hipStream_t s);
// Deterministic per-batch sums of Re(conj(gx) (A ex + B ey) + conj(gy)(C ex + D ey))
// for two 2x2 matrices (dJ/deta, dJ/dtheta): out[b*2 + m] (double, device).
template <typename T>
hipError_t launch_jones_grad(const cx<T>* gx, const cx<T>* gy, const cx<T>* ex, const cx<T>* ey,
                             const double* dJ /* 2 x 4 complex */, double* out, double* partial,
                             int nblk, int64_t npix, int batch, hipStream_t s);

// Wave plates with per-batch-item parameters params[b] = (eta, theta)
// (device doubles): out = J out of (ex, ey), or J^H when adjoint; with oy
// null, ox receives the sum of the two output components.
template <typename T>
hipError_t launch_jones_items(const cx<T>* ex, const cx<T>* ey, cx<T>* ox, cx<T>* oy, const double* params,
                              bool adjoint, int64_t npix, int batch, hipStream_t s);
// Per item (dL/deta, dL/dtheta) into out[b*2 + m]; partial: nblk*batch*2 doubles.
template <typename T>
hipError_t launch_jones_items_grad(const cx<T>* gx, const cx<T>* gy, const cx<T>* ex, const cx<T>* ey,
                                   const double* params, double* out, double* partial, int nblk, int64_t npix,
                                   int batch, hipStream_t s);
// Up to three component planes of one port ([batch][npix] each).
struct Planes {
  const void* p[3];
};
// grad[pix] (+)= sum_b Im(g conj(u)) (a phase shared by the batch).
template <typename T>
hipError_t launch_phase_grad_sum(const cx<T>* g, const cx<T>* u, T* grad, int64_t npix, int batch, int accumulate,
                                 hipStream_t s);
// out[k][b] = in[k][b] * scale[b] (device FP64), k < nplanes <= 3.
template <typename T>
hipError_t launch_scale_items(const Planes& in, const Planes& out, int nplanes, const double* scale, int64_t npix,
                              int batch, hipStream_t s);
// Beam splitter with mixing angle alpha[b] (device doubles) per item.
template <typename T>
hipError_t launch_beam_splitter(const Planes& a, const Planes& b, const Planes& c, const Planes& d, int ncomp,
                                bool has_a, bool has_b, const double* alpha, int64_t npix, int batch, hipStream_t s);
// Adjoint; flags: 1 a given, 2 b given, 4 write ga, 8 write gb, 16 write
// dalpha[b] (partial: nblk*batch*2 doubles).
template <typename T>
hipError_t launch_beam_splitter_adj(const Planes& gc, const Planes& gd, const Planes& a, const Planes& b,
                                    const Planes& ga, const Planes& gb, int ncomp, int flags, const double* alpha,
                                    double* dalpha, double* partial, int nblk, int64_t npix, int batch,
                                    hipStream_t s);

// input stage of a plan setup: out = in exp(i phase) exp(-i q r^2) (phase may
// be null, q = k/(2f) of a thin lens or 0), phase batch stride pbs (0 =
// shared); adjoint: g_in = g conj(factor) (if g_in), grad (+)= Im(g conj(u))
// (if grad; grad has the phase's layout).
template <typename T>
hipError_t launch_phase_stage(const cx<T>* in, const T* phase, cx<T>* out, int nx, int ny, double dx, double dy,
                              double cx0, double cy0, double q, int batch, int64_t pbs, hipStream_t s);
template <typename T>
hipError_t launch_phase_stage_adj(const cx<T>* g, const cx<T>* u, const T* phase, cx<T>* g_in, T* grad, int acc,
                                  int nx, int ny, double dx, double dy, double cx0, double cy0, double q, int batch,
                                  int64_t pbs, hipStream_t s);

// focusing pupil map (real 3x2 per sample, 1/sqrt(sz) apodisation folded in)
template <typename T>
hipError_t launch_pupil(const cx<T>* ex, const cx<T>* ey, cx<T>* o0, cx<T>* o1, cx<T>* o2,
                        int nx, int ny, double dx, double dy, double cx0, double cy0, double f,
                        double na, int batch, int64_t out_bstride, bool adjoint, hipStream_t s);

// free-space VCZT helpers
template <typename T>
hipError_t launch_vczt_prep(const cx<T>* ex, const cx<T>* ey, cx<T>* o, int nx, int ny, double dx,
                            double dy, double cx0, double cy0, int batch, hipStream_t s);
template <typename T>
hipError_t launch_vczt_combine(const cx<T>* cxp, const cx<T>* cyp, const cx<T>* c2, cx<T>* ez,
                               int nx, int ny, double dx, double dy, double cx0, double cy0,
                               double z, int batch, hipStream_t s);
// adjoint helpers: gz -> (X gz, Y gz) and final combination
template <typename T>
hipError_t launch_vczt_adj_prep(const cx<T>* gz, cx<T>* xg, cx<T>* yg, int nx, int ny, double dx,
                                double dy, double cx0, double cy0, double z, int batch,
                                hipStream_t s);
template <typename T>
hipError_t launch_vczt_adj_combine(cx<T>* gex, cx<T>* gey, const cx<T>* cxg, const cx<T>* cyg,
                                   const cx<T>* cz, int nx, int ny, double dx, double dy,
                                   double cx0, double cy0, double z, int batch, hipStream_t s);

// spot-size / E_z-fraction loss: per batch item res[b*8 + {0..5}] =
// (loss, sigma2, fz, P, Xbar - cx, Ybar - cy); seeds g_c = 2 E_c dL/dI_c
// (optional).
template <typename T>
hipError_t launch_spot_loss(const cx<T>* ex, const cx<T>* ey, const cx<T>* ez, int nx, int ny,
                            double dx, double dy, double cx0, double cy0, double wavelength,
                            double w_fz, double* res, double* partial, int nblk, cx<T>* gx,
                            cx<T>* gy, cx<T>* gz, int batch, hipStream_t s);

}  // namespace lp
