// Setup generators (RS kernel spectra, chirp vectors) in FP64 and the
// elementwise / reduction kernels of libprop (sources, SLM phase and its
// gradient, Jones matrices, the focusing pupil map, detector losses).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "kernels.hpp"

namespace lp {

template <typename T> __device__ __forceinline__ cx<T> zero() { return mk<T>(T(0), T(0)); }

// --------------------------------------------------- FP64 generators --
static constexpr double kTwoPi = 6.283185307179586476925286766559;
static constexpr double kPi = 3.1415926535897932384626433832795;

__global__ void k_rs_kernel_wrapped(cx<double>* out, int Mx, int My, int nx, int ny, double dx, double dy,
                                    double k, double z, int kind) {
  const int64_t total = (int64_t)Mx * My;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(t / Mx), bcol = (int)(t - (int64_t)a * Mx);
    int oy, ox;
    bool ok = true;
    if (a <= ny - 1) oy = a; else if (a >= My - (ny - 1)) oy = a - My; else { oy = 0; ok = false; }
    if (bcol <= nx - 1) ox = bcol; else if (bcol >= Mx - (nx - 1)) ox = bcol - Mx; else { ox = 0; ok = false; }
    cx<double> h = mk<double>(0.0, 0.0);
    if (ok) {
      const double X = ox * dx, Y = oy * dy;
      const double r2 = X * X + Y * Y + z * z;
      const double r = sqrt(r2);
      double sn, cs;
      sincos(k * r, &sn, &cs);
      double re, im;
      if (kind == 3) {
        // dH/dz = (1/2pi) e^{ikr} [1/r^3 - ik/r^2 + z^2 (k^2/r^3 + 3ik/r^4 - 3/r^5)]
        const double r3 = r2 * r, z2 = z * z;
        const double A = (1.0 + z2 * k * k) / r3 - 3.0 * z2 / (r3 * r2);
        const double B = -k / r2 + 3.0 * k * z2 / (r2 * r2);
        re = (A * cs - B * sn) / kTwoPi;
        im = (A * sn + B * cs) / kTwoPi;
      } else {
        const double pre = z / (kTwoPi * r2);
        // (1/r - i k) e^{ikr}
        re = (cs / r + k * sn) * pre;
        im = (sn / r - k * cs) * pre;
        if (kind == 1) { re *= X / z; im *= X / z; }
        if (kind == 2) { re *= Y / z; im *= Y / z; }
      }
      h = mk<double>(re, im);
    }
    out[t] = h;
  }
}

hipError_t launch_rs_kernel_wrapped(cx<double>* out, int Mx, int My, int nx, int ny, double dx, double dy,
                                    double k, double z, int kind, hipStream_t s) {
  const int64_t total = (int64_t)Mx * My;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_rs_kernel_wrapped, dim3(blocks), dim3(256), 0, s, out, Mx, My, nx, ny, dx, dy, k, z, kind);
  return hipGetLastError();
}

template <typename T>
__global__ void k_extract_half(const cx<double>* full, cx<T>* q, int Mx, int My) {
  const int qh = My / 2 + 1;
  const int64_t total = (int64_t)Mx * qh;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(t / Mx), kx = (int)(t - (int64_t)a * Mx);
    const cx<double> v = full[t];
    q[(int64_t)(kx >> 2) * qh * 4 + a * 4 + (kx & 3)] = mk<T>(T(v.x), T(v.y));
  }
}

template <typename T>
hipError_t launch_extract_half(const cx<double>* full, cx<T>* q, int Mx, int My, hipStream_t s) {
  const int64_t total = (int64_t)Mx * (My / 2 + 1);
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL((k_extract_half<T>), dim3(blocks), dim3(256), 0, s, full, q, Mx, My);
  return hipGetLastError();
}

template <typename T>
__global__ void k_zoom_vectors(ZoomSpec zs, cx<T>* pre, cx<T>* post, cx<double>* chirp) {
  const double alpha = zs.beta * zs.dx * zs.dX;
  const double sg = (double)zs.sigma;
  const int top = max(max(zs.n_in, zs.n_out), zs.L);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < top; t += gridDim.x * blockDim.x) {
    if (t < zs.n_in) {
      const double j = (double)t;
      const double xj = zs.x0 + j * zs.dx;
      const double ph = sg * kTwoPi * zs.beta * zs.X0 * zs.dx * j + sg * kPi * alpha * (j * j) + zs.qin * xj * xj;
      double sn, cs;
      sincos(ph, &sn, &cs);
      pre[t] = mk<T>(T(cs), T(sn));
    }
    if (t < zs.n_out) {
      const double p = (double)t;
      const double Xp = zs.X0 + p * zs.dX;
      const double ph = sg * kTwoPi * zs.beta * (zs.X0 * zs.x0 + zs.x0 * zs.dX * p) + sg * kPi * alpha * (p * p) +
                        zs.qout * Xp * Xp;
      double sn, cs;
      sincos(ph, &sn, &cs);
      const double kr = zs.Kre / zs.L, ki = zs.Kim / zs.L;
      post[t] = mk<T>(T(kr * cs - ki * sn), T(kr * sn + ki * cs));
    }
    if (t < zs.L) {
      double m = 0.0;
      bool ok = true;
      if (t <= zs.n_out - 1) m = (double)t;
      else if (t >= zs.L - (zs.n_in - 1)) m = (double)(t - zs.L);
      else ok = false;
      cx<double> v = mk<double>(0.0, 0.0);
      if (ok) {
        double sn, cs;
        sincos(-sg * kPi * alpha * (m * m), &sn, &cs);
        v = mk<double>(cs, sn);
      }
      chirp[t] = v;
    }
  }
}

template <typename T>
hipError_t launch_zoom_vectors(const ZoomSpec& zs, cx<T>* pre, cx<T>* post, cx<double>* chirp, hipStream_t s) {
  const int top = std::max(std::max(zs.n_in, zs.n_out), zs.L);
  hipLaunchKernelGGL((k_zoom_vectors<T>), dim3((top + 255) / 256), dim3(256), 0, s, zs, pre, post, chirp);
  return hipGetLastError();
}

template <typename T>
__global__ void k_convert(const cx<double>* in, cx<T>* out, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    out[t] = mk<T>(T(in[t].x), T(in[t].y));
}

template <typename T>
hipError_t launch_convert(const cx<double>* in, cx<T>* out, int64_t n, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL((k_convert<T>), dim3(std::max(blocks, 1)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

// ------------------------------------------------------- elementwise --
static int ew_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

template <typename T> __device__ __forceinline__ void sc(T x, T* s, T* c);
template <> __device__ __forceinline__ void sc<float>(float x, float* s, float* c) { sincosf(x, s, c); }
template <> __device__ __forceinline__ void sc<double>(double x, double* s, double* c) { sincos(x, s, c); }

// out = in exp(i phase), or in exp(-i phase) when conj (the adjoint)
template <typename T>
__global__ void k_modulate(const cx<T>* in, const T* phase, cx<T>* out, int64_t npix, int batch, int64_t pbs,
                           int conj) {
  const int64_t total = npix * batch;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = t / npix, i = t - b * npix;
    T sn, cs;
    sc<T>(phase[b * pbs + i], &sn, &cs);
    out[t] = cmul(in[t], mk<T>(cs, conj ? -sn : sn));
  }
}
template <typename T>
hipError_t launch_modulate(const cx<T>* in, const T* phase, cx<T>* out, int64_t npix, int batch, int64_t pbs,
                           hipStream_t s, bool conj) {
  hipLaunchKernelGGL((k_modulate<T>), dim3(ew_blocks(npix * batch)), dim3(256), 0, s, in, phase, out, npix, batch, pbs,
                     conj ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
__global__ void k_phase_grad(const cx<T>* g, const cx<T>* u, T* grad, int64_t total, int accumulate) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> a = g[t], v = u[t];
    const T val = a.y * v.x - a.x * v.y;
    grad[t] = accumulate ? grad[t] + val : val;
  }
}
template <typename T>
hipError_t launch_phase_grad(const cx<T>* g, const cx<T>* u, T* grad, int64_t npix, int batch, int accumulate,
                             hipStream_t s) {
  hipLaunchKernelGGL((k_phase_grad<T>), dim3(ew_blocks(npix * batch)), dim3(256), 0, s, g, u, grad, npix * batch,
                     accumulate);
  return hipGetLastError();
}

// Phase gradient of a phase shared by the batch: grad[pix] (+)= sum over b
// of Im(g conj(u)), the batch summed in a fixed order per pixel (FP64).
template <typename T>
__global__ void k_phase_grad_sum(const cx<T>* g, const cx<T>* u, T* grad, int64_t npix, int batch, int accumulate) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < npix; t += (int64_t)gridDim.x * blockDim.x) {
    double acc = accumulate ? (double)grad[t] : 0.0;
    for (int b = 0; b < batch; ++b) {
      const cx<T> a = g[(int64_t)b * npix + t], v = u[(int64_t)b * npix + t];
      acc += (double)a.y * (double)v.x - (double)a.x * (double)v.y;
    }
    grad[t] = T(acc);
  }
}
template <typename T>
hipError_t launch_phase_grad_sum(const cx<T>* g, const cx<T>* u, T* grad, int64_t npix, int batch, int accumulate,
                                 hipStream_t s) {
  hipLaunchKernelGGL((k_phase_grad_sum<T>), dim3(ew_blocks(npix)), dim3(256), 0, s, g, u, grad, npix, batch,
                     accumulate);
  return hipGetLastError();
}

// out[k] item b = in[k] item b times the real scale[b] (device FP64); out
// may be in (element by element).
template <typename T>
__global__ void k_scale_items(Planes in, Planes out, int nplanes, const double* scale, int64_t npix) {
  const int b = blockIdx.y;
  const T f = T(scale[b]);
  const int64_t off = (int64_t)b * npix;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npix; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k >= nplanes) break;
      const cx<T> v = ((const cx<T>*)in.p[k])[off + i];
      ((cx<T>*)out.p[k])[off + i] = mk<T>(v.x * f, v.y * f);
    }
  }
}
template <typename T>
hipError_t launch_scale_items(const Planes& in, const Planes& out, int nplanes, const double* scale, int64_t npix,
                              int batch, hipStream_t s) {
  const int64_t want = std::max<int64_t>(8, 4096 / std::max(batch, 1));
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((npix + 255) / 256, want));
  hipLaunchKernelGGL((k_scale_items<T>), dim3(nb, batch), dim3(256), 0, s, in, out, nplanes, scale, npix);
  return hipGetLastError();
}

template <typename T>
__global__ void k_source_gaussian(cx<T>* out, int nx, int ny, double dx, double dy, double cx0, double cy0,
                                  double w0, double amp, double f, double k, int batch) {
  const int64_t npix = (int64_t)nx * ny, total = npix * batch;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t % npix;
    const int row = (int)(i / nx), col = (int)(i - (int64_t)row * nx);
    const double x = cx0 + (double)(col - nx / 2) * dx, y = cy0 + (double)(row - ny / 2) * dy;
    const double r2 = x * x + y * y;
    const double a = amp * exp(-r2 / (w0 * w0));
    double re = a, im = 0.0;
    if (f > 0.0) {
      double sn, cs;
      sincos(-k * r2 / (2.0 * f), &sn, &cs);
      re = a * cs;
      im = a * sn;
    }
    out[t] = mk<T>(T(re), T(im));
  }
}
template <typename T>
hipError_t launch_source_gaussian(cx<T>* out, int nx, int ny, double dx, double dy, double cx0, double cy0,
                                  double w0, double amp, double f, double k, int batch, hipStream_t s) {
  hipLaunchKernelGGL((k_source_gaussian<T>), dim3(ew_blocks((int64_t)nx * ny * batch)), dim3(256), 0, s, out, nx,
                     ny, dx, dy, cx0, cy0, w0, amp, f, k, batch);
  return hipGetLastError();
}

template <typename T>
__global__ void k_source_radial(cx<T>* ex, cx<T>* ey, int nx, int ny, double dx, double dy, double cx0,
                                double cy0, double w0, int batch) {
  const int64_t npix = (int64_t)nx * ny, total = npix * batch;
  const double norm = 1.0 / (w0 * exp(-0.5) / sqrt(2.0));
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t % npix;
    const int row = (int)(i / nx), col = (int)(i - (int64_t)row * nx);
    const double x = cx0 + (double)(col - nx / 2) * dx, y = cy0 + (double)(row - ny / 2) * dy;
    const double g = exp(-(x * x + y * y) / (w0 * w0)) * norm;
    ex[t] = mk<T>(T(x * g), T(0));
    ey[t] = mk<T>(T(y * g), T(0));
  }
}
template <typename T>
hipError_t launch_source_radial(cx<T>* ex, cx<T>* ey, int nx, int ny, double dx, double dy, double cx0,
                                double cy0, double w0, int batch, hipStream_t s) {
  hipLaunchKernelGGL((k_source_radial<T>), dim3(ew_blocks((int64_t)nx * ny * batch)), dim3(256), 0, s, ex, ey, nx,
                     ny, dx, dy, cx0, cy0, w0, batch);
  return hipGetLastError();
}

struct J4 { double v[8]; };

template <typename T>
__global__ void k_jones(const cx<T>* ex, const cx<T>* ey, cx<T>* ox, cx<T>* oy, J4 J, int64_t total) {
  const cx<T> a = mk<T>(T(J.v[0]), T(J.v[1])), b = mk<T>(T(J.v[2]), T(J.v[3]));
  const cx<T> c = mk<T>(T(J.v[4]), T(J.v[5])), d = mk<T>(T(J.v[6]), T(J.v[7]));
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> x = ex[t], y = ey[t];
    ox[t] = cadd(cmul(a, x), cmul(b, y));
    oy[t] = cadd(cmul(c, x), cmul(d, y));
  }
}
template <typename T>
hipError_t launch_jones(const cx<T>* ex, const cx<T>* ey, cx<T>* ox, cx<T>* oy, const double* J, int64_t npix,
                        int batch, hipStream_t s) {
  J4 j4;
  for (int i = 0; i < 8; ++i) j4.v[i] = J[i];
  hipLaunchKernelGGL((k_jones<T>), dim3(ew_blocks(npix * batch)), dim3(256), 0, s, ex, ey, ox, oy, j4, npix * batch);
  return hipGetLastError();
}

// fixed-order block reduction of NV doubles
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double* sh /* NV * 256 */) {
  const int t = threadIdx.x;
#pragma unroll
  for (int m = 0; m < NV; ++m) sh[m * 256 + t] = v[m];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int m = 0; m < NV; ++m) sh[m * 256 + t] += sh[m * 256 + t + w];
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < NV; ++m) v[m] = sh[m * 256];
}

struct J8 { double v[16]; };

template <typename T>
__global__ __launch_bounds__(256) void k_jones_grad_partial(const cx<T>* gx, const cx<T>* gy, const cx<T>* ex,
                                                            const cx<T>* ey, J8 dJ, double* partial, int nblk,
                                                            int64_t npix) {
  __shared__ double sh[2 * 256];
  const int b = blockIdx.y;
  double acc[2] = {0.0, 0.0};
  const int64_t off = (int64_t)b * npix;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < npix; i += (int64_t)nblk * 256) {
    const cx<T> x = ex[off + i], y = ey[off + i], g0 = gx[off + i], g1 = gy[off + i];
    const double X[2] = {x.x, x.y}, Y[2] = {y.x, y.y}, G0[2] = {g0.x, g0.y}, G1[2] = {g1.x, g1.y};
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const double* d = dJ.v + 8 * m;
      const double o0r = d[0] * X[0] - d[1] * X[1] + d[2] * Y[0] - d[3] * Y[1];
      const double o0i = d[0] * X[1] + d[1] * X[0] + d[2] * Y[1] + d[3] * Y[0];
      const double o1r = d[4] * X[0] - d[5] * X[1] + d[6] * Y[0] - d[7] * Y[1];
      const double o1i = d[4] * X[1] + d[5] * X[0] + d[6] * Y[1] + d[7] * Y[0];
      acc[m] += G0[0] * o0r + G0[1] * o0i + G1[0] * o1r + G1[1] * o1i;
    }
  }
  block_reduce<2>(acc, sh);
  if (threadIdx.x == 0) {
    partial[((int64_t)b * nblk + blockIdx.x) * 2 + 0] = acc[0];
    partial[((int64_t)b * nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}

__global__ __launch_bounds__(256) void k_sum_partials2(const double* partial, int nblk, double* out) {
  __shared__ double sh[2 * 256];
  const int b = blockIdx.x;
  double acc[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < nblk; i += 256) {
    acc[0] += partial[((int64_t)b * nblk + i) * 2 + 0];
    acc[1] += partial[((int64_t)b * nblk + i) * 2 + 1];
  }
  block_reduce<2>(acc, sh);
  if (threadIdx.x == 0) { out[b * 2 + 0] = acc[0]; out[b * 2 + 1] = acc[1]; }
}

template <typename T>
hipError_t launch_jones_grad(const cx<T>* gx, const cx<T>* gy, const cx<T>* ex, const cx<T>* ey, const double* dJ,
                             double* out, double* partial, int nblk, int64_t npix, int batch, hipStream_t s) {
  J8 j8;
  for (int i = 0; i < 16; ++i) j8.v[i] = dJ[i];
  hipLaunchKernelGGL((k_jones_grad_partial<T>), dim3(nblk, batch), dim3(256), 0, s, gx, gy, ex, ey, j8, partial, nblk,
                     npix);
  hipLaunchKernelGGL(k_sum_partials2, dim3(batch), dim3(256), 0, s, partial, nblk, out);
  return hipGetLastError();
}

// ------------------------------------ wave plates, per-item parameters --
// Jones matrix R(-theta) diag(1, e^{i eta}) R(theta) of one batch item, and
// its derivatives in eta and theta, evaluated on the device from the
// item's (eta, theta) so that optimised parameters never leave HBM.
__device__ __forceinline__ void jones_item(double eta, double theta, double J[8]) {
  double c, s, ei, er;
  sincos(theta, &s, &c);
  sincos(eta, &ei, &er);
  J[0] = c * c + er * s * s; J[1] = ei * s * s;
  J[2] = c * s * (1 - er);   J[3] = -c * s * ei;
  J[4] = J[2];               J[5] = J[3];
  J[6] = s * s + er * c * c; J[7] = ei * c * c;
}

template <typename T>
__global__ void k_jones_items(const cx<T>* ex, const cx<T>* ey, cx<T>* ox, cx<T>* oy, const double* params,
                              int adjoint, int64_t npix) {
  const int bi = blockIdx.y;
  double J[8];
  jones_item(params[2 * bi], params[2 * bi + 1], J);
  if (adjoint) {  // J^H: transpose (J is symmetric) and conjugate
    J[1] = -J[1]; J[3] = -J[3]; J[5] = -J[5]; J[7] = -J[7];
  }
  const cx<T> a = mk<T>(T(J[0]), T(J[1])), b = mk<T>(T(J[2]), T(J[3]));
  const cx<T> c = mk<T>(T(J[4]), T(J[5])), d = mk<T>(T(J[6]), T(J[7]));
  const int64_t off = (int64_t)bi * npix;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npix; i += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> x = ex[off + i], y = ey[off + i];
    const cx<T> u = cadd(cmul(a, x), cmul(b, y)), v = cadd(cmul(c, x), cmul(d, y));
    if (oy) {
      ox[off + i] = u;
      oy[off + i] = v;
    } else {
      ox[off + i] = cadd(u, v);  // both components came from one field
    }
  }
}

// Blocks per batch item of the per-item elementwise passes: enough for
// about 4096 workgroups in all, at most one per 256 pixels.
static int item_blocks(int64_t npix, int batch) {
  const int64_t want = std::max<int64_t>(8, 4096 / std::max(batch, 1));
  return (int)std::max<int64_t>(1, std::min<int64_t>((npix + 255) / 256, want));
}

template <typename T>
hipError_t launch_jones_items(const cx<T>* ex, const cx<T>* ey, cx<T>* ox, cx<T>* oy, const double* params,
                              bool adjoint, int64_t npix, int batch, hipStream_t s) {
  hipLaunchKernelGGL((k_jones_items<T>), dim3(item_blocks(npix, batch), batch), dim3(256), 0, s, ex, ey, ox, oy,
                     params, adjoint ? 1 : 0, npix);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_jones_items_grad(const cx<T>* gx, const cx<T>* gy, const cx<T>* ex,
                                                          const cx<T>* ey, const double* params, double* partial,
                                                          int nblk, int64_t npix) {
  __shared__ double sh[2 * 256];
  const int bi = blockIdx.y;
  const double eta = params[2 * bi], theta = params[2 * bi + 1];
  double c, s, ei, er, s2, c2;
  sincos(theta, &s, &c);
  sincos(eta, &ei, &er);
  sincos(2 * theta, &s2, &c2);
  // dJ/deta = i e [[s^2, -cs], [-cs, c^2]];  dJ/dtheta = (1 - e) [[-s2, c2], [c2, s2]]
  double dJ[16];
  const double m[4] = {s * s, -c * s, -c * s, c * c};
  const double n[4] = {-s2, c2, c2, s2};
  for (int k = 0; k < 4; ++k) {
    dJ[2 * k] = -ei * m[k];
    dJ[2 * k + 1] = er * m[k];
    dJ[8 + 2 * k] = (1 - er) * n[k];
    dJ[8 + 2 * k + 1] = -ei * n[k];
  }
  double acc[2] = {0.0, 0.0};
  const int64_t off = (int64_t)bi * npix;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < npix; i += (int64_t)nblk * 256) {
    const cx<T> x = ex[off + i], y = ey[off + i], g0 = gx[off + i], g1 = gy[off + i];
    const double X[2] = {x.x, x.y}, Y[2] = {y.x, y.y}, G0[2] = {g0.x, g0.y}, G1[2] = {g1.x, g1.y};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double* d = dJ + 8 * q;
      const double o0r = d[0] * X[0] - d[1] * X[1] + d[2] * Y[0] - d[3] * Y[1];
      const double o0i = d[0] * X[1] + d[1] * X[0] + d[2] * Y[1] + d[3] * Y[0];
      const double o1r = d[4] * X[0] - d[5] * X[1] + d[6] * Y[0] - d[7] * Y[1];
      const double o1i = d[4] * X[1] + d[5] * X[0] + d[6] * Y[1] + d[7] * Y[0];
      acc[q] += G0[0] * o0r + G0[1] * o0i + G1[0] * o1r + G1[1] * o1i;
    }
  }
  block_reduce<2>(acc, sh);
  if (threadIdx.x == 0) {
    partial[((int64_t)bi * nblk + blockIdx.x) * 2 + 0] = acc[0];
    partial[((int64_t)bi * nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}

template <typename T>
hipError_t launch_jones_items_grad(const cx<T>* gx, const cx<T>* gy, const cx<T>* ex, const cx<T>* ey,
                                   const double* params, double* out, double* partial, int nblk, int64_t npix,
                                   int batch, hipStream_t s) {
  hipLaunchKernelGGL((k_jones_items_grad<T>), dim3(nblk, batch), dim3(256), 0, s, gx, gy, ex, ey, params, partial,
                     nblk, npix);
  hipLaunchKernelGGL(k_sum_partials2, dim3(batch), dim3(256), 0, s, partial, nblk, out);
  return hipGetLastError();
}

// ------------------------------------------------------- beam splitter --
// Lossless symmetric splitter with mixing angle alpha[b] per batch item, on
// each of ncomp components: c = cos a + i sin b, d = i sin a + cos b.  A
// port flagged absent reads as zero.
template <typename T>
__global__ void k_beam_splitter(Planes a, Planes b, Planes c, Planes d, int ncomp, int has_a, int has_b,
                                const double* alpha, int64_t npix) {
  const int bi = blockIdx.y;
  double sd, cd;
  sincos(alpha[bi], &sd, &cd);
  const T ct = T(cd), st = T(sd);
  const int64_t off = (int64_t)bi * npix;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npix; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k >= ncomp) break;
      const cx<T> x = has_a ? ((const cx<T>*)a.p[k])[off + i] : mk<T>(T(0), T(0));
      const cx<T> y = has_b ? ((const cx<T>*)b.p[k])[off + i] : mk<T>(T(0), T(0));
      ((cx<T>*)c.p[k])[off + i] = mk<T>(ct * x.x - st * y.y, ct * x.y + st * y.x);
      ((cx<T>*)d.p[k])[off + i] = mk<T>(ct * y.x - st * x.y, ct * y.y + st * x.x);
    }
  }
}

template <typename T>
hipError_t launch_beam_splitter(const Planes& a, const Planes& b, const Planes& c, const Planes& d, int ncomp,
                                bool has_a, bool has_b, const double* alpha, int64_t npix, int batch, hipStream_t s) {
  hipLaunchKernelGGL((k_beam_splitter<T>), dim3(item_blocks(npix, batch), batch), dim3(256), 0, s, a, b, c, d, ncomp,
                     has_a ? 1 : 0, has_b ? 1 : 0, alpha, npix);
  return hipGetLastError();
}

// Adjoint: ga = cos gc - i sin gd, gb = -i sin gc + cos gd (when wanted),
// and per block the FP64 partial sums A = Re(conj(gc) a + conj(gd) b),
// B = Im(conj(gc) b + conj(gd) a), from which dL/dalpha = -sin A - cos B.
template <typename T>
__global__ __launch_bounds__(256) void k_beam_splitter_adj(Planes gc, Planes gd, Planes a, Planes b, Planes ga,
                                                           Planes gb, int ncomp, int flags, const double* alpha,
                                                           double* partial, int nblk, int64_t npix) {
  __shared__ double sh[2 * 256];
  const bool has_a = flags & 1, has_b = flags & 2, want_ga = flags & 4, want_gb = flags & 8, want_da = flags & 16;
  const int bi = blockIdx.y;
  double sd, cd;
  sincos(alpha[bi], &sd, &cd);
  const T ct = T(cd), st = T(sd);
  const int64_t off = (int64_t)bi * npix;
  double acc[2] = {0.0, 0.0};
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < npix; i += (int64_t)nblk * 256) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k >= ncomp) break;
      const cx<T> p = ((const cx<T>*)gc.p[k])[off + i], q = ((const cx<T>*)gd.p[k])[off + i];
      if (want_ga) ((cx<T>*)ga.p[k])[off + i] = mk<T>(ct * p.x + st * q.y, ct * p.y - st * q.x);
      if (want_gb) ((cx<T>*)gb.p[k])[off + i] = mk<T>(st * p.y + ct * q.x, ct * q.y - st * p.x);
      if (want_da) {
        const cx<T> x = has_a ? ((const cx<T>*)a.p[k])[off + i] : mk<T>(T(0), T(0));
        const cx<T> y = has_b ? ((const cx<T>*)b.p[k])[off + i] : mk<T>(T(0), T(0));
        const double px = p.x, py = p.y, qx = q.x, qy = q.y;
        acc[0] += px * (double)x.x + py * (double)x.y + qx * (double)y.x + qy * (double)y.y;
        acc[1] += px * (double)y.y - py * (double)y.x + qx * (double)x.y - qy * (double)x.x;
      }
    }
  }
  if (!want_da) return;  // uniform over the grid
  block_reduce<2>(acc, sh);
  if (threadIdx.x == 0) {
    partial[((int64_t)bi * nblk + blockIdx.x) * 2 + 0] = acc[0];
    partial[((int64_t)bi * nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}

__global__ __launch_bounds__(256) void k_beam_splitter_dalpha(const double* partial, int nblk, const double* alpha,
                                                              double* dalpha) {
  __shared__ double sh[2 * 256];
  const int b = blockIdx.x;
  double acc[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < nblk; i += 256) {
    acc[0] += partial[((int64_t)b * nblk + i) * 2 + 0];
    acc[1] += partial[((int64_t)b * nblk + i) * 2 + 1];
  }
  block_reduce<2>(acc, sh);
  if (threadIdx.x == 0) {
    double sd, cd;
    sincos(alpha[b], &sd, &cd);
    dalpha[b] = -sd * acc[0] - cd * acc[1];
  }
}

template <typename T>
hipError_t launch_beam_splitter_adj(const Planes& gc, const Planes& gd, const Planes& a, const Planes& b,
                                    const Planes& ga, const Planes& gb, int ncomp, int flags, const double* alpha,
                                    double* dalpha, double* partial, int nblk, int64_t npix, int batch,
                                    hipStream_t s) {
  hipLaunchKernelGGL((k_beam_splitter_adj<T>), dim3(nblk, batch), dim3(256), 0, s, gc, gd, a, b, ga, gb, ncomp, flags,
                     alpha, partial, nblk, npix);
  if (flags & 16)
    hipLaunchKernelGGL(k_beam_splitter_dalpha, dim3(batch), dim3(256), 0, s, partial, nblk, alpha, dalpha);
  return hipGetLastError();
}

// ---------------------------------------------------- distance gradients --
// Re sum conj(a) b over each batch item's npix elements (FP64, fixed order).
template <typename T>
__global__ __launch_bounds__(256) void k_redot_partial(const cx<T>* a, const cx<T>* b, double* partial, int nblk,
                                                       int64_t npix) {
  __shared__ double sh[256];
  const int bi = blockIdx.y;
  double acc[1] = {0.0};
  const int64_t off = (int64_t)bi * npix;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < npix; i += (int64_t)nblk * 256) {
    const cx<T> x = a[off + i], y = b[off + i];
    acc[0] += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
  }
  block_reduce<1>(acc, sh);
  if (threadIdx.x == 0) partial[(int64_t)bi * nblk + blockIdx.x] = acc[0];
}

__global__ __launch_bounds__(256) void k_sum_partials1(const double* partial, int nblk, double scale, double* out) {
  __shared__ double sh[256];
  const int b = blockIdx.x;
  double acc[1] = {0.0};
  for (int i = threadIdx.x; i < nblk; i += 256) acc[0] += partial[(int64_t)b * nblk + i];
  block_reduce<1>(acc, sh);
  if (threadIdx.x == 0) out[b] = scale * acc[0];
}

template <typename T>
hipError_t launch_redot(const cx<T>* a, const cx<T>* b, double* out, double* partial, int nblk, int64_t npix,
                        int batch, hipStream_t s, double scale) {
  hipLaunchKernelGGL((k_redot_partial<T>), dim3(nblk, batch), dim3(256), 0, s, a, b, partial, nblk, npix);
  hipLaunchKernelGGL(k_sum_partials1, dim3(batch), dim3(256), 0, s, partial, nblk, scale, out);
  return hipGetLastError();
}

// CZT distance gradient, inputs of the three extra transforms:
// o = [ (x^2 + y^2) u | x u | y u ], each [batch][ny][nx].
template <typename T>
__global__ void k_czt_dz_prep(const cx<T>* u, cx<T>* o, int nx, int ny, double dx, double dy, double cx0,
                              double cy0, int64_t plane_b) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < plane_b;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pix = t % ((int64_t)nx * ny);
    const int i = (int)(pix / nx), j = (int)(pix - (int64_t)i * nx);
    const double x = cx0 + (j - nx / 2) * dx, y = cy0 + (i - ny / 2) * dy;
    const cx<T> v = u[t];
    o[t] = cscale(v, (T)(x * x + y * y));
    o[plane_b + t] = cscale(v, (T)x);
    o[2 * plane_b + t] = cscale(v, (T)y);
  }
}

template <typename T>
hipError_t launch_czt_dz_prep(const cx<T>* u, cx<T>* o, int nx, int ny, double dx, double dy, double cx0, double cy0,
                              int batch, hipStream_t s) {
  const int64_t pb = (int64_t)nx * ny * batch;
  hipLaunchKernelGGL((k_czt_dz_prep<T>), dim3(ew_blocks(pb)), dim3(256), 0, s, u, o, nx, ny, dx, dy, cx0, cy0, pb);
  return hipGetLastError();
}

// Per batch item: Re sum conj(g) [a U + c1 T1 + c2 (X T2 + Y T3)] with
// a = -1/z + i (k - k |X|^2 / (2 z^2)), c1 = -i k / (2 z^2),
// c2 = i 2 pi / (lambda z^2) (the z-derivative of the Fresnel sum).
template <typename T>
__global__ __launch_bounds__(256) void k_czt_dz_partial(const cx<T>* g, const cx<T>* U, const cx<T>* Tt, int nx,
                                                        int ny, double dX, double dY, double cX, double cY, double k,
                                                        double z, double wl, double* partial, int nblk,
                                                        int64_t plane_b) {
  __shared__ double sh[256];
  const int bi = blockIdx.y;
  const int64_t npix = (int64_t)nx * ny;
  const int64_t off = (int64_t)bi * npix;
  const double iz2 = 1.0 / (z * z);
  const double c1 = -0.5 * k * iz2;       // times i
  const double c2 = kTwoPi / wl * iz2;    // times i
  double acc[1] = {0.0};
  for (int64_t p = blockIdx.x * 256 + threadIdx.x; p < npix; p += (int64_t)nblk * 256) {
    const int q = (int)(p / nx), pp = (int)(p - (int64_t)q * nx);
    const double X = cX + (pp - nx / 2) * dX, Y = cY + (q - ny / 2) * dY;
    const cx<T> gv = g[off + p], u = U[off + p], t1 = Tt[off + p], t2 = Tt[plane_b + off + p],
                t3 = Tt[2 * plane_b + off + p];
    const double ar = -1.0 / z, ai = k - 0.5 * k * (X * X + Y * Y) * iz2;
    // w = a U + i c1 T1 + i c2 (X T2 + Y T3)
    const double sr = X * t2.x + Y * t3.x, si = X * t2.y + Y * t3.y;
    const double wr = ar * u.x - ai * u.y - c1 * t1.y - c2 * si;
    const double wi = ar * u.y + ai * u.x + c1 * t1.x + c2 * sr;
    acc[0] += (double)gv.x * wr + (double)gv.y * wi;
  }
  block_reduce<1>(acc, sh);
  if (threadIdx.x == 0) partial[(int64_t)bi * nblk + blockIdx.x] = acc[0];
}

template <typename T>
hipError_t launch_czt_dz_reduce(const cx<T>* g, const cx<T>* U, const cx<T>* Tt, int nx, int ny, double dX, double dY,
                                double cX, double cY, double k, double z, double wl, double* out, double* partial,
                                int nblk, int batch, hipStream_t s) {
  const int64_t pb = (int64_t)nx * ny * batch;
  hipLaunchKernelGGL((k_czt_dz_partial<T>), dim3(nblk, batch), dim3(256), 0, s, g, U, Tt, nx, ny, dX, dY, cX, cY, k,
                     z, wl, partial, nblk, pb);
  hipLaunchKernelGGL(k_sum_partials1, dim3(batch), dim3(256), 0, s, partial, nblk, 1.0, out);
  return hipGetLastError();
}

// ------------------------------------------------------ detector losses --
// Threshold-density loss L = Area / I_eps of the intensity of up to three
// field components, optionally STED-modulated by up to three depletion
// components: I_eff = I_ex [1 - beta (1 - exp(-I_dep / I_ex))], 0 where
// I_ex = 0.  Intensities are formed in FP64 without contraction, component
// by component (re^2 + im^2), so that the threshold decisions do not depend
// on instruction selection.
struct Comps {
  const void* p[3];
  int n;
};

template <typename T>
__device__ __forceinline__ double comp_intensity(const Comps& c, int64_t i) {
  double acc = 0.0;
  for (int k = 0; k < c.n; ++k) {
    const cx<T> v = reinterpret_cast<const cx<T>*>(c.p[k])[i];
    const double t = __dadd_rn(__dmul_rn((double)v.x, (double)v.x), __dmul_rn((double)v.y, (double)v.y));
    acc = k == 0 ? t : __dadd_rn(acc, t);
  }
  return acc;
}

__device__ __forceinline__ double sted_eff(double iex, double idep, double beta) {
  if (!(iex > 0.0)) return 0.0;
  return iex * (1.0 - beta * (1.0 - exp(-idep / iex)));
}

template <typename T>
__device__ __forceinline__ double det_intensity(const Comps& ex, const Comps& dep, double beta, int64_t i,
                                                double* iex_out, double* idep_out) {
  const double iex = comp_intensity<T>(ex, i);
  const double idep = dep.n > 0 ? comp_intensity<T>(dep, i) : 0.0;
  *iex_out = iex;
  *idep_out = idep;
  return dep.n > 0 ? sted_eff(iex, idep, beta) : iex;
}

__device__ __forceinline__ double block_max256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  return sh[0];
}

template <typename T>
__global__ __launch_bounds__(256) void k_dens_max(Comps ex, Comps dep, double beta, int64_t npix, int nblk,
                                                  double* pmax) {
  __shared__ double sh[256];
  const int b = blockIdx.y;
  double m = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < npix; i += (int64_t)nblk * 256) {
    double a, d;
    m = fmax(m, det_intensity<T>(ex, dep, beta, (int64_t)b * npix + i, &a, &d));
  }
  const double r = block_max256(m, sh);
  if (threadIdx.x == 0) pmax[(int64_t)b * nblk + blockIdx.x] = r;
}

__device__ __forceinline__ double batch_max(const double* pmax, int nblk, int b) {
  double m = 0.0;
  for (int k = 0; k < nblk; ++k) m = fmax(m, pmax[(int64_t)b * nblk + k]);
  return m;
}

template <typename T>
__global__ __launch_bounds__(256) void k_dens_sum(Comps ex, Comps dep, double beta, double eps, int64_t npix,
                                                  int nblk, const double* pmax, double* psum) {
  __shared__ double sh[2 * 256];
  const int b = blockIdx.y;
  const double thr = eps * batch_max(pmax, nblk, b);
  double acc[2] = {0.0, 0.0};
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < npix; i += (int64_t)nblk * 256) {
    double a, d;
    const double v = det_intensity<T>(ex, dep, beta, (int64_t)b * npix + i, &a, &d);
    if (v > thr && v > 0.0) {
      acc[0] += 1.0;
      acc[1] += v;
    }
  }
  block_reduce<2>(acc, sh);
  if (threadIdx.x == 0) {
    psum[((int64_t)b * nblk + blockIdx.x) * 2 + 0] = acc[0];
    psum[((int64_t)b * nblk + blockIdx.x) * 2 + 1] = acc[1];
  }
}

__global__ __launch_bounds__(256) void k_dens_final(const double* pmax, const double* psum, int nblk, double* res) {
  __shared__ double sh[2 * 256];
  const int b = blockIdx.x;
  double acc[2] = {0.0, 0.0};
  for (int k = threadIdx.x; k < nblk; k += 256) {
    acc[0] += psum[((int64_t)b * nblk + k) * 2 + 0];
    acc[1] += psum[((int64_t)b * nblk + k) * 2 + 1];
  }
  block_reduce<2>(acc, sh);
  if (threadIdx.x == 0) {
    res[b * 4 + 0] = acc[0] / acc[1];
    res[b * 4 + 1] = acc[0];
    res[b * 4 + 2] = acc[1];
    res[b * 4 + 3] = batch_max(pmax, nblk, b);
  }
}

// Seeds g_c = 2 E_c dL/dI_c: dL/dI = -Area / I_eps^2 on the selected pixels,
// chained through the STED partials dI_eff/dI_ex = 1 - beta + beta e^{-r}
// (1 + r), dI_eff/dI_dep = -beta e^{-r} (r = I_dep / I_ex; limits at I_ex = 0).
struct Outs {
  void* p[3];
  int n;
};

template <typename T>
__global__ void k_dens_seed(Comps ex, Comps dep, double beta, double eps, int64_t npix, int batch, const double* res,
                            Outs gex, Outs gdep) {
  const int64_t total = npix * batch;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(t / npix);
    const double area = res[b * 4 + 1], ieps = res[b * 4 + 2], thr = eps * res[b * 4 + 3];
    double iex, idep;
    const double v = det_intensity<T>(ex, dep, beta, t, &iex, &idep);
    const double dldi = (v > thr && v > 0.0) ? -area / (ieps * ieps) : 0.0;
    double pe = 1.0, pd = 0.0;
    if (dep.n > 0) {
      double r, e;
      if (iex > 0.0) {
        r = idep / iex;
        e = exp(-r);
        pe = 1.0 - beta + beta * e * (1.0 + r);
      } else if (idep > 0.0) {
        e = 0.0;
        pe = 1.0 - beta;
      } else {
        e = 1.0;
        pe = 1.0;
      }
      pd = -beta * e;
    }
    for (int k = 0; k < gex.n; ++k) {
      if (!gex.p[k]) continue;
      const cx<T> a = reinterpret_cast<const cx<T>*>(ex.p[k])[t];
      const double f = 2.0 * dldi * pe;
      reinterpret_cast<cx<T>*>(gex.p[k])[t] = mk<T>((T)(f * a.x), (T)(f * a.y));
    }
    for (int k = 0; k < gdep.n; ++k) {
      if (!gdep.p[k]) continue;
      const cx<T> a = reinterpret_cast<const cx<T>*>(dep.p[k])[t];
      const double f = 2.0 * dldi * pd;
      reinterpret_cast<cx<T>*>(gdep.p[k])[t] = mk<T>((T)(f * a.x), (T)(f * a.y));
    }
  }
}

template <typename T>
hipError_t launch_density_loss(const void* const* comps, int ncomp, const void* const* dep, int ndep, double beta,
                               int64_t npix, double eps, double* res, double* scratch, int nblk, void* const* seeds,
                               void* const* dep_seeds, int batch, hipStream_t s) {
  Comps ce{{nullptr, nullptr, nullptr}, ncomp}, cd{{nullptr, nullptr, nullptr}, ndep};
  for (int k = 0; k < ncomp; ++k) ce.p[k] = comps[k];
  for (int k = 0; k < ndep; ++k) cd.p[k] = dep[k];
  double* pmax = scratch;
  double* psum = scratch + (size_t)batch * nblk;
  hipLaunchKernelGGL((k_dens_max<T>), dim3(nblk, batch), dim3(256), 0, s, ce, cd, beta, npix, nblk, pmax);
  hipLaunchKernelGGL((k_dens_sum<T>), dim3(nblk, batch), dim3(256), 0, s, ce, cd, beta, eps, npix, nblk, pmax, psum);
  hipLaunchKernelGGL(k_dens_final, dim3(batch), dim3(256), 0, s, pmax, psum, nblk, res);
  Outs oe{{nullptr, nullptr, nullptr}, seeds ? ncomp : 0}, od{{nullptr, nullptr, nullptr}, dep_seeds ? ndep : 0};
  bool any = false;
  for (int k = 0; k < oe.n; ++k) any |= (oe.p[k] = seeds[k]) != nullptr;
  for (int k = 0; k < od.n; ++k) any |= (od.p[k] = dep_seeds[k]) != nullptr;
  if (any)
    hipLaunchKernelGGL((k_dens_seed<T>), dim3(ew_blocks(npix * batch)), dim3(256), 0, s, ce, cd, beta, eps, npix, batch,
                       res, oe, od);
  return hipGetLastError();
}

// Soft minimum over detectors per batch item: value = m - log(sum exp(-beta
// (l - m))) / beta with m = min l; weights = d value / d l.
__global__ void k_softmin(const double* l, int ndet, double beta, double* val, double* w, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const double* lb = l + (int64_t)b * ndet;
  double m = lb[0];
  for (int i = 1; i < ndet; ++i) m = fmin(m, lb[i]);
  double sum = 0.0;
  for (int i = 0; i < ndet; ++i) sum += exp(-beta * (lb[i] - m));
  val[b] = m - log(sum) / beta;
  if (w)
    for (int i = 0; i < ndet; ++i) w[(int64_t)b * ndet + i] = exp(-beta * (lb[i] - m)) / sum;
}

hipError_t launch_softmin(const double* l, int ndet, double beta, double* val, double* w, int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_softmin, dim3((batch + 63) / 64), dim3(64), 0, s, l, ndet, beta, val, w, batch);
  return hipGetLastError();
}

// ------------------------------------------------------------ optimiser --
// Stopping rule: per batch item, the best objective so far and the number of
// steps since it last fell.  A step improves only when its objective is
// strictly below the best (a NaN objective never improves).
__global__ void k_track_best(const double* loss, double* best, int64_t* since, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const double l = loss[b];
  if (l < best[b]) {
    best[b] = l;
    since[b] = 0;
  } else {
    since[b] = since[b] + 1;
  }
}

hipError_t launch_track_best(const double* loss, double* best, int64_t* since, int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_track_best, dim3((batch + 63) / 64), dim3(64), 0, s, loss, best, since, batch);
  return hipGetLastError();
}

// Adam step with bias correction, in the parameters' precision for the
// moments and FP64 for the scalar factors; weight_decay > 0 adds the
// decoupled (AdamW) decay.  One pass: reads p, g, m, v, writes p, m, v.
template <typename T>
__global__ void k_adam(T* p, const T* g, T* m, T* v, int64_t n, T lr, T b1, T b2, T c1, T c2, T eps, T lrwd) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T gi = g[i];
    const T mi = b1 * m[i] + (T(1) - b1) * gi;
    const T vi = b2 * v[i] + (T(1) - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const T pi = p[i];
    p[i] = pi - lrwd * pi - lr * (mi * c1) / (sqrt(vi * c2) + eps);
  }
}

template <typename T>
hipError_t launch_adam(T* p, const T* g, T* m, T* v, int64_t n, double lr, double b1, double b2, double eps,
                       double wd, int step, hipStream_t s) {
  const double c1 = 1.0 / (1.0 - std::pow(b1, step)), c2 = 1.0 / (1.0 - std::pow(b2, step));
  hipLaunchKernelGGL((k_adam<T>), dim3(ew_blocks(n)), dim3(256), 0, s, p, g, m, v, n, (T)lr, (T)b1, (T)b2, (T)c1,
                     (T)c2, (T)eps, (T)(lr * wd));
  return hipGetLastError();
}

// focusing pupil map
__device__ __forceinline__ bool pupil_coeffs(double x, double y, double f, double na, double m[6]) {
  const double X2 = x * x + y * y;
  const double rmax = f * na;
  if (!(X2 <= rmax * rmax * (1.0 + 1e-9))) {
    for (int i = 0; i < 6; ++i) m[i] = 0.0;
    return false;
  }
  const double sx = x / f, sy = y / f;
  const double sz = sqrt(fmax(1.0 - X2 / (f * f), 0.0));
  const double w = 1.0 / sqrt(sz);
  const double a = 1.0 / (1.0 + sz);
  m[0] = w * (1.0 - sx * sx * a);
  m[1] = w * (-sx * sy * a);
  m[2] = w * (-sx * sy * a);
  m[3] = w * (1.0 - sy * sy * a);
  m[4] = w * (-sx);
  m[5] = w * (-sy);
  return true;
}

template <typename T>
__global__ void k_pupil_fwd(const cx<T>* ex, const cx<T>* ey, cx<T>* o0, cx<T>* o1, cx<T>* o2, int nx, int ny,
                            double dx, double dy, double cx0, double cy0, double f, double na, int batch,
                            int64_t obs) {
  const int64_t npix = (int64_t)nx * ny, total = npix * batch;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = t / npix, i = t - b * npix;
    const int row = (int)(i / nx), col = (int)(i - (int64_t)row * nx);
    const double x = cx0 + (double)(col - nx / 2) * dx, y = cy0 + (double)(row - ny / 2) * dy;
    double m[6];
    pupil_coeffs(x, y, f, na, m);
    const cx<T> a = ex[t], c = ey[t];
    const int64_t o = b * obs + i;
    o0[o] = mk<T>(T(m[0]) * a.x + T(m[1]) * c.x, T(m[0]) * a.y + T(m[1]) * c.y);
    o1[o] = mk<T>(T(m[2]) * a.x + T(m[3]) * c.x, T(m[2]) * a.y + T(m[3]) * c.y);
    o2[o] = mk<T>(T(m[4]) * a.x + T(m[5]) * c.x, T(m[4]) * a.y + T(m[5]) * c.y);
  }
}

template <typename T>
__global__ void k_pupil_adj(cx<T>* gex, cx<T>* gey, const cx<T>* g0, const cx<T>* g1, const cx<T>* g2, int nx,
                            int ny, double dx, double dy, double cx0, double cy0, double f, double na, int batch,
                            int64_t ibs) {
  const int64_t npix = (int64_t)nx * ny, total = npix * batch;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = t / npix, i = t - b * npix;
    const int row = (int)(i / nx), col = (int)(i - (int64_t)row * nx);
    const double x = cx0 + (double)(col - nx / 2) * dx, y = cy0 + (double)(row - ny / 2) * dy;
    double m[6];
    pupil_coeffs(x, y, f, na, m);
    const int64_t o = b * ibs + i;
    const cx<T> a = g0[o], c = g1[o], d = g2[o];
    gex[t] = mk<T>(T(m[0]) * a.x + T(m[2]) * c.x + T(m[4]) * d.x, T(m[0]) * a.y + T(m[2]) * c.y + T(m[4]) * d.y);
    gey[t] = mk<T>(T(m[1]) * a.x + T(m[3]) * c.x + T(m[5]) * d.x, T(m[1]) * a.y + T(m[3]) * c.y + T(m[5]) * d.y);
  }
}

template <typename T>
hipError_t launch_pupil(const cx<T>* ex, const cx<T>* ey, cx<T>* o0, cx<T>* o1, cx<T>* o2, int nx, int ny,
                        double dx, double dy, double cx0, double cy0, double f, double na, int batch,
                        int64_t out_bstride, bool adjoint, hipStream_t s) {
  const int blocks = ew_blocks((int64_t)nx * ny * batch);
  if (!adjoint)
    hipLaunchKernelGGL((k_pupil_fwd<T>), dim3(blocks), dim3(256), 0, s, ex, ey, o0, o1, o2, nx, ny, dx, dy, cx0, cy0,
                       f, na, batch, out_bstride);
  else  // here ex/ey are the outputs and o0..o2 the inputs
    hipLaunchKernelGGL((k_pupil_adj<T>), dim3(blocks), dim3(256), 0, s, const_cast<cx<T>*>(ex),
                       const_cast<cx<T>*>(ey), o0, o1, o2, nx, ny, dx, dy, cx0, cy0, f, na, batch, out_bstride);
  return hipGetLastError();
}

// free-space VCZT helpers
template <typename T>
__global__ void k_vczt_prep(const cx<T>* ex, const cx<T>* ey, cx<T>* o, int nx, int ny, double dx, double dy,
                            double cx0, double cy0, int batch) {
  const int64_t npix = (int64_t)nx * ny, total = npix * batch;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t % npix;
    const int row = (int)(i / nx), col = (int)(i - (int64_t)row * nx);
    const T x = T(cx0 + (double)(col - nx / 2) * dx), y = T(cy0 + (double)(row - ny / 2) * dy);
    const cx<T> a = ex[t], c = ey[t];
    o[t] = mk<T>(x * a.x + y * c.x, x * a.y + y * c.y);
  }
}
template <typename T>
hipError_t launch_vczt_prep(const cx<T>* ex, const cx<T>* ey, cx<T>* o, int nx, int ny, double dx, double dy,
                            double cx0, double cy0, int batch, hipStream_t s) {
  hipLaunchKernelGGL((k_vczt_prep<T>), dim3(ew_blocks((int64_t)nx * ny * batch)), dim3(256), 0, s, ex, ey, o, nx, ny,
                     dx, dy, cx0, cy0, batch);
  return hipGetLastError();
}

template <typename T>
__global__ void k_vczt_combine(const cx<T>* cxp, const cx<T>* cyp, const cx<T>* c2, cx<T>* ez, int nx, int ny,
                               double dx, double dy, double cx0, double cy0, double z, int batch) {
  const int64_t npix = (int64_t)nx * ny, total = npix * batch;
  const T iz = T(1.0 / z);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t % npix;
    const int row = (int)(i / nx), col = (int)(i - (int64_t)row * nx);
    const T X = T(cx0 + (double)(col - nx / 2) * dx), Y = T(cy0 + (double)(row - ny / 2) * dy);
    const cx<T> a = cxp[t], b = cyp[t], c = c2[t];
    ez[t] = mk<T>(-(X * a.x + Y * b.x - c.x) * iz, -(X * a.y + Y * b.y - c.y) * iz);
  }
}
template <typename T>
hipError_t launch_vczt_combine(const cx<T>* cxp, const cx<T>* cyp, const cx<T>* c2, cx<T>* ez, int nx, int ny,
                               double dx, double dy, double cx0, double cy0, double z, int batch, hipStream_t s) {
  hipLaunchKernelGGL((k_vczt_combine<T>), dim3(ew_blocks((int64_t)nx * ny * batch)), dim3(256), 0, s, cxp, cyp, c2, ez,
                     nx, ny, dx, dy, cx0, cy0, z, batch);
  return hipGetLastError();
}

template <typename T>
__global__ void k_vczt_adj_prep(const cx<T>* gz, cx<T>* xg, cx<T>* yg, int nx, int ny, double dx, double dy,
                                double cx0, double cy0, double z, int batch) {
  const int64_t npix = (int64_t)nx * ny, total = npix * batch;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t % npix;
    const int row = (int)(i / nx), col = (int)(i - (int64_t)row * nx);
    const T X = T(cx0 + (double)(col - nx / 2) * dx), Y = T(cy0 + (double)(row - ny / 2) * dy);
    const cx<T> g = gz[t];
    xg[t] = mk<T>(X * g.x, X * g.y);
    yg[t] = mk<T>(Y * g.x, Y * g.y);
  }
}
template <typename T>
hipError_t launch_vczt_adj_prep(const cx<T>* gz, cx<T>* xg, cx<T>* yg, int nx, int ny, double dx, double dy,
                                double cx0, double cy0, double z, int batch, hipStream_t s) {
  hipLaunchKernelGGL((k_vczt_adj_prep<T>), dim3(ew_blocks((int64_t)nx * ny * batch)), dim3(256), 0, s, gz, xg, yg, nx,
                     ny, dx, dy, cx0, cy0, z, batch);
  return hipGetLastError();
}

template <typename T>
__global__ void k_vczt_adj_combine(cx<T>* gex, cx<T>* gey, const cx<T>* cxg, const cx<T>* cyg, const cx<T>* cz,
                                   int nx, int ny, double dx, double dy, double cx0, double cy0, double z, int batch) {
  const int64_t npix = (int64_t)nx * ny, total = npix * batch;
  const T iz = T(1.0 / z);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t % npix;
    const int row = (int)(i / nx), col = (int)(i - (int64_t)row * nx);
    const T x = T(cx0 + (double)(col - nx / 2) * dx), y = T(cy0 + (double)(row - ny / 2) * dy);
    const cx<T> a = cxg[t], b = cyg[t], c = cz[t], ge = gex[t], gf = gey[t];
    gex[t] = mk<T>(ge.x - (a.x - x * c.x) * iz, ge.y - (a.y - x * c.y) * iz);
    gey[t] = mk<T>(gf.x - (b.x - y * c.x) * iz, gf.y - (b.y - y * c.y) * iz);
  }
}
template <typename T>
hipError_t launch_vczt_adj_combine(cx<T>* gex, cx<T>* gey, const cx<T>* cxg, const cx<T>* cyg, const cx<T>* cz,
                                   int nx, int ny, double dx, double dy, double cx0, double cy0, double z, int batch,
                                   hipStream_t s) {
  hipLaunchKernelGGL((k_vczt_adj_combine<T>), dim3(ew_blocks((int64_t)nx * ny * batch)), dim3(256), 0, s, gex, gey,
                     cxg, cyg, cz, nx, ny, dx, dy, cx0, cy0, z, batch);
  return hipGetLastError();
}

// ------------------------------------------------- input phase stage --
// u = in exp(i phase) exp(-i q r^2), q = k / (2 f) (thin lens; q = 0: none).
// The lens phase is evaluated in FP64 (up to thousands of radians).
__device__ __forceinline__ void lens_factor(double q, double x, double y, double* c, double* s) {
  if (q == 0.0) {
    *c = 1.0;
    *s = 0.0;
    return;
  }
  sincos(-q * (x * x + y * y), s, c);
}

template <typename T>
__global__ void k_phase_stage(const cx<T>* in, const T* phase, cx<T>* out, int nx, int ny, double dx, double dy,
                              double cx0, double cy0, double q, int64_t npix, int batch, int64_t pbs) {
  const int64_t total = npix * batch;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = t / npix, i = t - b * npix;
    const int row = (int)(i / nx), col = (int)(i - (int64_t)row * nx);
    double lc, ls;
    lens_factor(q, cx0 + (double)(col - nx / 2) * dx, cy0 + (double)(row - ny / 2) * dy, &lc, &ls);
    cx<T> f = mk<T>(T(lc), T(ls));
    if (phase) {
      T sn, cs;
      sc<T>(phase[b * pbs + i], &sn, &cs);
      f = cmul(f, mk<T>(cs, sn));
    }
    out[t] = cmul(in[t], f);
  }
}

template <typename T>
__global__ void k_phase_stage_adj(const cx<T>* g, const cx<T>* u, const T* phase, cx<T>* g_in, T* grad, int acc,
                                  int nx, int ny, double dx, double dy, double cx0, double cy0, double q,
                                  int64_t npix, int batch, int64_t pbs) {
  const int64_t total = npix * batch;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = t / npix, i = t - b * npix;
    const cx<T> gv = g[t];
    if (g_in) {
      const int row = (int)(i / nx), col = (int)(i - (int64_t)row * nx);
      double lc, ls;
      lens_factor(q, cx0 + (double)(col - nx / 2) * dx, cy0 + (double)(row - ny / 2) * dy, &lc, &ls);
      cx<T> f = mk<T>(T(lc), T(ls));
      if (phase) {
        T sn, cs;
        sc<T>(phase[b * pbs + i], &sn, &cs);
        f = cmul(f, mk<T>(cs, sn));
      }
      g_in[t] = cmulc(gv, f);
    }
    if (grad) {
      const cx<T> uv = u[t];
      const T val = gv.y * uv.x - gv.x * uv.y;
      const int64_t gi = b * pbs + i;
      grad[gi] = acc ? grad[gi] + val : val;
    }
  }
}

template <typename T>
hipError_t launch_phase_stage(const cx<T>* in, const T* phase, cx<T>* out, int nx, int ny, double dx, double dy,
                              double cx0, double cy0, double q, int batch, int64_t pbs, hipStream_t s) {
  const int64_t npix = (int64_t)nx * ny;
  hipLaunchKernelGGL((k_phase_stage<T>), dim3(ew_blocks(npix * batch)), dim3(256), 0, s, in, phase, out, nx, ny, dx,
                     dy, cx0, cy0, q, npix, batch, pbs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_phase_stage_adj(const cx<T>* g, const cx<T>* u, const T* phase, cx<T>* g_in, T* grad, int acc,
                                  int nx, int ny, double dx, double dy, double cx0, double cy0, double q, int batch,
                                  int64_t pbs, hipStream_t s) {
  const int64_t npix = (int64_t)nx * ny;
  hipLaunchKernelGGL((k_phase_stage_adj<T>), dim3(ew_blocks(npix * batch)), dim3(256), 0, s, g, u, phase, g_in, grad,
                     acc, nx, ny, dx, dy, cx0, cy0, q, npix, batch, pbs);
  return hipGetLastError();
}

// --------------------------------------------------- batch reductions --
// out[j] = sum_i in[i * m + j] over i = 0..n-1, in order (FP64): per-item
// gradients of a parameter shared by the batch.
__global__ void k_sum_items(const double* in, double* out, int n, int m) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += in[(int64_t)i * m + j];
    out[j] = acc;
  }
}

hipError_t launch_sum_items(const double* in, double* out, int n, int m, hipStream_t s) {
  const int blocks = std::max(1, std::min((m + 255) / 256, 1024));
  hipLaunchKernelGGL(k_sum_items, dim3(blocks), dim3(256), 0, s, in, out, n, m);
  return hipGetLastError();
}

// ---------------------------------------------------------- spot loss --
template <typename T>
__global__ __launch_bounds__(256) void k_spot_partial(const cx<T>* ex, const cx<T>* ey, const cx<T>* ez, int nx,
                                                      int ny, double dx, double dy, double* partial, int nblk) {
  __shared__ double sh[5 * 256];
  const int b = blockIdx.y;
  const int64_t npix = (int64_t)nx * ny, off = (int64_t)b * npix;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < npix; i += (int64_t)nblk * 256) {
    const int row = (int)(i / nx), col = (int)(i - (int64_t)row * nx);
    const double X = (double)(col - nx / 2) * dx, Y = (double)(row - ny / 2) * dy;
    const cx<T> a = ex[off + i], c = ey[off + i];
    double Iz = 0.0;
    if (ez) { const cx<T> e = ez[off + i]; Iz = (double)e.x * e.x + (double)e.y * e.y; }
    const double I = (double)a.x * a.x + (double)a.y * a.y + (double)c.x * c.x + (double)c.y * c.y + Iz;
    acc[0] += I;
    acc[1] += I * X;
    acc[2] += I * Y;
    acc[3] += I * (X * X + Y * Y);
    acc[4] += Iz;
  }
  block_reduce<5>(acc, sh);
  if (threadIdx.x == 0)
    for (int m = 0; m < 5; ++m) partial[((int64_t)b * nblk + blockIdx.x) * 5 + m] = acc[m];
}

__global__ __launch_bounds__(256) void k_spot_final(const double* partial, int nblk, double wavelength, double w_fz,
                                                    double* res) {
  __shared__ double sh[5 * 256];
  const int b = blockIdx.x;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < nblk; i += 256)
    for (int m = 0; m < 5; ++m) acc[m] += partial[((int64_t)b * nblk + i) * 5 + m];
  block_reduce<5>(acc, sh);
  if (threadIdx.x == 0) {
    const double P = acc[0];
    const double xb = acc[1] / P, yb = acc[2] / P;
    const double s2 = acc[3] / P - xb * xb - yb * yb;
    const double fz = acc[4] / P;
    double* r = res + 8 * b;
    r[0] = s2 / (wavelength * wavelength) + w_fz * fz;
    r[1] = s2;
    r[2] = fz;
    r[3] = P;
    r[4] = xb;
    r[5] = yb;
    r[6] = 0.0;
    r[7] = 0.0;
  }
}

template <typename T>
__global__ void k_spot_seed(const cx<T>* ex, const cx<T>* ey, const cx<T>* ez, cx<T>* gx, cx<T>* gy, cx<T>* gz,
                            int nx, int ny, double dx, double dy, double wavelength, double w_fz, const double* res,
                            int batch) {
  const int64_t npix = (int64_t)nx * ny, total = npix * batch;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = t / npix, i = t - b * npix;
    const double* r = res + 8 * b;
    const double P = r[3], s2 = r[1], fz = r[2], xb = r[4], yb = r[5];
    const int row = (int)(i / nx), col = (int)(i - (int64_t)row * nx);
    const double X = (double)(col - nx / 2) * dx - xb, Y = (double)(row - ny / 2) * dy - yb;
    const double dI = (X * X + Y * Y - s2) / (P * wavelength * wavelength);
    const double dxy = 2.0 * (dI - w_fz * fz / P);
    const T ct = T(dxy);
    const cx<T> a = ex[t], c = ey[t];
    gx[t] = mk<T>(ct * a.x, ct * a.y);
    gy[t] = mk<T>(ct * c.x, ct * c.y);
    if (ez && gz) {
      const T cz = T(2.0 * (dI + w_fz * (1.0 - fz) / P));
      const cx<T> e = ez[t];
      gz[t] = mk<T>(cz * e.x, cz * e.y);
    }
  }
}

template <typename T>
hipError_t launch_spot_loss(const cx<T>* ex, const cx<T>* ey, const cx<T>* ez, int nx, int ny, double dx, double dy,
                            double cx0, double cy0, double wavelength, double w_fz, double* res, double* partial,
                            int nblk, cx<T>* gx, cx<T>* gy, cx<T>* gz, int batch, hipStream_t s) {
  (void)cx0;
  (void)cy0;  // moments are taken relative to the window centre
  hipLaunchKernelGGL((k_spot_partial<T>), dim3(nblk, batch), dim3(256), 0, s, ex, ey, ez, nx, ny, dx, dy, partial,
                     nblk);
  hipLaunchKernelGGL(k_spot_final, dim3(batch), dim3(256), 0, s, partial, nblk, wavelength, w_fz, res);
  if (gx && gy)
    hipLaunchKernelGGL((k_spot_seed<T>), dim3(ew_blocks((int64_t)nx * ny * batch)), dim3(256), 0, s, ex, ey, ez, gx,
                       gy, gz, nx, ny, dx, dy, wavelength, w_fz, res, batch);
  return hipGetLastError();
}

// ------------------------------------------------------ instantiations --
#define LP_INST(T)                                                                                                  \
  template hipError_t launch_extract_half<T>(const cx<double>*, cx<T>*, int, int, hipStream_t);                  \
  template hipError_t launch_redot<T>(const cx<T>*, const cx<T>*, double*, double*, int, int64_t, int, hipStream_t,   \
                                      double);                                                                      \
  template hipError_t launch_adam<T>(T*, const T*, T*, T*, int64_t, double, double, double, double, double, int,   \
                                     hipStream_t);                                                                  \
  template hipError_t launch_density_loss<T>(const void* const*, int, const void* const*, int, double, int64_t,     \
                                             double, double*, double*, int, void* const*, void* const*, int,       \
                                             hipStream_t);                                                          \
  template hipError_t launch_czt_dz_prep<T>(const cx<T>*, cx<T>*, int, int, double, double, double, double, int,   \
                                            hipStream_t);                                                           \
  template hipError_t launch_czt_dz_reduce<T>(const cx<T>*, const cx<T>*, const cx<T>*, int, int, double, double,  \
                                              double, double, double, double, double, double*, double*, int, int,  \
                                              hipStream_t);                                                         \
  template hipError_t launch_zoom_vectors<T>(const ZoomSpec&, cx<T>*, cx<T>*, cx<double>*, hipStream_t);            \
  template hipError_t launch_convert<T>(const cx<double>*, cx<T>*, int64_t, hipStream_t);                           \
  template hipError_t launch_phase_stage<T>(const cx<T>*, const T*, cx<T>*, int, int, double, double, double,       \
                                            double, double, int, int64_t, hipStream_t);                             \
  template hipError_t launch_phase_stage_adj<T>(const cx<T>*, const cx<T>*, const T*, cx<T>*, T*, int, int, int,   \
                                                double, double, double, double, double, int, int64_t, hipStream_t); \
  template hipError_t launch_modulate<T>(const cx<T>*, const T*, cx<T>*, int64_t, int, int64_t, hipStream_t, bool); \
  template hipError_t launch_phase_grad<T>(const cx<T>*, const cx<T>*, T*, int64_t, int, int, hipStream_t);         \
  template hipError_t launch_phase_grad_sum<T>(const cx<T>*, const cx<T>*, T*, int64_t, int, int, hipStream_t);     \
  template hipError_t launch_scale_items<T>(const Planes&, const Planes&, int, const double*, int64_t, int,     \
                                            hipStream_t);                                                           \
  template hipError_t launch_source_gaussian<T>(cx<T>*, int, int, double, double, double, double, double, double,  \
                                                double, double, int, hipStream_t);                                  \
  template hipError_t launch_source_radial<T>(cx<T>*, cx<T>*, int, int, double, double, double, double, double,    \
                                              int, hipStream_t);                                                    \
  template hipError_t launch_jones<T>(const cx<T>*, const cx<T>*, cx<T>*, cx<T>*, const double*, int64_t, int,     \
                                      hipStream_t);                                                                 \
  template hipError_t launch_jones_grad<T>(const cx<T>*, const cx<T>*, const cx<T>*, const cx<T>*, const double*, \
                                           double*, double*, int, int64_t, int, hipStream_t);                       \
  template hipError_t launch_jones_items<T>(const cx<T>*, const cx<T>*, cx<T>*, cx<T>*, const double*, bool,       \
                                            int64_t, int, hipStream_t);                                             \
  template hipError_t launch_jones_items_grad<T>(const cx<T>*, const cx<T>*, const cx<T>*, const cx<T>*,           \
                                                 const double*, double*, double*, int, int64_t, int, hipStream_t);  \
  template hipError_t launch_beam_splitter<T>(const Planes&, const Planes&, const Planes&, const Planes&, int, bool, \
                                              bool, const double*, int64_t, int, hipStream_t);                      \
  template hipError_t launch_beam_splitter_adj<T>(const Planes&, const Planes&, const Planes&, const Planes&,      \
                                                  const Planes&, const Planes&, int, int, const double*, double*,  \
                                                  double*, int, int64_t, int, hipStream_t);                         \
  template hipError_t launch_pupil<T>(const cx<T>*, const cx<T>*, cx<T>*, cx<T>*, cx<T>*, int, int, double,       \
                                      double, double, double, double, double, int, int64_t, bool, hipStream_t);     \
  template hipError_t launch_vczt_prep<T>(const cx<T>*, const cx<T>*, cx<T>*, int, int, double, double, double,    \
                                          double, int, hipStream_t);                                                \
  template hipError_t launch_vczt_combine<T>(const cx<T>*, const cx<T>*, const cx<T>*, cx<T>*, int, int, double,   \
                                             double, double, double, double, int, hipStream_t);                     \
  template hipError_t launch_vczt_adj_prep<T>(const cx<T>*, cx<T>*, cx<T>*, int, int, double, double, double,      \
                                              double, double, int, hipStream_t);                                    \
  template hipError_t launch_vczt_adj_combine<T>(cx<T>*, cx<T>*, const cx<T>*, const cx<T>*, const cx<T>*, int,    \
                                                 int, double, double, double, double, double, int, hipStream_t);    \
  template hipError_t launch_spot_loss<T>(const cx<T>*, const cx<T>*, const cx<T>*, int, int, double, double,       \
                                          double, double, double, double, double*, double*, int, cx<T>*, cx<T>*,    \
                                          cx<T>*, int, hipStream_t);

LP_INST(float)
LP_INST(double)

}  // namespace lp
