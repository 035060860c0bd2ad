"""FP64 CPU oracle for scalar/vectorial RS and CZT propagation and adjoints.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py``; the library's product path never
calls, links or imports anything here, and nothing here imports the library.

Scope (paper: Methods, "Features and performance"; Software section):
light propagation by the Rayleigh-Sommerfeld (RS) diffraction integral and by
the chirped z-transform (CZT), each scalar and vectorial (VRS, VCZT), the
high-NA objective evaluated with CZT methods, and gradients with respect to
optical parameters (the paper obtains them by reverse-mode autodiff; here the
adjoint of every linear operator is written out).  The paper prints no
propagator formulas; it cites Shen & Wang 2006 (RS), Ye et al. 2013 (VRS) and
Hu et al. 2020 (CZT).  The readings taken where the paper is silent are:

C1 grid: x_j = cx + (j - nx//2)*dx (the origin falls on a sample).
C2 time convention exp(-i w t): outgoing waves exp(+i k r); converging thin
   lens exp(-i k r^2 / 2f); k = 2 pi / lambda; vacuum.
C3 Gaussian source A exp(-r^2/w0^2) (w0 = 1/e^2 intensity radius).
C4 radial source E = (x, y) g(r), g = exp(-r^2/w0^2) / (w0 exp(-1/2)/sqrt 2),
   so that max |E_perp| = 1.
C5 gradient convention g = dL/dRe + i dL/dIm; for y = A x, g_x = A^H g_y;
   for U = V exp(i phi), dL/dphi = Im(g_U conj(U)).
C6 global phases are kept as written below (fields compare as complex values).

Every routine here evaluates its plain definition.  Library primitives serve
as steps: ``scipy.signal.fftconvolve`` for the discrete linear convolution of
the RS sums, ``numpy`` matrix products for the separable DFT sums of CZT and
the focusing integral.  There is no padding trick, blocking or fusion beyond
what the definitions state.

Pins: see tests/test_oracle_*.py (brute-force sums, closed forms for the
Gaussian beam, Airy and Gaussian foci, Richards-Wolf 1D integrals, Parseval,
library DFT/CZT routines, dot-product adjoint identities, finite differences).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.signal import fftconvolve

TWO_PI = 2.0 * math.pi
C128 = np.complex128


# --------------------------------------------------------------------------
# Grid (C1)
# --------------------------------------------------------------------------

def axis(n: int, d: float, c: float = 0.0) -> np.ndarray:
    """Sample positions c + (j - n//2) d, j = 0..n-1."""
    return c + (np.arange(n, dtype=np.float64) - (n // 2)) * d


def coords(g):
    """(x[nx], y[ny]) sample positions of grid ``g``."""
    return axis(g.nx, g.dx, g.cx), axis(g.ny, g.dy, g.cy)


def _as_c128(u):
    return np.asarray(u, dtype=C128)


def _batched(fn, u, *rest):
    """Apply a 2-D routine over leading batch dimensions."""
    u = _as_c128(u)
    if u.ndim == 2:
        return fn(u, *rest)
    lead = u.shape[:-2]
    flat = u.reshape((-1,) + u.shape[-2:])
    out = [fn(flat[b], *rest) for b in range(flat.shape[0])]
    return np.stack(out).reshape(lead + out[0].shape)


# --------------------------------------------------------------------------
# Sources and elementwise elements (Methods: light sources, SLMs, lenses)
# --------------------------------------------------------------------------

def gaussian_beam(g, w0: float, amplitude: float = 1.0, f: float | None = None,
                  wavelength: float | None = None) -> np.ndarray:
    """A exp(-r^2/w0^2) [times the thin-lens phase exp(-i k r^2 / 2f)] (C2, C3)."""
    x, y = coords(g)
    r2 = x[None, :] ** 2 + y[:, None] ** 2
    u = amplitude * np.exp(-r2 / w0 ** 2).astype(C128)
    if f is not None:
        k = TWO_PI / wavelength
        u = u * np.exp(-1j * k * r2 / (2.0 * f))
    return u


def radial_beam(g, w0: float):
    """Radially polarised beam (C4): returns (Ex, Ey)."""
    x, y = coords(g)
    r2 = x[None, :] ** 2 + y[:, None] ** 2
    gn = np.exp(-r2 / w0 ** 2) / (w0 * math.exp(-0.5) / math.sqrt(2.0))
    ex = (x[None, :] * gn).astype(C128)
    ey = (y[:, None] * gn).astype(C128)
    return ex, ey


def modulate(u, phase):
    """SLM: U = V exp(i phi), one free phase per pixel (Methods, SLMs)."""
    return _as_c128(u) * np.exp(1j * np.asarray(phase, dtype=np.float64))


def phase_grad(g_u, u_mod):
    """dL/dphi = Im(g_U conj(U)) for U = V exp(i phi) (C5)."""
    return np.imag(_as_c128(g_u) * np.conj(_as_c128(u_mod)))


def waveplate_matrix(eta: float, theta: float) -> np.ndarray:
    """Jones matrix of a retarder: R(-theta) diag(1, e^{i eta}) R(theta).

    The paper names the retardance eta and angle theta of wave plates
    (Methods; Results, topology discovery) but gives no matrix; the fast
    axis is taken along x at theta = 0.
    """
    c, s = math.cos(theta), math.sin(theta)
    e = complex(math.cos(eta), math.sin(eta))
    return np.array([[c * c + e * s * s, c * s * (1 - e)],
                     [c * s * (1 - e), s * s + e * c * c]], dtype=C128)


def waveplate(ex, ey, eta, theta):
    J = waveplate_matrix(eta, theta)
    ex, ey = _as_c128(ex), _as_c128(ey)
    return J[0, 0] * ex + J[0, 1] * ey, J[1, 0] * ex + J[1, 1] * ey


def waveplate_adjoint(gx, gy, ex, ey, eta, theta):
    """Returns (g_ex, g_ey, dL/deta, dL/dtheta) for out = J(eta,theta) (ex, ey)."""
    J = waveplate_matrix(eta, theta)
    gx, gy, ex, ey = (_as_c128(a) for a in (gx, gy, ex, ey))
    Jh = J.conj().T
    gex = Jh[0, 0] * gx + Jh[0, 1] * gy
    gey = Jh[1, 0] * gx + Jh[1, 1] * gy
    c, s = math.cos(theta), math.sin(theta)
    e = complex(math.cos(eta), math.sin(eta))
    dJ_eta = 1j * e * np.array([[s * s, -c * s], [-c * s, c * c]])
    s2, c2 = math.sin(2 * theta), math.cos(2 * theta)
    dJ_th = (1 - e) * np.array([[-s2, c2], [c2, s2]])

    def dot(dJ):
        ox = dJ[0, 0] * ex + dJ[0, 1] * ey
        oy = dJ[1, 0] * ex + dJ[1, 1] * ey
        return float(np.sum(np.real(np.conj(gx) * ox + np.conj(gy) * oy)))

    return gex, gey, dot(dJ_eta), dot(dJ_th)


# --------------------------------------------------------------------------
# RS: scalar Rayleigh-Sommerfeld (first kind) by discrete convolution
# --------------------------------------------------------------------------

def rs_kernel(X, Y, z: float, wavelength: float):
    """RS-I impulse response H = (1/2pi)(z/r^2)(1/r - ik) e^{ikr}, r = |(X,Y,z)|.

    Equals -(1/2pi) d/dz (e^{ikr}/r) (Shen & Wang, cited by the paper for RS).
    """
    k = TWO_PI / wavelength
    r = np.sqrt(np.asarray(X) ** 2 + np.asarray(Y) ** 2 + z * z)
    return (z / (TWO_PI * r * r)) * (1.0 / r - 1j * k) * np.exp(1j * k * r)


def _offset_axis(n: int, d: float) -> np.ndarray:
    """Output-minus-input offsets -(n-1)..(n-1) times the pitch."""
    return np.arange(-(n - 1), n, dtype=np.float64) * d


def _kernel_on_offsets(g, kern):
    X = _offset_axis(g.nx, g.dx)[None, :]
    Y = _offset_axis(g.ny, g.dy)[:, None]
    return kern(X, Y)


def _lin_conv_same_grid(u, K, g):
    """out[l,m] = sum_{i,j} u[i,j] K[(l-i)+(ny-1), (m-j)+(nx-1)] (linear convolution)."""
    full = fftconvolve(u, K, mode="full")
    return full[g.ny - 1:2 * g.ny - 1, g.nx - 1:2 * g.nx - 1]


def _rs_one(u, g, wavelength, z):
    H = _kernel_on_offsets(g, lambda X, Y: rs_kernel(X, Y, z, wavelength))
    return _lin_conv_same_grid(u, H, g) * (g.dx * g.dy)


def rs_propagate(u, g, wavelength: float, z: float):
    """U(x_m, y_l; z) = dx dy sum_{i,j} U0(x_j, y_i) H(x_m - x_j, y_l - y_i; z).

    The output lies on the input grid (rectangle-rule quadrature of the RS-I
    integral).  Leading batch dimensions are allowed.
    """
    return _batched(_rs_one, u, g, wavelength, z)


def _rs_adj_one(gout, g, wavelength, z):
    H = _kernel_on_offsets(g, lambda X, Y: rs_kernel(X, Y, z, wavelength))
    Hadj = np.conj(H[::-1, ::-1])  # kernel at the negated offset, conjugated
    return _lin_conv_same_grid(gout, Hadj, g) * (g.dx * g.dy)


def rs_adjoint(gout, g, wavelength: float, z: float):
    """g_in[i,j] = dx dy sum_{l,m} conj(H(x_m - x_j, y_l - y_i)) g_out[l,m]."""
    return _batched(_rs_adj_one, gout, g, wavelength, z)


def rs_at(u, g, wavelength: float, z: float, pixels):
    """Direct RS sum at selected output pixels [(l, m), ...] (no FFT)."""
    u = _as_c128(u)
    x, y = coords(g)
    out = np.empty(len(pixels), dtype=C128)
    for n, (l, m) in enumerate(pixels):
        H = rs_kernel(x[m] - x[None, :], y[l] - y[:, None], z, wavelength)
        out[n] = np.sum(u * H) * g.dx * g.dy
    return out


def rs_adjoint_at(gout, g, wavelength: float, z: float, pixels):
    """Direct adjoint sum at selected input pixels [(i, j), ...]."""
    gout = _as_c128(gout)
    x, y = coords(g)
    out = np.empty(len(pixels), dtype=C128)
    for n, (i, j) in enumerate(pixels):
        H = rs_kernel(x[None, :] - x[j], y[:, None] - y[i], z, wavelength)
        out[n] = np.sum(np.conj(H) * gout) * g.dx * g.dy
    return out


def rs_sampling_ok(g, wavelength: float, z: float) -> bool:
    """Sampling reading: e^{ikr} must be Nyquist-sampled at the largest offset.

    The paper only asks for "reasonable sampling" and cites an energy
    criterion; this reading warns when 2 dx > lambda and
    z < sqrt((2 L dx / lambda)^2 - L^2) along either axis (L = extent).
    """
    for n, d in ((g.nx, g.dx), (g.ny, g.dy)):
        if 2.0 * d <= wavelength:
            continue
        L = n * d
        zmin = math.sqrt((2.0 * L * d / wavelength) ** 2 - L * L)
        if z < zmin:
            return False
    return True


# --------------------------------------------------------------------------
# VRS: vectorial RS (transversality fixes E_z)
# --------------------------------------------------------------------------

def _vrs_kernels(g, wavelength, z):
    X = _offset_axis(g.nx, g.dx)[None, :]
    Y = _offset_axis(g.ny, g.dy)[:, None]
    H = rs_kernel(X, Y, z, wavelength)
    return H, (X / z) * H, (Y / z) * H


def _vrs_one(ex, ey, g, wavelength, z):
    H, Hx, Hy = _vrs_kernels(g, wavelength, z)
    s = g.dx * g.dy
    Ex = _lin_conv_same_grid(ex, H, g) * s
    Ey = _lin_conv_same_grid(ey, H, g) * s
    Ez = -(_lin_conv_same_grid(ex, Hx, g) + _lin_conv_same_grid(ey, Hy, g)) * s
    return Ex, Ey, Ez


def vrs_at(ex, ey, g, wavelength: float, z: float, pixels):
    """Direct VRS sums at selected output pixels [(l, m), ...] (no FFT):
    (E_x, E_y, E_z) with E_z = -dx dy sum [E_x0 (x_m - x')/z + E_y0 (y_l - y')/z] H."""
    ex, ey = _as_c128(ex), _as_c128(ey)
    x, y = coords(g)
    s = g.dx * g.dy
    out = np.empty((3, len(pixels)), dtype=C128)
    for n, (l, m) in enumerate(pixels):
        X, Y = x[m] - x[None, :], y[l] - y[:, None]
        H = rs_kernel(X, Y, z, wavelength)
        out[0, n] = np.sum(ex * H) * s
        out[1, n] = np.sum(ey * H) * s
        out[2, n] = -np.sum((ex * X / z + ey * Y / z) * H) * s
    return out[0], out[1], out[2]


def vrs_adjoint_at(gx, gy, gz, g, wavelength: float, z: float, pixels):
    """Direct adjoint VRS sums at selected input pixels [(i, j), ...]:
    g_ex = dx dy sum conj(H) g_x - conj((x - x_j)/z H) g_z, and likewise for g_ey."""
    gx, gy, gz = _as_c128(gx), _as_c128(gy), _as_c128(gz)
    x, y = coords(g)
    s = g.dx * g.dy
    out = np.empty((2, len(pixels)), dtype=C128)
    for n, (i, j) in enumerate(pixels):
        X, Y = x[None, :] - x[j], y[:, None] - y[i]
        Hc = np.conj(rs_kernel(X, Y, z, wavelength))
        out[0, n] = np.sum(Hc * gx - (X / z) * Hc * gz) * s
        out[1, n] = np.sum(Hc * gy - (Y / z) * Hc * gz) * s
    return out[0], out[1]


def vrs_propagate(ex, ey, g, wavelength: float, z: float):
    """E_x, E_y by scalar RS; E_z = -dx dy sum [E_x0 (x-x')/z + E_y0 (y-y')/z] H.

    The E_z kernel follows from div E = 0 applied to the RS-I kernel
    (vectorial RS, Ye et al., cited by the paper).
    """
    ex, ey = _as_c128(ex), _as_c128(ey)
    if ex.ndim == 2:
        return _vrs_one(ex, ey, g, wavelength, z)
    outs = [_vrs_one(a, b, g, wavelength, z) for a, b in
            zip(ex.reshape((-1,) + ex.shape[-2:]), ey.reshape((-1,) + ey.shape[-2:]))]
    return tuple(np.stack([o[c] for o in outs]).reshape(ex.shape) for c in range(3))


def _vrs_adj_one(gx, gy, gz, g, wavelength, z):
    H, Hx, Hy = _vrs_kernels(g, wavelength, z)
    flip = lambda K: np.conj(K[::-1, ::-1])
    s = g.dx * g.dy
    gex = (_lin_conv_same_grid(gx, flip(H), g) - _lin_conv_same_grid(gz, flip(Hx), g)) * s
    gey = (_lin_conv_same_grid(gy, flip(H), g) - _lin_conv_same_grid(gz, flip(Hy), g)) * s
    return gex, gey


def vrs_adjoint(gx, gy, gz, g, wavelength: float, z: float):
    gx, gy, gz = _as_c128(gx), _as_c128(gy), _as_c128(gz)
    if gx.ndim == 2:
        return _vrs_adj_one(gx, gy, gz, g, wavelength, z)
    sh = gx.shape
    f = lambda a: a.reshape((-1,) + sh[-2:])
    outs = [_vrs_adj_one(a, b, c, g, wavelength, z) for a, b, c in zip(f(gx), f(gy), f(gz))]
    return tuple(np.stack([o[c] for o in outs]).reshape(sh) for c in range(2))


# --------------------------------------------------------------------------
# CZT: Fresnel diffraction integral sampled on an arbitrary output window
# --------------------------------------------------------------------------

def czt_factors(g_in, win, wavelength: float, z: float):
    """Separable pieces of the Fresnel integral on window ``win``.

    U(X_p, Y_q) = K P_y[q] P_x[p] sum_{i,j} A_y[q,i] A_x[p,j] Q_y[i] Q_x[j] U0[i,j]
    with K = e^{ikz} dx dy / (i lambda z), Q = e^{ik x^2/2z}, P = e^{ik X^2/2z},
    A_x[p,j] = e^{-i 2 pi X_p x_j / (lambda z)}.
    """
    k = TWO_PI / wavelength
    x, y = coords(g_in)
    X, Y = coords(win)
    K = np.exp(1j * k * z) * g_in.dx * g_in.dy / (1j * wavelength * z)
    Qx, Qy = np.exp(1j * k * x ** 2 / (2 * z)), np.exp(1j * k * y ** 2 / (2 * z))
    Px, Py = np.exp(1j * k * X ** 2 / (2 * z)), np.exp(1j * k * Y ** 2 / (2 * z))
    Ax = np.exp(-1j * TWO_PI * np.outer(X, x) / (wavelength * z))
    Ay = np.exp(-1j * TWO_PI * np.outer(Y, y) / (wavelength * z))
    return K, Qx, Qy, Px, Py, Ax, Ay


def _czt_one(u, g_in, win, wavelength, z):
    K, Qx, Qy, Px, Py, Ax, Ay = czt_factors(g_in, win, wavelength, z)
    v = u * Qy[:, None] * Qx[None, :]
    return K * Py[:, None] * Px[None, :] * (Ay @ v @ Ax.T)


def czt_propagate(u, g_in, win, wavelength: float, z: float):
    """Fresnel propagation onto an arbitrary window (position and pitch).

    Reading of the paper's CZT (Methods: "arbitrary selection and sampling of
    the region of interest"; Hu et al. 2020): the Fresnel diffraction integral
    evaluated as a zoom DFT.  The plain definition is the separable sum in
    ``czt_factors``; it is evaluated here by two matrix products.
    """
    return _batched(_czt_one, u, g_in, win, wavelength, z)


def _czt_adj_one(gout, g_in, win, wavelength, z):
    K, Qx, Qy, Px, Py, Ax, Ay = czt_factors(g_in, win, wavelength, z)
    w = np.conj(K * Py[:, None] * Px[None, :]) * gout
    v = Ay.conj().T @ w @ Ax.conj()
    return v * np.conj(Qy)[:, None] * np.conj(Qx)[None, :]


def czt_adjoint(gout, g_in, win, wavelength: float, z: float):
    """Exact adjoint of ``czt_propagate`` (window grid -> input grid)."""
    return _batched(_czt_adj_one, gout, g_in, win, wavelength, z)


def czt_at(u, g_in, win, wavelength: float, z: float, pixels):
    """Direct Fresnel sum at selected window pixels [(q, p), ...]."""
    u = _as_c128(u)
    k = TWO_PI / wavelength
    x, y = coords(g_in)
    X, Y = coords(win)
    K = np.exp(1j * k * z) * g_in.dx * g_in.dy / (1j * wavelength * z)
    out = np.empty(len(pixels), dtype=C128)
    for n, (q, p) in enumerate(pixels):
        ph = (k * (x[None, :] ** 2 + y[:, None] ** 2) / (2 * z)
              - TWO_PI * (X[p] * x[None, :] + Y[q] * y[:, None]) / (wavelength * z))
        out[n] = K * np.exp(1j * k * (X[p] ** 2 + Y[q] ** 2) / (2 * z)) * np.sum(u * np.exp(1j * ph))
    return out


def czt_adjoint_at(gout, g_in, win, wavelength: float, z: float, pixels):
    """Direct adjoint sum at selected input pixels [(i, j), ...]."""
    gout = _as_c128(gout)
    k = TWO_PI / wavelength
    x, y = coords(g_in)
    X, Y = coords(win)
    K = np.exp(1j * k * z) * g_in.dx * g_in.dy / (1j * wavelength * z)
    out = np.empty(len(pixels), dtype=C128)
    for n, (i, j) in enumerate(pixels):
        ph = (k * (X[None, :] ** 2 + Y[:, None] ** 2 + x[j] ** 2 + y[i] ** 2) / (2 * z)
              - TWO_PI * (X[None, :] * x[j] + Y[:, None] * y[i]) / (wavelength * z))
        out[n] = np.conj(K) * np.sum(np.exp(-1j * ph) * gout)
    return out


# --------------------------------------------------------------------------
# VCZT, free space: the VRS E_z kernel in Fresnel form
# --------------------------------------------------------------------------

def vczt_propagate(ex, ey, g_in, win, wavelength: float, z: float):
    """E_x = C[E_x0], E_y = C[E_y0],
    E_z = -(1/z) (X C[E_x0] + Y C[E_y0] - C[x E_x0 + y E_y0]).

    Obtained by putting the VRS E_z kernel ((X - x)/z) H into the Fresnel
    form of the CZT operator C.
    """
    x, y = coords(g_in)
    X, Y = coords(win)
    ex, ey = _as_c128(ex), _as_c128(ey)
    C = lambda u: czt_propagate(u, g_in, win, wavelength, z)
    cx, cy = C(ex), C(ey)
    c2 = C(x[None, :] * ex + y[:, None] * ey)
    ez = -(X[None, :] * cx + Y[:, None] * cy - c2) / z
    return cx, cy, ez


def vczt_adjoint(gx, gy, gz, g_in, win, wavelength: float, z: float):
    x, y = coords(g_in)
    X, Y = coords(win)
    gx, gy, gz = _as_c128(gx), _as_c128(gy), _as_c128(gz)
    Ch = lambda g: czt_adjoint(g, g_in, win, wavelength, z)
    cz = Ch(gz)
    gex = Ch(gx) - (Ch(X[None, :] * gz) - x[None, :] * cz) / z
    gey = Ch(gy) - (Ch(Y[:, None] * gz) - y[:, None] * cz) / z
    return gex, gey


# --------------------------------------------------------------------------
# VCZT, focusing: high-NA objective (Richards-Wolf / Debye) evaluated by CZT
# --------------------------------------------------------------------------

def rw_pupil(g_in, na: float, f: float):
    """Direction cosines and the aperture for pupil samples.

    Pupil sample (x, y) maps to s_perp = (x, y)/f, s_z = sqrt(1 - |s_perp|^2);
    the aperture keeps x^2 + y^2 <= (f NA)^2 (FP64 test with a 1e-9 relative
    margin so that samples on the rim are kept on both sides of any rounding).
    """
    x, y = coords(g_in)
    X2 = x[None, :] ** 2 + y[:, None] ** 2
    inside = X2 <= (f * na) ** 2 * (1.0 + 1e-9)
    sx = np.broadcast_to(x[None, :] / f, X2.shape)
    sy = np.broadcast_to(y[:, None] / f, X2.shape)
    sz = np.sqrt(np.clip(1.0 - X2 / f ** 2, 0.0, None))
    return sx, sy, sz, inside


def rw_pupil_matrix(g_in, na: float, f: float):
    """Real 3x2 map per pupil sample: E_inf / s_z = M (E_x0, E_y0).

    E_inf = sqrt(s_z) [(E0.n_phi) n_phi + (E0.n_rho) n_theta] (aplanatic
    apodisation, Novotny & Hecht), written without phi:
    (E0.n_phi) n_phi + (E0.n_rho) n_theta =
      (Ex (1 - sx^2/(1+sz)) - Ey sx sy/(1+sz),
       -Ex sx sy/(1+sz) + Ey (1 - sy^2/(1+sz)),
       -(sx Ex + sy Ey)).
    The 1/s_z of the angular-spectrum measure is folded in.
    """
    sx, sy, sz, inside = rw_pupil(g_in, na, f)
    w = np.where(inside, 1.0 / np.sqrt(np.where(inside, sz, 1.0)), 0.0)
    a = 1.0 / (1.0 + sz)
    M = np.empty((3, 2) + sx.shape)
    M[0, 0] = w * (1 - sx * sx * a)
    M[0, 1] = w * (-sx * sy * a)
    M[1, 0] = w * (-sx * sy * a)
    M[1, 1] = w * (1 - sy * sy * a)
    M[2, 0] = w * (-sx)
    M[2, 1] = w * (-sy)
    return M


def rw_factors(g_in, win, wavelength: float, f: float):
    """E(X,Y) = K sum_pupil (E_inf/s_z) e^{ik(s_x X + s_y Y)} with
    K = (i k f e^{-ikf} / 2pi) dx dy / f^2 (Novotny & Hecht prefactor)."""
    k = TWO_PI / wavelength
    x, y = coords(g_in)
    X, Y = coords(win)
    K = 1j * k * f * np.exp(-1j * k * f) / TWO_PI * (g_in.dx * g_in.dy) / (f * f)
    Bx = np.exp(1j * k * np.outer(X, x) / f)
    By = np.exp(1j * k * np.outer(Y, y) / f)
    return K, Bx, By


def _rw_one(ex, ey, g_in, win, wavelength, na, f):
    M = rw_pupil_matrix(g_in, na, f)
    K, Bx, By = rw_factors(g_in, win, wavelength, f)
    return tuple(K * (By @ (M[c, 0] * ex + M[c, 1] * ey) @ Bx.T) for c in range(3))


def vczt_focus(ex, ey, g_in, win, wavelength: float, na: float, f: float):
    """Focal field (E_x, E_y, E_z) of an aplanatic objective (NA, f) on ``win``.

    The paper's high-NA objective "with CZT methods" (Methods); reading:
    Richards-Wolf/Debye integral, the pupil is the input grid.
    """
    ex, ey = _as_c128(ex), _as_c128(ey)
    if ex.ndim == 2:
        return _rw_one(ex, ey, g_in, win, wavelength, na, f)
    outs = [_rw_one(a, b, g_in, win, wavelength, na, f) for a, b in
            zip(ex.reshape((-1,) + ex.shape[-2:]), ey.reshape((-1,) + ey.shape[-2:]))]
    return tuple(np.stack([o[c] for o in outs]).reshape(ex.shape[:-2] + outs[0][c].shape) for c in range(3))


def _rw_adj_one(gx, gy, gz, g_in, win, wavelength, na, f):
    M = rw_pupil_matrix(g_in, na, f)
    K, Bx, By = rw_factors(g_in, win, wavelength, f)
    w = [np.conj(K) * (By.conj().T @ gc @ Bx.conj()) for gc in (gx, gy, gz)]
    gex = M[0, 0] * w[0] + M[1, 0] * w[1] + M[2, 0] * w[2]
    gey = M[0, 1] * w[0] + M[1, 1] * w[1] + M[2, 1] * w[2]
    return gex, gey


def vczt_focus_at(ex, ey, g_in, win, wavelength: float, na: float, f: float, pixels):
    """The focal field at selected window pixels [(q, p), ...]: the same
    Richards-Wolf sum as vczt_focus, taken pixel by pixel over the pupil."""
    ex, ey = _as_c128(ex), _as_c128(ey)
    M = rw_pupil_matrix(g_in, na, f)
    k = TWO_PI / wavelength
    x, y = coords(g_in)
    X, Y = coords(win)
    K = 1j * k * f * np.exp(-1j * k * f) / TWO_PI * (g_in.dx * g_in.dy) / (f * f)
    F = [M[c, 0] * ex + M[c, 1] * ey for c in range(3)]
    out = np.empty((3, len(pixels)), dtype=C128)
    for n, (q, p) in enumerate(pixels):
        phase = np.exp(1j * k * (Y[q] * y[:, None] + X[p] * x[None, :]) / f)
        for c in range(3):
            out[c, n] = K * np.sum(F[c] * phase)
    return out[0], out[1], out[2]


def vczt_focus_adjoint_at(gx, gy, gz, g_in, win, wavelength: float, na: float, f: float, pixels):
    """The focus adjoint at selected pupil pixels [(i, j), ...]."""
    gs = [_as_c128(a) for a in (gx, gy, gz)]
    M = rw_pupil_matrix(g_in, na, f)
    k = TWO_PI / wavelength
    x, y = coords(g_in)
    X, Y = coords(win)
    K = 1j * k * f * np.exp(-1j * k * f) / TWO_PI * (g_in.dx * g_in.dy) / (f * f)
    out = np.empty((2, len(pixels)), dtype=C128)
    for n, (i, j) in enumerate(pixels):
        phase = np.exp(-1j * k * (Y[:, None] * y[i] + X[None, :] * x[j]) / f)
        w = [np.conj(K) * np.sum(gc * phase) for gc in gs]
        out[0, n] = M[0, 0][i, j] * w[0] + M[1, 0][i, j] * w[1] + M[2, 0][i, j] * w[2]
        out[1, n] = M[0, 1][i, j] * w[0] + M[1, 1][i, j] * w[1] + M[2, 1][i, j] * w[2]
    return out[0], out[1]


def vczt_focus_adjoint(gx, gy, gz, g_in, win, wavelength: float, na: float, f: float):
    gx, gy, gz = _as_c128(gx), _as_c128(gy), _as_c128(gz)
    if gx.ndim == 2:
        return _rw_adj_one(gx, gy, gz, g_in, win, wavelength, na, f)
    sh = gx.shape
    r = lambda a: a.reshape((-1,) + sh[-2:])
    outs = [_rw_adj_one(a, b, c, g_in, win, wavelength, na, f) for a, b, c in zip(r(gx), r(gy), r(gz))]
    return tuple(np.stack([o[c] for o in outs]).reshape(sh[:-2] + outs[0][c].shape) for c in range(2))


# --------------------------------------------------------------------------
# Detector side: intensity, spot size, E_z fraction, gradient seeds
# --------------------------------------------------------------------------

def intensity(*fields):
    return sum(np.abs(_as_c128(e)) ** 2 for e in fields)


def spot_loss(win, wavelength: float, ex, ey, ez=None, w_fz: float = 0.0):
    """Loss = sigma^2 / lambda^2 + w_fz F_z and its seeds g_c = 2 E_c dL/dI_c.

    sigma^2 = sum I ((X - Xbar)^2 + (Y - Ybar)^2) / P about the intensity
    centroid; F_z = sum |E_z|^2 / P; I = |E_x|^2 + |E_y|^2 + |E_z|^2.
    (Detector losses of the spot-size experiments; the form is a reading.)
    Returns (loss, sigma2, fz, (g_x, g_y, g_z)).
    """
    X, Y = coords(win)
    fields = [_as_c128(ex), _as_c128(ey)] + ([_as_c128(ez)] if ez is not None else [])
    I = intensity(*fields)
    P = I.sum()
    xb = (I * X[None, :]).sum() / P
    yb = (I * Y[:, None]).sum() / P
    d2 = (X[None, :] - xb) ** 2 + (Y[:, None] - yb) ** 2
    s2 = (I * d2).sum() / P
    dLdI = (d2 - s2) / (P * wavelength ** 2)
    fz = 0.0
    if ez is not None:
        Iz = np.abs(fields[2]) ** 2
        fz = Iz.sum() / P
    loss = s2 / wavelength ** 2 + w_fz * fz
    seeds = []
    for c, e in enumerate(fields):
        d = dLdI.copy()
        if ez is not None and w_fz != 0.0:
            d = d + w_fz * ((1.0 if c == 2 else 0.0) - fz) / P
        seeds.append(2.0 * d * e)
    if ez is None:
        seeds.append(None)
    return float(loss), float(s2), float(fz), tuple(seeds)


# --------------------------------------------------------------------------
# Optical table: SLM -> RS -> SLM -> wave plate -> wave plate -> objective
# --------------------------------------------------------------------------

def table_chain(v, phi1, phi2, wp1, wp2, g, win, wavelength: float, z: float, na: float, f: float,
                w_fz: float = 0.0):
    """One parameter set of the virtual optical table and its gradients.

    Both input polarisation components equal ``v`` (linear 45 degree light
    with the 1/sqrt 2 already in ``v``).  Elements in order: SLM phi1, RS over
    z, SLM phi2, wave plate wp1 = (eta, theta), wave plate wp2, high-NA
    objective into ``win``; loss ``spot_loss`` with weight w_fz on F_z
    (Results, discovery of sharp-focus and STED-like setups from SLMs, wave
    plates and a high-NA lens).  Every intermediate is kept; the reverse pass
    applies the adjoint of each element in reverse order (C5).

    Returns (loss, dL/dphi1, dL/dphi2, (dL/deta1, dL/dtheta1), (dL/deta2, dL/dtheta2)).
    """
    v = _as_c128(v)
    u1 = modulate(v, phi1)
    s = rs_propagate(u1, g, wavelength, z)
    a = modulate(s, phi2)
    bx, by = waveplate(a, a, *wp1)
    cx, cy = waveplate(bx, by, *wp2)
    Ex, Ey, Ez = vczt_focus(cx, cy, g, win, wavelength, na, f)
    loss, _, _, (gx, gy, gz) = spot_loss(win, wavelength, Ex, Ey, Ez, w_fz=w_fz)
    gcx, gcy = vczt_focus_adjoint(gx, gy, gz, g, win, wavelength, na, f)
    gbx, gby, de2, dt2 = waveplate_adjoint(gcx, gcy, bx, by, *wp2)
    gax, gay, de1, dt1 = waveplate_adjoint(gbx, gby, a, a, *wp1)
    ga = gax + gay
    g_phi2 = phase_grad(ga, a)
    gs = ga * np.exp(-1j * np.asarray(phi2, dtype=np.float64))
    gu1 = rs_adjoint(gs, g, wavelength, z)
    g_phi1 = phase_grad(gu1, u1)
    return loss, g_phi1, g_phi2, (de1, dt1), (de2, dt2)


# --------------------------------------------------------------------------
# Distance gradients dL/dz (every setup of the paper optimises distances)
# --------------------------------------------------------------------------

def rs_kernel_dz(X, Y, z: float, wavelength: float):
    """dH/dz of the RS-I kernel, differentiated by hand from H = (z/2pi)
    e^{ikr} (1/r^3 - ik/r^2) with dr/dz = z/r:
    dH/dz = (1/2pi) e^{ikr} [1/r^3 - ik/r^2 + z^2 (k^2/r^3 + 3ik/r^4 - 3/r^5)].
    """
    k = TWO_PI / wavelength
    r = np.sqrt(np.asarray(X) ** 2 + np.asarray(Y) ** 2 + z * z)
    z2 = z * z
    return np.exp(1j * k * r) / TWO_PI * (1.0 / r ** 3 - 1j * k / r ** 2
                                          + z2 * (k * k / r ** 3 + 3j * k / r ** 4 - 3.0 / r ** 5))


def rs_grad_z(u, g_out, g, wavelength: float, z: float):
    """dL/dz = Re sum conj(g_out) dU/dz per batch item, with
    dU/dz = dx dy sum U0 dH/dz (the RS sum differentiated under the sum)."""
    u, g_out = _as_c128(u), _as_c128(g_out)

    def one(uu, gg):
        K = _kernel_on_offsets(g, lambda X, Y: rs_kernel_dz(X, Y, z, wavelength))
        du = _lin_conv_same_grid(uu, K, g) * (g.dx * g.dy)
        return float(np.sum(np.real(np.conj(gg) * du)))

    if u.ndim == 2:
        return one(u, g_out)
    return np.array([one(a, b) for a, b in zip(u.reshape(-1, *u.shape[-2:]), g_out.reshape(-1, *u.shape[-2:]))])


def czt_grad_z(u, g_out, g_in, win, wavelength: float, z: float):
    """dL/dz = Re sum conj(g_out) dU/dz for the Fresnel sum of czt_propagate.

    Differentiating every z-dependent factor of
    U = K(z) P_z(X) sum U0 Q_z(x) e^{-i 2pi X.x/(lambda z)} gives
    dU/dz = (ik - 1/z - ik|X|^2/(2z^2)) U - (ik/(2z^2)) C[|x|^2 U0]
            + (2 pi i/(lambda z^2)) (X C[x U0] + Y C[y U0]),
    with C the CZT operator itself.
    """
    u, g_out = _as_c128(u), _as_c128(g_out)
    k = TWO_PI / wavelength
    x, y = coords(g_in)
    X, Y = coords(win)
    r2 = x[None, :] ** 2 + y[:, None] ** 2
    R2 = X[None, :] ** 2 + Y[:, None] ** 2
    C = lambda a: czt_propagate(a, g_in, win, wavelength, z)
    U = C(u)
    du = ((1j * k - 1.0 / z - 1j * k * R2 / (2 * z * z)) * U
          - (1j * k / (2 * z * z)) * C(r2 * u)
          + (TWO_PI * 1j / (wavelength * z * z)) * (X[None, :] * C(x[None, :] * u) + Y[:, None] * C(y[:, None] * u)))
    red = np.sum(np.real(np.conj(g_out) * du), axis=(-2, -1))
    return float(red) if np.ndim(red) == 0 else red


# --------------------------------------------------------------------------
# The paper's detector side: STED effective intensity, threshold-density
# loss, soft minimum over detectors (Methods: STED microscopy; loss function)
# --------------------------------------------------------------------------

def sted_intensity(i_ex, i_dep, beta: float):
    """Effective fluorescence I_eff = I_ex [1 - beta (1 - exp(-I_dep/I_ex))]
    (Methods, STED microscopy, Beer-Lambert-type quenching).  Where I_ex = 0
    the paper's limit applies: I_eff = 0."""
    i_ex = np.asarray(i_ex, dtype=np.float64)
    i_dep = np.asarray(i_dep, dtype=np.float64)
    out = np.zeros(np.broadcast(i_ex, i_dep).shape)
    pos = i_ex > 0
    r = np.where(pos, i_dep / np.where(pos, i_ex, 1.0), 0.0)
    out = np.where(pos, i_ex * (1.0 - beta * (1.0 - np.exp(-r))), 0.0)
    return out


def sted_intensity_partials(i_ex, i_dep, beta: float):
    """(dI_eff/dI_ex, dI_eff/dI_dep), differentiated by hand with r = I_dep/I_ex:
    dI_eff/dI_ex = 1 - beta + beta e^{-r} (1 + r), dI_eff/dI_dep = -beta e^{-r}.
    At I_ex = 0 the limits are taken: r -> infinity if I_dep > 0
    (partials 1 - beta, 0), r = 0 if I_dep = 0 (partials 1, -beta)."""
    i_ex = np.asarray(i_ex, dtype=np.float64)
    i_dep = np.asarray(i_dep, dtype=np.float64)
    pos = i_ex > 0
    r = np.where(pos, i_dep / np.where(pos, i_ex, 1.0), np.where(i_dep > 0, np.inf, 0.0))
    e = np.exp(-r)
    fin = np.isfinite(r)
    re = np.zeros_like(r)
    re[fin] = r[fin] * e[fin]  # r e^{-r} -> 0 as r -> infinity
    return 1.0 - beta + beta * (e + re), -beta * e


def intensity_ordered(*fields):
    """I = sum_c (Re E_c^2 + Im E_c^2), accumulated component by component in
    FP64 in the order given (the order the GPU reduction also uses, so that
    threshold decisions are taken on identical values)."""
    acc = None
    for e in fields:
        e = _as_c128(e)
        t = e.real * e.real + e.imag * e.imag
        acc = t if acc is None else acc + t
    return acc


def density_loss(intensity, eps: float):
    """Threshold-density loss L = Area / I_eps (Results, loss function;
    Methods, loss function): i_eps = i where i > eps * i_max else 0,
    I_eps = sum i_eps, Area = number of pixels with i_eps > 0.

    The selection is a comparison, so (as with the paper's where()-based
    evaluation) the gradient flows through the selected values only:
    dL/di = -Area / I_eps^2 on the selected pixels, 0 elsewhere.
    Returns (loss, area, I_eps, i_max, dL/di)."""
    i = np.asarray(intensity, dtype=np.float64)
    imax = float(i.max())
    sel = i > eps * imax
    area = float(np.count_nonzero(sel & (i > 0)))
    ieps = float(np.sum(np.where(sel, i, 0.0)))
    loss = area / ieps
    grad = np.where(sel & (i > 0), -area / (ieps * ieps), 0.0)
    return loss, area, ieps, imax, grad


def density_loss_fields(comps, eps: float, dep=None, beta: float = 1.0):
    """Density loss of the intensity of field components `comps` (optionally
    STED-modulated by the depletion components `dep`), with the gradient
    seeds g_c = 2 E_c dL/dI_c of every component (C5).
    Returns (loss, area, I_eps, i_max, seeds_comps, seeds_dep)."""
    i_ex = intensity_ordered(*comps)
    if dep:
        i_dep = intensity_ordered(*dep)
        i = sted_intensity(i_ex, i_dep, beta)
    else:
        i = i_ex
    loss, area, ieps, imax, dldi = density_loss(i, eps)
    if dep:
        pe, pd = sted_intensity_partials(i_ex, i_dep, beta)
        d_ex, d_dep = dldi * pe, dldi * pd
    else:
        d_ex, d_dep = dldi, None
    seeds = [2.0 * d_ex * _as_c128(e) for e in comps]
    seeds_dep = [2.0 * d_dep * _as_c128(e) for e in dep] if dep else []
    return loss, area, ieps, imax, seeds, seeds_dep


def softmin(losses, beta: float):
    """Smooth minimum over detectors, -log(sum exp(-beta l)) / beta (Methods,
    exploration of optical topologies), evaluated with the minimum factored
    out; returns (value, weights) with weights = d value / d l (a softmax)."""
    l = np.asarray(losses, dtype=np.float64)
    m = l.min()
    w = np.exp(-beta * (l - m))
    s = w.sum()
    return float(m - np.log(s) / beta), w / s


# --------------------------------------------------------------------------
# Optimiser step (the paper optimises with Adam; AdamW in its comparisons)
# --------------------------------------------------------------------------

def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
              weight_decay: float = 0.0):
    """One Adam step (Kingma & Ba) with bias correction; weight_decay > 0
    adds the decoupled (AdamW) decay lr * weight_decay * p.  Returns new
    (p, m, v); step counts from 1."""
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p = p - lr * weight_decay * p - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v


def stop_step(losses, patience: int = 500, check_every: int = 100):
    """Stopping condition of the discovery runs (Methods): every
    `check_every` steps, stop if the best loss so far was reached
    `patience` or more steps ago.  Improvement means strictly below the
    best loss so far (the first finite loss always improves; NaN never does).
    losses[k] is the loss of step k + 1.  Returns the number of steps taken
    when the rule first fires, or None if it never does."""
    best = math.inf
    last_improvement = 0        # step of the last improvement (0: none yet)
    for step, loss in enumerate(losses, start=1):
        if loss < best:
            best = loss
            last_improvement = step
        if step % check_every == 0 and step - last_improvement >= patience:
            return step
    return None
