"""Plain FP64 CPU oracle of ILS smoothing (Liu et al., Sec. 3, Algorithm 1).

TEST INFRASTRUCTURE ONLY -- used by tests/, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.  It shares no code
with the HIP library: no kernels, tables, constants or helpers.

Every quantity is float64.  Images are 2-D arrays (H, W); a colour image is
a stack (C, H, W) whose channels are smoothed independently (Sec. 3.4, the
paper's default of filtering each RGB channel separately).

Notation follows the paper:
  f        input image, u output image, s pixel index
  nabla_x  discrete differential operator [1, -1] along x (Sec. 3); read as
           the periodic forward difference  u[y, x+1] - u[y, x]
  nabla_y  the same along y:                  u[y+1, x] - u[y, x]
  phi_p    generalized Charbonnier penalty (x^2 + eps)^(p/2)      Eq. (2)
  c        c0 = p * eps^(p/2 - 1)                                  Eq. (11)
  mu       c * grad - phi_p'(grad)                                  Eq. (7)
  solve    u^{n+1} = F^-1[(F(f) + lam/2 * sum conj(F(nabla))F(mu))
                         / (F(1) + c/2 * lam * sum |F(nabla)|^2)]   Eq. (9)

Readings taken where the paper is silent or garbled (each is listed in the
design notes of the repository):
  * periodic boundaries for the differences as well as for the solve
    (Sec. 3.2 states them for f and u);
  * the misplaced parenthesis of Eq. (9) is read as conj(F(nabla_x)) F(mu_x);
  * c = c0 exactly (Sec. 3.3.3); 0 < p <= 2 is accepted (App. B's argument
    that the maximum of h is h(0) still holds for 1 < p <= 2);
  * the Welsch penalty of Eq. (18) is printed with exp(+x^2/2g^2); it is
    read as 2 g^2 (1 - exp(-x^2 / 2 g^2)), the form whose derivative is the
    one used in Eq. (19);
  * no clipping of the output.

Parity status: pinned.  The linear solve is pinned by a dense least-squares
solve of Eq. (8) (dense_ls_step), the FFT by a naive DFT, mu by finite
differences of phi_p, and the iteration by closed forms and invariants
(mean, constants, p = 2, lam = 0, symmetries, monotone energy, stationarity).
The exact output values on the synthetic workloads are pinned only through
those checks: the paper prints no worked example.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

__all__ = [
    "phi_p", "dphi_p", "charbonnier_c0", "grad_x", "grad_y", "mu_update",
    "transfer_functions", "fft_solve", "ils", "ils_channels", "energy",
    "dense_ls_step", "fixed_point_residual", "phi_welsch", "dphi_welsch",
    "welsch_c0", "mu_update_welsch", "ils_welsch", "energy_welsch",
    "luma", "ils_luminance", "detail_enhance", "tone_map", "tone_map_multiscale",
]


# --------------------------------------------------------------------------
# Penalty, its derivative and the constant c  (Eq. (2), Eq. (7), Eq. (11))
# --------------------------------------------------------------------------
def phi_p(x, p, eps):
    """Generalized Charbonnier penalty (x^2 + eps)^(p/2), Eq. (2)."""
    x = np.asarray(x, dtype=np.float64)
    return (x * x + eps) ** (p / 2.0)


def dphi_p(x, p, eps):
    """d/dx phi_p(x) = p x (x^2 + eps)^(p/2 - 1)  (second line of Eq. (7))."""
    x = np.asarray(x, dtype=np.float64)
    return p * x * (x * x + eps) ** (p / 2.0 - 1.0)


def charbonnier_c0(p, eps):
    """c0 = p eps^(p/2 - 1), Eq. (11) / Eq. (23); the paper uses c = c0."""
    if not (0.0 < p <= 2.0):
        raise ValueError("p must lie in (0, 2]")
    if not eps > 0.0:
        raise ValueError("eps must be positive")
    return p * eps ** (p / 2.0 - 1.0)


# --------------------------------------------------------------------------
# Gradient operators (Sec. 3: kernels [1, -1] and [1, -1]^T), periodic
# --------------------------------------------------------------------------
def grad_x(u):
    """Periodic forward difference along x: u[y, x+1] - u[y, x]."""
    return np.roll(u, -1, axis=-1) - u


def grad_y(u):
    """Periodic forward difference along y: u[y+1, x] - u[y, x]."""
    return np.roll(u, -1, axis=-2) - u


# --------------------------------------------------------------------------
# Intermediate variable mu (Eq. (7))
# --------------------------------------------------------------------------
def mu_update(g, p, eps, c):
    """mu = c g - phi_p'(g) = c g - p g (g^2 + eps)^(p/2 - 1), Eq. (7)."""
    return c * g - dphi_p(g, p, eps)


# --------------------------------------------------------------------------
# The FFT solve of the LS problem (Eq. (8)) as written in Eq. (9)
# --------------------------------------------------------------------------
def transfer_functions(H, W):
    """F(nabla_x), F(nabla_y) and F(1) on the H x W periodic grid.

    Each operator is the circular convolution with a kernel placed on the
    grid: nabla_x u = u[x+1] - u[x] has kernel k[0, 0] = -1, k[0, -1] = +1
    (and likewise along y).  F(1) is the transform of the delta function.
    """
    kx = np.zeros((H, W))
    kx[0, 0] = -1.0
    kx[0, W - 1] = 1.0
    ky = np.zeros((H, W))
    ky[0, 0] = -1.0
    ky[H - 1, 0] = 1.0
    delta = np.zeros((H, W))
    delta[0, 0] = 1.0
    return sfft.fft2(kx), sfft.fft2(ky), sfft.fft2(delta)


def fft_solve(f, mu_x, mu_y, lam, c, tf=None, workers=None):
    """u^{n+1} of Eq. (9) (the exact minimiser of Eq. (8), periodic case).

    Numerator   F(f) + lam/2 (conj(F(nabla_x)) F(mu_x) + conj(F(nabla_y)) F(mu_y))
    Denominator F(1) + c/2 lam (conj(F(nabla_x)) F(nabla_x) + conj(F(nabla_y)) F(nabla_y))
    The real part of the inverse transform is returned (the imaginary part
    is rounding noise: every operand is the transform of a real image).
    """
    H, W = f.shape
    Fx, Fy, F1 = tf if tf is not None else transfer_functions(H, W)
    num = (sfft.fft2(f, workers=workers)
           + lam / 2.0 * (np.conj(Fx) * sfft.fft2(mu_x, workers=workers)
                          + np.conj(Fy) * sfft.fft2(mu_y, workers=workers)))
    den = F1 + c / 2.0 * lam * (np.conj(Fx) * Fx + np.conj(Fy) * Fy)
    return np.real(sfft.ifft2(num / den, workers=workers))


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------
def ils(f, lam, p, eps=1e-4, N=4, u0=None, workers=None, return_iterates=False,
        c=None):
    """Iterative least squares on one channel (Algorithm 1).

    u^0 = f (or u0 when given: the fixed-point check starts from a candidate
    output v while the data term keeps f).  For n = 0..N-1: mu^n from
    nabla u^n by Eq. (7), then u^{n+1} by Eq. (9).  Returns u^N (and the
    list u^0..u^N when return_iterates is set).  c defaults to c0 (Sec.
    3.3.3); any c >= c0 is admissible by Eq. (11).
    """
    f = np.asarray(f, dtype=np.float64)
    if f.ndim != 2:
        raise ValueError("ils expects one channel (H, W)")
    if lam < 0 or not np.isfinite(lam):
        raise ValueError("lam must be finite and >= 0")
    if N < 0:
        raise ValueError("N must be >= 0")
    c0 = charbonnier_c0(p, eps)
    c = c0 if c is None else float(c)
    tf = transfer_functions(*f.shape)
    u = f.copy() if u0 is None else np.asarray(u0, dtype=np.float64).copy()
    its = [u.copy()]
    for _ in range(N):
        mu_x = mu_update(grad_x(u), p, eps, c)
        mu_y = mu_update(grad_y(u), p, eps, c)
        u = fft_solve(f, mu_x, mu_y, lam, c, tf=tf, workers=workers)
        its.append(u.copy())
    return its if return_iterates else u


def ils_channels(f, lam, p, eps=1e-4, N=4, u0=None, workers=None):
    """Each channel of a (C, H, W) stack smoothed independently (Sec. 3.4)."""
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 2:
        return ils(f, lam, p, eps, N, u0=u0, workers=workers)
    out = np.empty_like(f)
    for ch in range(f.shape[0]):
        out[ch] = ils(f[ch], lam, p, eps, N,
                      u0=None if u0 is None else u0[ch], workers=workers)
    return out


# --------------------------------------------------------------------------
# Energy of Eq. (1)
# --------------------------------------------------------------------------
def energy(u, f, lam, p, eps=1e-4):
    """E(u, f) = sum_s (u_s - f_s)^2 + lam sum_{*} phi_p(nabla_* u_s), Eq. (1)."""
    u = np.asarray(u, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    return float(np.sum((u - f) ** 2)
                 + lam * (np.sum(phi_p(grad_x(u), p, eps))
                          + np.sum(phi_p(grad_y(u), p, eps))))


# --------------------------------------------------------------------------
# Dense least-squares solve of Eq. (8) (tiny images only)
# --------------------------------------------------------------------------
def _difference_matrices(H, W):
    """nabla_x and nabla_y as explicit (HW x HW) matrices, periodic, from
    the definition of the [1, -1] kernels (row-major pixel numbering)."""
    n = H * W
    Dx = np.zeros((n, n))
    Dy = np.zeros((n, n))
    for y in range(H):
        for x in range(W):
            s = y * W + x
            Dx[s, y * W + (x + 1) % W] += 1.0
            Dx[s, s] -= 1.0
            Dy[s, ((y + 1) % H) * W + x] += 1.0
            Dy[s, s] -= 1.0
    return Dx, Dy


def dense_ls_step(u, f, lam, p, eps=1e-4):
    """One iteration of Eq. (8) solved as a dense linear least-squares
    problem, never touching a Fourier transform:

        argmin_u  ||u - f||^2 + lam/2 sum_* ||sqrt(c) nabla_* u - mu_*/sqrt(c)||^2

    stacked as  [I; a Dx; a Dy] u ~ [f; a mu_x / c; a mu_y / c],
    a = sqrt(lam c / 2), and handed to LAPACK (numpy.linalg.lstsq).
    mu comes from Eq. (7) evaluated with the explicit matrices.
    """
    u = np.asarray(u, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    H, W = u.shape
    Dx, Dy = _difference_matrices(H, W)
    c = charbonnier_c0(p, eps)
    uv = u.reshape(-1)
    gx = Dx @ uv
    gy = Dy @ uv
    mu_x = c * gx - p * gx * (gx * gx + eps) ** (p / 2.0 - 1.0)
    mu_y = c * gy - p * gy * (gy * gy + eps) ** (p / 2.0 - 1.0)
    a = np.sqrt(lam * c / 2.0)
    A = np.vstack([np.eye(H * W), a * Dx, a * Dy])
    b = np.concatenate([f.reshape(-1), a * mu_x / c, a * mu_y / c])
    sol, *_ = np.linalg.lstsq(A, b, rcond=None)
    return sol.reshape(H, W)


# --------------------------------------------------------------------------
# Fixed-point residual used to assess a candidate output
# --------------------------------------------------------------------------
def fixed_point_residual(v, f, lam, p, eps=1e-4, workers=None):
    """RMS over all pixels of T(v) - v, where T is one ILS iteration started
    from u^0 = v with the data term on f.  v and f are (H, W) or (C, H, W);
    the RMS runs over every channel of the frame."""
    v = np.asarray(v, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    t = ils_channels(f, lam, p, eps, N=1, u0=v, workers=workers)
    return float(np.sqrt(np.mean((t - v) ** 2)))


# --------------------------------------------------------------------------
# Welsch-penalty ILS (Sec. 5, Eqs. (18)-(20))
# --------------------------------------------------------------------------
def phi_welsch(x, gamma):
    """Welsch penalty 2 g^2 (1 - exp(-x^2 / (2 g^2))) (Eq. (18), sign read
    so that the derivative is the one of Eq. (19))."""
    x = np.asarray(x, dtype=np.float64)
    return 2.0 * gamma * gamma * (1.0 - np.exp(-x * x / (2.0 * gamma * gamma)))


def dphi_welsch(x, gamma):
    """phi_W'(x) = 2 x exp(-x^2 / (2 g^2))  (Eq. (19))."""
    x = np.asarray(x, dtype=np.float64)
    return 2.0 * x * np.exp(-x * x / (2.0 * gamma * gamma))


def welsch_c0():
    """c0 = 2 for the Welsch penalty, Eq. (20) / Eq. (24)."""
    return 2.0


def mu_update_welsch(g, gamma, c):
    """mu = c g - 2 g exp(-g^2 / (2 g^2)), Eq. (19)."""
    return c * g - dphi_welsch(g, gamma)


def ils_welsch(f, lam, gamma, N=10, workers=None):
    """Algorithm 1 with the Welsch penalty (Sec. 5): only the pointwise
    mu step and c change."""
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 3:  # channels are independent problems (Sec. 3.4)
        return np.stack([ils_welsch(ch, lam, gamma, N, workers) for ch in f])
    if f.ndim != 2:
        raise ValueError("ils_welsch expects (H, W) or (C, H, W)")
    c = welsch_c0()
    tf = transfer_functions(*f.shape)
    u = f.copy()
    for _ in range(N):
        mu_x = mu_update_welsch(grad_x(u), gamma, c)
        mu_y = mu_update_welsch(grad_y(u), gamma, c)
        u = fft_solve(f, mu_x, mu_y, lam, c, tf=tf, workers=workers)
    return u


def energy_welsch(u, f, lam, gamma):
    """E(u, f) of Eq. (1) with the Welsch penalty of Eq. (18) in place of
    phi_p (the objective the Sec. 5 iteration decreases)."""
    u = np.asarray(u, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    return float(np.sum((u - f) ** 2)
                 + lam * (np.sum(phi_welsch(grad_x(u), gamma))
                          + np.sum(phi_welsch(grad_y(u), gamma))))


# --------------------------------------------------------------------------
# Applications (Sec. 3.4 colour handling, Sec. 4 detail enhancement)
# --------------------------------------------------------------------------
LUMA = (0.299, 0.587, 0.114)  # BT.601 luma weights (the Y of YUV)


def luma(f):
    """Y = 0.299 R + 0.587 G + 0.114 B of a (3, H, W) frame."""
    f = np.asarray(f, dtype=np.float64)
    return LUMA[0] * f[0] + LUMA[1] * f[1] + LUMA[2] * f[2]


def detail_enhance(f, u, k):
    """Details f - u boosted k times on top of the smoothed image: u + k (f - u)."""
    f = np.asarray(f, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    return u + k * (f - u)


def ils_luminance(f, lam, p, eps=1e-4, N=4, k=0.0, workers=None):
    """Sec. 3.4 option (I): go to YUV, smooth (and optionally enhance) only
    Y, come back with U and V unchanged.  The inverse YUV transform adds the
    same multiple (1) of Y to R, G and B, so each channel receives the change
    of Y: out_c = f_c + (v - Y), v = Y's smoothed (enhanced) version."""
    f = np.asarray(f, dtype=np.float64)
    if f.ndim != 3 or f.shape[0] != 3:
        raise ValueError("ils_luminance expects a (3, H, W) RGB frame")
    y = luma(f)
    v = detail_enhance(y, ils(y, lam, p, eps, N, workers=workers), k)
    return f + (v - y)[None]


LUMA_FLOOR = 1e-6  # luminance below this is taken as this before the logarithm


def tone_map(f, lam, p, eps=1e-4, N=4, contrast=100.0, detail=1.0, workers=None):
    """Single-scale HDR tone mapping on the logarithm of the luminance (the
    application the paper shows with p = 1, lambda = 10): L = log Y, base
    B = ILS(L), detail D = L - B; the base is scaled so that its range is
    log(contrast) and its maximum is 0, the detail is kept (times `detail`);
    each channel is multiplied by the ratio of new to old luminance, which
    keeps the colour ratios of every pixel."""
    f = np.asarray(f, dtype=np.float64)
    if f.ndim != 3 or f.shape[0] != 3:
        raise ValueError("tone_map expects a (3, H, W) RGB frame")
    y = np.maximum(luma(f), LUMA_FLOOR)
    L = np.log(y)
    B = ils(L, lam, p, eps, N, workers=workers)
    bmax, bmin = float(B.max()), float(B.min())
    s = np.log(contrast) / (bmax - bmin) if bmax > bmin else 1.0
    Lout = (B - bmax) * s + detail * (L - B)
    return f * (np.exp(Lout) / y)[None]


def tone_map_multiscale(f, lams=(0.125, 1.0, 8.0), p=1.0, eps=1e-4, N=4, contrast=100.0,
                        weights=(1.0, 1.0, 1.0), workers=None):
    """Multi-scale HDR tone mapping on the logarithm of the luminance
    (Sec. 4.2, the multi-scale figure: p = 1 with lambda = 1/8, 1, 8).

    L = log Y is smoothed once per scale, each time from L itself with a
    larger lambda: B_i = ILS(L, lambda_i), i = 1..K (lambda increasing).  The
    detail layers are the differences between successive levels,
    D_1 = L - B_1, D_i = B_{i-1} - B_i; B_K is the base.  The base is shifted
    to maximum 0 and scaled to span log(contrast); detail layer i is kept
    times weights[i]; colour ratios are kept as in tone_map.  With unit
    weights and a contrast equal to the base's own range the log luminance
    is returned unchanged up to a shift (the layers telescope)."""
    f = np.asarray(f, dtype=np.float64)
    if f.ndim != 3 or f.shape[0] != 3:
        raise ValueError("tone_map_multiscale expects a (3, H, W) RGB frame")
    if len(lams) != len(weights) or len(lams) < 1:
        raise ValueError("one weight per scale")
    y = np.maximum(luma(f), LUMA_FLOOR)
    L = np.log(y)
    levels = [L] + [ils(L, lam, p, eps, N, workers=workers) for lam in lams]
    base = levels[-1]
    bmax, bmin = float(base.max()), float(base.min())
    s = np.log(contrast) / (bmax - bmin) if bmax > bmin else 1.0
    Lout = (base - bmax) * s
    for i, w in enumerate(weights):
        Lout = Lout + w * (levels[i] - levels[i + 1])
    return f * (np.exp(Lout) / y)[None]
