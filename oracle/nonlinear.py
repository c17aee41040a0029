"""The dealiased nonlinear term and its variants (oracle; test infrastructure only).

For a spectral velocity u_hat (shape [3, N, N, N//2+1]) the nonlinear operator of
Eq. base-eq, N(S) = P[-(u.grad)u], is evaluated in rotational form,
N(u_hat) = M . P . FFT(u x omega), which has the same projection for a clean
(alias-free) product since u x omega = grad(|u|^2/2) - (u.grad)u.

Phase shifting (Eqs. shift_operator and shift_operator_3d): the state is
multiplied by exp(i k.Delta) before the product and the result by
exp(-i k.Delta) after it.  Shifts are given in units of the grid spacing, so a
shift s means Delta = s * 2*pi/N and the factor is exp(2*pi*i k.s/N).

The state lives in the retained set: the input is masked first, then the result
is masked and projected (Sec. "Standard dealiasing with truncation").  The k = 0
component of the result is zero.
"""

import numpy as np

from . import grid
from .transforms import fwd, inv

PS_SHIFT = (0.5, 0.5, 0.5)  # isotropic half-cell shift (Sec. "Extension to the multidimensional case")


def phase(n, shift):
    """exp(2*pi*i (kx sx + ky sy + kz sz)/N) on the half spectrum (Eq. shift_operator_3d)."""
    kx, ky, kz = grid.kgrid(n)
    sx, sy, sz = (float(v) for v in shift)
    ang = 2.0 * np.pi * (kx * sx + ky * sy + kz * sz) / n
    return np.exp(1j * ang)


def curl(a):
    """Spectral curl omega_hat = i k x a_hat."""
    n = a.shape[-2]
    kx, ky, kz = grid.kgrid(n)
    ax, ay, az = a
    return np.stack([1j * (ky * az - kz * ay),
                     1j * (kz * ax - kx * az),
                     1j * (kx * ay - ky * ax)])


def project(f):
    """Divergence-free projection P(k) f = f - k (k.f)/|k|^2, with P(0) = 0."""
    n = f.shape[-2]
    kx, ky, kz = grid.kgrid(n)
    k2 = kx * kx + ky * ky + kz * kz
    kdotf = kx * f[0] + ky * f[1] + kz * f[2]
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(k2 > 0, kdotf / np.where(k2 > 0, k2, 1), 0.0)
    out = np.stack([f[0] - kx * r, f[1] - ky * r, f[2] - kz * r])
    out[:, 0, 0, 0] = 0.0
    return out


def cross(a, b):
    """Pointwise cross product of two real 3-component fields."""
    return np.stack([a[1] * b[2] - a[2] * b[1],
                     a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]])


def nonlinear(uh, m, shift=None):
    """N(u_hat; s) = M . conj(phi) . P . FFT( IFFT(phi M u_hat) x IFFT(i k x phi M u_hat) ).

    m is a boolean mask (grid.mask); shift None or (0,0,0) means unshifted.
    Follows the pseudo-spectral product (Sec. "Aliasing description": two inverse
    transforms, a pointwise product, one forward transform) with the shift and
    deshift of Eq. shift_operator_3d around it.
    """
    n = uh.shape[-2]
    a = uh * m
    shifted = shift is not None and any(float(v) != 0.0 for v in shift)
    if shifted:
        phi = phase(n, shift)
        a = a * phi
    u = inv(a, n)
    w = inv(curl(a), n)
    fh = fwd(cross(u, w))
    nh = project(fh)
    if shifted:
        nh = nh * np.conj(phi)
    return nh * m


def nonlinear_avg(uh, m, shifts):
    """Average of N(u_hat; s) over a list of shifts (Eq. sum_ps_non_ps and its 3D form)."""
    acc = 0
    for s in shifts:
        acc = acc + nonlinear(uh, m, s)
    return acc / len(shifts)


def nonlinear_ps(uh, m):
    """Two-grid phase-shift average 1/2 [N(u;0) + N(u;(1/2,1/2,1/2))]: removes single and
    triple aliases, keeps double aliases (Sec. "Extension to the multidimensional case")."""
    return nonlinear_avg(uh, m, [(0.0, 0.0, 0.0), PS_SHIFT])


EIGHT_SHIFTS = [(a, b, c) for a in (0.0, 0.5) for b in (0.0, 0.5) for c in (0.0, 0.5)]


def nonlinear_8(uh, m):
    """Average over all 2^3 shifts in {0, 1/2}^3: removes every alias class."""
    return nonlinear_avg(uh, m, EIGHT_SHIFTS)


def _embed(ah, n, mp):
    """Copy an N-grid half spectrum (Nyquist entries zero) into an M-grid one."""
    out = np.zeros(ah.shape[:-3] + (mp, mp, mp // 2 + 1), dtype=np.complex128)
    kk = grid.axis_k(n) % mp
    out[..., kk[:, None], kk[None, :], : n // 2 + 1] = ah
    return out


def _extract(bh, n, mp):
    kk = grid.axis_k(n) % mp
    return bh[..., kk[:, None], kk[None, :], : n // 2 + 1]


def nonlinear_pad(uh, m, mpad=None):
    """Clean (alias-free) product by zero padding to an M^3 grid (the 3/2 rule of
    Sec. "Introduction": extend the grid, multiply, truncate back).  Default
    M = 2N, which is alias-free for any retained set."""
    n = uh.shape[-2]
    mp = 2 * n if mpad is None else int(mpad)
    a = _embed(uh * m, n, mp)
    u = inv(a, mp)
    w = inv(curl(a), mp)
    fh = _extract(fwd(cross(u, w)), n, mp)
    return project(fh) * m


def nonlinear_vjp(uh, lam, m, shift=None):
    """Transpose of the linearised nonlinear term, (dN[u_hat])^T lam.

    The inner product is the Parseval one, <a, b> = sum_k w Re(conj(a) . b) over the
    half spectrum (w from grid.hermitian_weight), under which the inverse
    transform is an isometry onto real fields with the grid mean.  With
    u = IFFT(phi M a), omega = IFFT(i k x phi M a), lt = IFFT(phi P M lam):
        result = M conj(phi) [ FFT(omega x lt) + i k x FFT(lt x u) ]
    (derived from a.(b x c) = b.(c x a) and the self-adjointness of the curl).
    """
    n = uh.shape[-2]
    a = uh * m
    lm = project(lam * m)
    shifted = shift is not None and any(float(v) != 0.0 for v in shift)
    if shifted:
        phi = phase(n, shift)
        a = a * phi
        lm = lm * phi
    u = inv(a, n)
    w = inv(curl(a), n)
    lt = inv(lm, n)
    g = fwd(cross(w, lt)) + curl(fwd(cross(lt, u)))
    if shifted:
        g = g * np.conj(phi)
    return g * m


class NSModel:
    """3D Navier-Stokes as a scheme model: sigma = -nu k^2 (Eq. base-eq), nonlinear
    term `nonlinear`, shifts in grid-spacing units; `clean=True` swaps in the
    padded (alias-free) product for the reference runs used by the tests."""

    zero = (0.0, 0.0, 0.0)
    half = PS_SHIFT

    def __init__(self, n, nu, m, clean=False):
        self.n, self.nu, self.m, self.clean = n, float(nu), m, clean
        self.k2 = grid.k2grid(n).astype(np.float64)

    def nl(self, s, shift):
        if self.clean:
            return nonlinear_pad(s, self.m)
        return nonlinear(s, self.m, shift)

    def nl_vjp(self, s, lam, shift):
        return nonlinear_vjp(s, lam, self.m, shift)

    def E(self, tau):
        return np.exp(-self.nu * self.k2 * tau)
