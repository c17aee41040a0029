"""Seeded synthetic inputs (velocity fields in spectral form, shifts).

Pure NumPy, float64/complex128, on the host.  These generators build the
workloads of the paper (Taylor-Green vortex, isotropic random fields with a
prescribed spectrum, perturbations) directly in spectral space from their
definitions; they contain no transform, product, projection or time stepping.

Spectral layout: complex array [3, N, N, N//2+1], axes 0/1 in FFT index order
(index i < N/2 is k = i, else k = i - N), axis 2 holds k_z = 0..N/2; the
coefficients follow u(x) = sum_k u_hat(k) exp(i k.x) on the 2*pi box.
"""

import numpy as np


def _axis_k(n):
    i = np.arange(n)
    return np.where(i < (n + 1) // 2, i, i - n)


def _kgrid(n):
    k = _axis_k(n)
    return k[:, None, None], k[None, :, None], np.arange(n // 2 + 1)[None, None, :]


def sphere_keep(n, k2max):
    """Boolean array of modes with integer |k|^2 <= k2max (k2max < (N/2)^2 keeps the
    Nyquist planes empty)."""
    kx, ky, kz = _kgrid(n)
    return (kx * kx + ky * ky + kz * kz) <= k2max


def taylor_green(n):
    """Eq. T-G-init: u = (sin x cos y cos z, -cos x sin y cos z, 0).

    sin x cos y cos z has coefficient s_x/(8i) on each of the eight modes
    (s_x, s_y, s_z) in {-1,1}^3; -cos x sin y cos z has -s_y/(8i).  Only k_z = +1 is
    stored.
    """
    u = np.zeros((3, n, n, n // 2 + 1), dtype=np.complex128)
    for sx in (-1, 1):
        for sy in (-1, 1):
            u[0, sx % n, sy % n, 1] = sx / 8j
            u[1, sx % n, sy % n, 1] = -sy / 8j
    return u


def _hermitian_plane(a, n):
    """Make the k_z = 0 plane of `a` the transform of a real field:
    a(-kx, -ky, 0) = conj(a(kx, ky, 0)); the k_z = N/2 plane likewise."""
    idx = (-_axis_k(n)) % n
    for p in ([0, n // 2] if n % 2 == 0 else [0]):
        plane = a[..., :, :, p]
        partner = np.conj(plane[..., idx[:, None], idx[None, :]])
        a[..., :, :, p] = 0.5 * (plane + partner)
    return a


def random_solenoidal(n, seed, k2max, slope=None, energy=None):
    """Random divergence-free field with modes |k|^2 <= k2max.

    u_hat = i k x a_hat with a_hat complex Gaussian (so k.u_hat = 0 exactly), real-field
    symmetric.  `slope(k)` optionally scales a_hat by a function of |k|; `energy`
    optionally rescales to total kinetic energy (1/2) sum w |u_hat|^2.
    """
    rng = np.random.default_rng(seed)
    shape = (3, n, n, n // 2 + 1)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    kx, ky, kz = _kgrid(n)
    kmag = np.sqrt((kx * kx + ky * ky + kz * kz).astype(np.float64))
    if slope is not None:
        a = a * slope(kmag)
    a = _hermitian_plane(a, n)
    u = np.stack([1j * (ky * a[2] - kz * a[1]),
                  1j * (kz * a[0] - kx * a[2]),
                  1j * (kx * a[1] - ky * a[0])])
    u = u * sphere_keep(n, k2max)
    if energy is not None:
        w = np.full(n // 2 + 1, 2.0)
        w[0] = 1.0
        if n % 2 == 0:
            w[-1] = 1.0
        e = 0.5 * np.sum(w * np.abs(u) ** 2)
        u = u * np.sqrt(energy / e)
    return u


def hit_initial(n, seed, k2max, energy=1.5, kpeak=4.0):
    """Isotropic random field with E(k) ~ k^4 exp(-2 (k/kpeak)^2) and total energy `energy`.

    With u_hat = i k x a_hat, |u_hat|^2 ~ k^2 |a_hat|^2; a shell of radius k holds ~k^2
    modes, so |a_hat| ~ exp(-(k/kpeak)^2) gives E(k) ~ k^4 exp(-2 (k/kpeak)^2).
    """
    return random_solenoidal(n, seed, k2max, slope=lambda k: np.exp(-(k / kpeak) ** 2),
                             energy=energy)


def embed(a, n):
    """A spectral field of an m^3 grid, zero at and beyond |k_i| = m/2, placed at the same
    wavevectors of an n^3 grid (n >= m): the same physical field on the finer grid."""
    m = a.shape[-2]
    out = np.zeros(a.shape[:-3] + (n, n, n // 2 + 1), dtype=a.dtype)
    k = _axis_k(m)
    idx = k % n
    out[..., idx[:, None], idx[None, :], : m // 2] = a[..., :, :, : m // 2]
    return out


def hit_field(n, seed, k2max, energy=1.5, kpeak=4.0, base=64):
    """The field of hit_initial drawn on a base^3 grid (|k| < base/2; the spectrum
    k^4 exp(-2 (k/4)^2) is below 1e-10 of its peak there) and embedded in the n^3 grid,
    so that every grid n >= base starts from the same physical field."""
    k2 = min(k2max, (base // 2 - 1) ** 2)
    return embed(hit_initial(base, seed, k2, energy=energy, kpeak=kpeak), n)


def tg_perturbed(n, seed, k2max, rel=1e-2):
    """Taylor-Green plus a random divergence-free perturbation whose L2 norm is `rel`
    times that of the Taylor-Green field."""
    tg = taylor_green(n)
    p = random_solenoidal(n, seed, k2max)
    nt = np.sqrt(np.sum(np.abs(tg) ** 2))
    npn = np.sqrt(np.sum(np.abs(p) ** 2))
    return tg + p * (rel * nt / npn)


def shear_wave(n, k=2):
    """u = (sin(k y), 0, 0): u x omega is a gradient, so the projected nonlinear term
    vanishes and the flow decays as exp(-nu k^2 t)."""
    u = np.zeros((3, n, n, n // 2 + 1), dtype=np.complex128)
    u[0, 0, k % n, 0] = 1 / 2j
    u[0, 0, (-k) % n, 0] = -1 / 2j
    return u


def random_shifts(seed, nsteps):
    """Shifts alpha ~ U[0,1)^3 per step, in grid-spacing units, shape [nsteps, 3]."""
    return np.random.default_rng(seed).random((nsteps, 3))


def model1d_initial(n, k0=10, amp=0.7):
    """Spectrum k = 0..n/2 of S0 = 1 + amp cos(k0 x) (the 1D model's initial value)."""
    s = np.zeros(n // 2 + 1, dtype=np.complex128)
    s[0] = 1.0
    s[k0] = amp / 2.0
    return s


def model1d_random(n, seed, batch, kmax, amp=0.3):
    """Batch of real signals 1 + (random modes 1..kmax with Gaussian coefficients,
    amplitudes falling as exp(-(k/8)^2)), spectra [batch, n/2 + 1]."""
    rng = np.random.default_rng(seed)
    s = np.zeros((batch, n // 2 + 1), dtype=np.complex128)
    k = np.arange(1, kmax + 1)
    s[:, 0] = 1.0
    s[:, 1:kmax + 1] = amp * np.exp(-(k / 8.0) ** 2) * (rng.standard_normal((batch, kmax))
                                                        + 1j * rng.standard_normal((batch, kmax))) / np.sqrt(2)
    return s
