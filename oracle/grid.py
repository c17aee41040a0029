"""Grid, wavenumbers and truncation masks (oracle; test infrastructure only).

Box of side 2*pi, so the wavenumber spacing is 1 and every wavenumber is an
integer (Sec. "Example: quadratic model in 1D"; Sec. "Numerical methods": the
cubic domain of side 2*pi).  Grid points x_j = 2*pi*j/N (supplementary
Eq. grid_points).

Spectral layout of a real field: complex array of shape [N, N, N//2+1]; axes 0
(k_x) and 1 (k_y) in FFT index order (index i < N/2 -> k = i, else k = i - N, so
the Nyquist index carries k = -N/2 as in supplementary Eq. dft_def), axis 2
holds k_z = 0..N/2.
"""

import math

import numpy as np


def axis_k(n):
    """Integer wavenumbers of one full axis in FFT index order (Eq. dft_def range)."""
    i = np.arange(n, dtype=np.int64)
    return np.where(i < (n + 1) // 2, i, i - n)


def half_k(n):
    """Non-negative wavenumbers k_z = 0..N/2 kept for a real field."""
    return np.arange(n // 2 + 1, dtype=np.int64)


def kgrid(n):
    """Broadcastable integer (kx, ky, kz) arrays over the half-spectrum layout."""
    k = axis_k(n)
    return k[:, None, None], k[None, :, None], half_k(n)[None, None, :]


def k2grid(n):
    """Exact integer |k|^2 on the half-spectrum layout."""
    kx, ky, kz = kgrid(n)
    return kx * kx + ky * ky + kz * kz


def largest_int_below(x):
    """Largest integer strictly below the real x, with x regarded as exact.

    The truncation rule zeroes modes with |k| >= C_t k_N (Sec. "Standard dealiasing
    with truncation": "equal to or larger"), so the retained bound is strict.  A
    value within a relative 1e-9 of an integer is taken to be that integer, so
    that e.g. (2/3 * 96)^2 = 4096 keeps 4095 whatever the last bit of 2/3.
    """
    eps = 1e-9 * max(1.0, abs(x))
    return int(math.ceil(x - eps)) - 1


def sphere_k2max(n, ct):
    """K2max: the largest retained integer |k|^2 for spherical truncation, k_max = C_t N/2."""
    kmax = ct * n / 2.0
    return largest_int_below(kmax * kmax)


def cube_kmax(n, ct):
    """Largest retained |k_i| for cubic truncation (keep every |k_i| < C_t N/2)."""
    return largest_int_below(ct * n / 2.0)


def double_alias_free(n):
    """Modes with |k_i| + |k_j| < 2N/3 for every pair of axes.

    A double alias on the axes (i, j) adds to k the products of input pairs with
    k_n + k_m = k + N (s_i e_i + s_j e_j) (Sec. "Extension to the multidimensional
    case": two components of the nonlinear wavevector out of range), so
    |q_i| + |q_j| >= 2N - |k_i| - |k_j| for q = k_n + k_m.  If every input and the
    output keep |k_i| + |k_j| < 2N/3, then |q_i| + |q_j| < 4N/3 < 2N - |k_i| - |k_j|:
    a state held in this set never receives a double (or triple) alias.
    """
    kx, ky, kz = kgrid(n)
    a, b, c = np.abs(kx), np.abs(ky), np.abs(kz)
    return (3 * (a + b) < 2 * n) & (3 * (a + c) < 2 * n) & (3 * (b + c) < 2 * n)


def mask(n, ct, kind="sphere"):
    """Boolean truncation mask on the half spectrum.

    sphere: keep |k| < C_t k_N (Fig. 1b, parameterised by C_t with k_max = C_t k_N);
    cube:   keep max_i |k_i| < C_t k_N (Fig. 1a);
    no_multiple_aliases: the sphere intersected with double_alias_free (Fig. 7b;
            the paper draws the regions but gives no formula).  For
            C_t <= 2 sqrt(2)/3 the sphere lies inside and nothing is removed.
    rogallo: the cube intersected with double_alias_free: Rogallo's truncation,
            which removes only the double aliases, the cube less thin prisms along
            its edges (Fig. 5; the same reading of the removed regions).
    """
    if kind == "sphere":
        return k2grid(n) <= sphere_k2max(n, ct)
    if kind == "cube":
        kx, ky, kz = kgrid(n)
        km = cube_kmax(n, ct)
        return (np.abs(kx) <= km) & (np.abs(ky) <= km) & (np.abs(kz) <= km)
    if kind == "no_multiple_aliases":
        return (k2grid(n) <= sphere_k2max(n, ct)) & double_alias_free(n)
    if kind == "rogallo":
        return mask(n, ct, "cube") & double_alias_free(n)
    raise ValueError(kind)


def hermitian_weight(n):
    """Weight of each stored k_z plane when summing over the full spectrum of a real
    field: 1 for k_z = 0 and k_z = N/2, 2 for every other plane (the negative k_z
    modes are the complex conjugates of the stored ones)."""
    w = np.full(n // 2 + 1, 2.0)
    w[0] = 1.0
    if n % 2 == 0:
        w[-1] = 1.0
    return w[None, None, :]


def shell_index(k2):
    """Shell n of an integer |k|^2: the n with n(n-1) < k^2 <= n(n+1), i.e. the
    integer nearest to |k| (n = 0 only for k = 0)."""
    k2 = np.asarray(k2, dtype=np.int64)
    n = np.floor(np.sqrt(k2.astype(np.float64))).astype(np.int64)
    # fix the float estimate with exact integer tests
    n = np.where(n * (n + 1) < k2, n + 1, n)
    n = np.where((n > 0) & ((n - 1) * n >= k2), n - 1, n)
    return n


def n_shells(n):
    """Number of shells needed to bin every mode of an N^3 grid."""
    k2top = 3 * (n // 2) ** 2
    return int(shell_index(np.array([k2top]))[0]) + 1
