"""Real 3D discrete Fourier transforms (oracle; test infrastructure only).

Convention of Eqs. u_fft_1d / u_expansion_1d and supplementary Eq. dft_def:
forward  u_hat(k) = (1/N^3) sum_j u(x_j) exp(-i k.x_j)   (1/N per axis)
inverse  u(x_j)   = sum_k u_hat(k) exp(+i k.x_j)          (unnormalised)
Both act on the last three axes, so a leading component axis is allowed.
scipy.fft (pocketfft) does the work; the inverse, as every c2r transform, uses
only the real part of the k_z = 0 and k_z = N/2 coefficients after the two
complex passes.
"""

import os

import numpy as np
import scipy.fft as sfft

def _workers():
    # threads this process may use: its CPU affinity, capped by OMP_NUM_THREADS when set
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


WORKERS = _workers()
AXES = (-3, -2, -1)


def fwd(u):
    """Forward real-to-complex transform with the 1/N^3 normalisation."""
    n = u.shape[-1]
    return sfft.rfftn(np.asarray(u, dtype=np.float64), axes=AXES, norm="forward", workers=WORKERS)


def inv(uh, n=None):
    """Unnormalised complex-to-real inverse transform onto the N^3 grid."""
    if n is None:
        n = uh.shape[-2]
    return sfft.irfftn(np.asarray(uh, dtype=np.complex128), s=(n, n, n), axes=AXES,
                       norm="forward", workers=WORKERS)


def fwd1(u):
    """1D forward real transform, 1/N normalisation (Eq. u_fft_1d)."""
    return sfft.rfft(np.asarray(u, dtype=np.float64), norm="forward")


def inv1(uh, n):
    """1D unnormalised inverse real transform (Eq. u_expansion_1d)."""
    return sfft.irfft(np.asarray(uh, dtype=np.complex128), n=n, norm="forward")
