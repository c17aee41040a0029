"""The 1D quadratic model dS/dt = -S^2 (Eqs. model-1d-2, 1d_exact, 1d_initial)
(oracle; test infrastructure only).

Domain 2*pi, N points, spectral state S_hat(k), k = 0..N/2 (real field).  The
nonlinear term evaluated on a grid shifted by s cells is
    N(S_hat; s) = M conj(phi) FFT( -(IFFT(phi M S_hat))^2 ),  phi = exp(2 pi i k s / N),
with M the truncation |k| < C_t N/2.  sigma = 0, so every integrating factor is 1.
"""

import numpy as np

from .grid import largest_int_below
from .transforms import fwd1, inv1


class NL1DModel:
    zero = 0.0
    half = 0.5

    def __init__(self, n, ct, clean=False):
        self.n = n
        self.k = np.arange(n // 2 + 1)
        self.m = self.k <= largest_int_below(ct * n / 2.0)
        self.clean = clean

    def nl(self, s, shift):
        n = self.n
        a = s * self.m
        if self.clean:
            # alias-free product on a grid of 2N points
            big = np.zeros(n + 1, dtype=np.complex128)
            big[: n // 2 + 1] = a
            v = inv1(big, 2 * n)
            return fwd1(-v * v)[: n // 2 + 1] * self.m
        phi = np.exp(2j * np.pi * self.k * shift / n) if shift else 1.0
        v = inv1(a * phi, n)
        out = fwd1(-v * v)
        if shift:
            out = out * np.conj(phi)
        return out * self.m

    def nl_vjp(self, s, lam, shift):
        raise NotImplementedError

    def E(self, tau):
        return 1.0


def initial(n, k0=10, amp=0.7):
    """S0 = 1 + amp cos(k0 x) in spectral form (Eq. 1d_initial)."""
    s = np.zeros(n // 2 + 1, dtype=np.complex128)
    s[0] = 1.0
    s[k0] = amp / 2.0
    return s


def exact(n, t, k0=10, amp=0.7, nfine=4096):
    """Spectral coefficients k = 0..N/2 of S0/(1 + S0 t) (Eq. 1d_exact), from a fine
    grid whose aliasing is below double precision."""
    x = 2 * np.pi * np.arange(nfine) / nfine
    s0 = 1.0 + amp * np.cos(k0 * x)
    return fwd1(s0 / (1.0 + s0 * t))[: n // 2 + 1]
