"""Counter-based random draws and the large-scale forcing (oracle; test infrastructure only).

The paper forces HIT at large scales with a random forcing injecting energy at a
constant unit rate (Sec. "Numerical methods") and gives no formula for it.  The
reading used here:
* the forcing acts on the shell 4 <= |k|^2 <= 9 (2 <= |k| <= 3, 96 full-grid modes);
* its shape g is a complex Gaussian per independent mode and component, projected
  onto divergence-free fields, with the k_z = 0 partners set to the conjugates;
* its amplitude a > 0 makes the one-step injection exactly one:
  a sum w Re(conj(u0).g) + a^2 dt/2 sum w |g|^2 = 1;
* O0 = O1 = a g in the split phase-shift scheme (Eq. forcing-eq).
Parity unpinned against the paper (no formula given); only the unit injection is
pinned.

Draws come from SplitMix64 (Steele, Lea & Flood 2014), used counter-based:
    mix(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
            z *= 0x94D049BB133111EB; z ^= z >> 31
    stream(seed, step) = mix(seed + GAMMA * (step + 1))
    draw(seed, step, j) = mix(stream(seed, step) + GAMMA * (j + 1)),  GAMMA = 0x9E3779B97F4A7C15
    uniform = (draw >> 11) * 2^-53 in [0, 1)
Gaussians: Box-Muller on consecutive uniform pairs (u1, u2):
    r = sqrt(-2 log(1 - u1)), (r cos 2 pi u2, r sin 2 pi u2).
"""

import math

import numpy as np

from . import grid

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def mix64(z):
    z &= MASK64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & MASK64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & MASK64
    z ^= z >> 31
    return z


def draw(seed, step, j):
    s = mix64(seed + GAMMA * (step + 1))
    return mix64(s + GAMMA * (j + 1))


def uniform(seed, step, j):
    return (draw(seed, step, j) >> 11) * (1.0 / 9007199254740992.0)


def random_shift(seed, step):
    """alpha ~ U[0,1)^3 (grid-spacing units) for step `step` (Sec. "Extension to the
    multidimensional case": components drawn uniformly in [0, dx] each step)."""
    return tuple(uniform(seed, step, j) for j in range(3))


def gaussians(seed, step, count):
    out = np.empty(count)
    for p in range((count + 1) // 2):
        u1 = uniform(seed, step, 2 * p)
        u2 = uniform(seed, step, 2 * p + 1)
        r = math.sqrt(-2.0 * math.log(1.0 - u1))
        out[2 * p] = r * math.cos(2.0 * math.pi * u2)
        if 2 * p + 1 < count:
            out[2 * p + 1] = r * math.sin(2.0 * math.pi * u2)
    return out


K2_LO, K2_HI = 4, 9


def forcing_modes():
    """Independent forced modes in draw order: k_z from 0 to 3, then k_x and k_y from -3
    to 3; on k_z = 0 only the half with k_x > 0, or k_x = 0 and k_y > 0."""
    modes = []
    for kz in range(0, 4):
        for kx in range(-3, 4):
            for ky in range(-3, 4):
                k2 = kx * kx + ky * ky + kz * kz
                if not (K2_LO <= k2 <= K2_HI):
                    continue
                if kz == 0 and not (kx > 0 or (kx == 0 and ky > 0)):
                    continue
                modes.append((kx, ky, kz))
    return modes


def forcing_shape(n, seed, step):
    """Divergence-free forcing shape g on the half spectrum of an N^3 grid (dense array)."""
    modes = forcing_modes()
    z = gaussians(seed, step, 6 * len(modes))
    g = np.zeros((3, n, n, n // 2 + 1), dtype=np.complex128)
    for i, (kx, ky, kz) in enumerate(modes):
        v = np.array([complex(z[6 * i + 2 * c], z[6 * i + 2 * c + 1]) for c in range(3)])
        kv = np.array([kx, ky, kz], dtype=np.float64)
        v = v - kv * (kv @ v) / (kv @ kv)
        g[:, kx % n, ky % n, kz] = v
        if kz == 0:
            g[:, (-kx) % n, (-ky) % n, 0] = np.conj(v)
    return g


def amplitude(uh0, g, dt):
    """Positive root a of a B + a^2 (dt/2) G = 1, B = sum w Re(conj(u0).g), G = sum w |g|^2."""
    n = uh0.shape[-2]
    w = grid.hermitian_weight(n)
    b = float(np.sum(w * np.real(np.conj(uh0) * g)))
    gg = float(np.sum(w * np.abs(g) ** 2))
    return 2.0 / (b + math.sqrt(b * b + 2.0 * dt * gg))


def forcing(uh0, dt, seed, step):
    """The forcing O = a g applied during step `step` from state u_hat0."""
    g = forcing_shape(uh0.shape[-2], seed, step)
    return amplitude(uh0, g, dt) * g


def forcing_vjp(uh0, dt, seed, step):
    """Transpose of the derivative of the forcing O(u0) = a(u0) g with respect to u0,
    as a map mu -> (dO/du0)^T mu (Parseval inner product).  Only the amplitude
    depends on u0, through B = <u0, g>: from a B + a^2 dt/2 G = 1,
    da/dB = -a / sqrt(B^2 + 2 dt G), so (dO/du0)^T mu = (da/dB) <mu, g> g."""
    n = uh0.shape[-2]
    w = grid.hermitian_weight(n)
    g = forcing_shape(n, seed, step)
    b = float(np.sum(w * np.real(np.conj(uh0) * g)))
    gg = float(np.sum(w * np.abs(g) ** 2))
    r = math.sqrt(b * b + 2.0 * dt * gg)
    dadb = -(2.0 / (b + r)) / r

    def apply(mu):
        return dadb * float(np.sum(w * np.real(np.conj(mu) * g))) * g
    return apply


def injected(uh0, o, dt):
    """Energy the forcing O puts into the state over one step of length dt from
    u_hat0: E(u0 + dt O) - E(u0) = dt sum w Re(conj(u0).O) + dt^2/2 sum w |O|^2.
    With O from `forcing` it equals dt (unit injection rate); summed over the steps
    it is the integral of the injected power in the energy budget."""
    n = uh0.shape[-2]
    w = grid.hermitian_weight(n)
    b = float(np.sum(w * np.real(np.conj(uh0) * o)))
    gg = float(np.sum(w * np.abs(o) ** 2))
    return dt * b + 0.5 * dt * dt * gg
