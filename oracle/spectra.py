"""Energy spectra and global budgets in FP64 (oracle; test infrastructure only).

Quantities of Sec. "3D flow: Taylor-Green vortices" (Figs. 3-4): kinetic energy
E = <|u|^2>/2, dissipation eps = nu <|grad u|^2> = nu sum_k w k^2 |u_hat|^2, the
1D spectra E(k_x), E(k_y), E(k_z), the shell spectrum E(k), the dissipation
spectrum D(k) (whose running sum is the cumulative dissipation) and the
nonlinear transfer T(k) = sum_shell w Re(conj(u_hat).N_hat) (whose running sum
from the top gives the flux).  Helicity H = <u.omega>/2.

w is the Hermitian weight of the stored k_z plane (grid.hermitian_weight).  The
shell of a mode is the integer n with n(n-1) < k^2 <= n(n+1).
"""

import numpy as np

from . import grid
from .nonlinear import curl


def spectra(uh, nu, nh=None):
    """Return dict with e_shell, d_shell, t_shell [n_shells], e_1d [3, N/2+1] and
    totals [E, eps, H, T, nonfinite] (nonfinite = number of non-finite entries of
    u_hat, plus those of N_hat when given)."""
    n = uh.shape[-2]
    w = grid.hermitian_weight(n)
    k2 = grid.k2grid(n)
    kx, ky, kz = grid.kgrid(n)
    ns = grid.n_shells(n)
    emode = 0.5 * w * np.sum(np.abs(uh) ** 2, axis=0)
    shell = np.broadcast_to(grid.shell_index(k2), emode.shape).ravel()
    e_shell = np.bincount(shell, emode.ravel(), minlength=ns)
    dmode = 2.0 * nu * k2 * emode
    d_shell = np.bincount(shell, dmode.ravel(), minlength=ns)
    e_1d = np.zeros((3, n // 2 + 1))
    for axis, kk in enumerate((kx, ky, kz)):
        idx = np.broadcast_to(np.abs(kk), emode.shape).ravel()
        e_1d[axis] = np.bincount(idx, emode.ravel(), minlength=n // 2 + 1)
    if nh is not None:
        tmode = w * np.sum(np.real(np.conj(uh) * nh), axis=0)
        t_shell = np.bincount(shell, tmode.ravel(), minlength=ns)
        t_tot = float(np.sum(tmode))
    else:
        t_shell = np.zeros(ns)
        t_tot = 0.0
    hel = 0.5 * float(np.sum(w * np.sum(np.real(np.conj(uh) * curl(uh)), axis=0)))
    bad = int(np.count_nonzero(~np.isfinite(uh)))
    if nh is not None:
        bad += int(np.count_nonzero(~np.isfinite(nh)))
    totals = np.array([float(np.sum(emode)), float(np.sum(dmode)), hel, t_tot, float(bad)])
    return {"e_shell": e_shell, "d_shell": d_shell, "t_shell": t_shell, "e_1d": e_1d,
            "totals": totals}


def budget(e, eps, inj, dt):
    """Time-integrated energy budget of a run sampled every step (Sec. "3D flow:
    Taylor-Green vortices": dE/dt = -eps for the decaying flow; Sec. "Numerical
    methods": the forced runs inject energy at a given rate).

    e, eps: E and eps at t_j = j dt, j = 0..M; inj: energy injected by the forcing
    in each step j -> j + 1 (M values, or None for a free run).  Returns the
    residuals r_j = E_j - E_0 + int_0^{t_j} eps dt - int_0^{t_j} P dt, j = 0..M,
    with the dissipation integrated by the trapezoid rule step by step and the
    injection summed.  Written as an explicit loop.
    """
    e = [float(v) for v in e]
    eps = [float(v) for v in eps]
    m = len(e) - 1
    if len(eps) != m + 1 or (inj is not None and len(inj) != m):
        raise ValueError("need M + 1 samples of E and eps and M injections")
    out = [0.0]
    diss, work = 0.0, 0.0
    for j in range(m):
        diss += 0.5 * dt * (eps[j] + eps[j + 1])
        if inj is not None:
            work += float(inj[j])
        out.append(e[j + 1] - e[0] + diss - work)
    return np.array(out)


def energy(uh):
    """Total kinetic energy E = (1/2) sum_k w |u_hat|^2."""
    n = uh.shape[-2]
    return 0.5 * float(np.sum(grid.hermitian_weight(n) * np.abs(uh) ** 2))


def inner(a, b):
    """Parseval inner product <a, b> = sum_k w Re(conj(a).b) over the half spectrum."""
    n = a.shape[-2]
    return float(np.sum(grid.hermitian_weight(n) * np.real(np.conj(a) * b)))
