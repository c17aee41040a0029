"""Integrating-factor time schemes (oracle; test infrastructure only).

Every scheme advances dS/dt = sigma S + N(S) (Eq. base-eq) with the linear term
integrated exactly, E_tau = exp(sigma tau), sigma = -nu k^2 for Navier-Stokes.
A stage with sub-step tau, approximate state S_a and approximate nonlinear term
N_a gives S(t0 + tau) = (S0 + tau N_a) E_tau (the first-order stage formula of
Sec. "Phase shifting for one-dimensional problems").

The schemes are generic over a ``model`` with
    model.nl(S, shift)          nonlinear term evaluated on the grid shifted by `shift`
    model.nl_vjp(S, lam, shift) transpose of its linearisation at S applied to lam
    model.E(tau)                integrating factor (array broadcastable against S)
    model.zero, model.half      the unshifted and the half-cell shift
so the same code serves the 3D Navier-Stokes oracle and the 1D model.

Readings (where the paper does not print a formula):
* RK4 is the classical four-stage scheme in Lawson (integrating-factor) form.
* In the midpoint RK2 the stage-2 ratio N_a/S_a is read as N_a exp(-sigma dt/2)/S0,
  i.e. S_new = E_dt S0 + dt E_{dt/2} N_a (as in the Rogallo formula).
* Heun / Rogallo: S1 = E_dt (S0 + dt N0); S_new = E_dt S0 + dt/2 E_{dt/2} (N0 + N1)
  (Eq. Rogallo1981 and its 3D form with two shifts alpha, beta).
* Split forcing (Eq. forcing-eq and the stage formulas after it) with O0 = O1 = O.
* The RK4 baseline takes the same forcing as an additive term of every stage slope,
  held constant over the step (the paper forces both schemes; it prints no RK4 form).
"""

import numpy as np


def euler(model, s0, dt):
    """Forward Euler stage: tau = dt, S_a = S0, N_a = N0."""
    return model.E(dt) * (s0 + dt * model.nl(s0, model.zero))


def euler_ps(model, s0, dt):
    """Euler phase shift: N_a = 1/2 (N0 + shifted-and-deshifted N0) (Eq. sum_ps_non_ps)."""
    na = 0.5 * (model.nl(s0, model.zero) + model.nl(s0, model.half))
    return model.E(dt) * (s0 + dt * na)


def rk2(model, s0, dt, avg=False, shifts=None):
    """Midpoint RK2: stage 1 tau = dt/2 with N0, stage 2 tau = dt with N(S1).
    With avg=True every evaluation is the two-shift average ("RK2 phase-shift exact");
    `shifts` (a list of shift vectors) makes it the average over those shifts instead."""
    if shifts is None:
        shifts = [model.zero, model.half] if avg else [model.zero]

    def a(s):
        acc = 0
        for sh in shifts:
            acc = acc + model.nl(s, sh)
        return acc / len(shifts)
    h = 0.5 * dt
    eh = model.E(h)
    sh = eh * (s0 + h * a(s0))
    return model.E(dt) * s0 + dt * eh * a(sh)


def ps_exact(model, s0, dt):
    """RK2 phase-shift exact (midpoint RK2 with the two-shift average at both stages)."""
    return rk2(model, s0, dt, avg=True)


def ps_exact8(model, s0, dt):
    """Midpoint RK2 with every evaluation averaged over the eight shifts {0, 1/2}^3
    (the fully exact 3D shift of Sec. "Extension to the multidimensional case":
    it removes every alias class, double ones included)."""
    eight = [(a, b, c) for a in (0.0, 0.5) for b in (0.0, 0.5) for c in (0.0, 0.5)]
    return rk2(model, s0, dt, shifts=eight)


def rk4(model, s0, dt, forcing=None):
    """Classical RK4 in Lawson form, unshifted (the truncation baseline).

    forcing: an additive term O held constant over the step (drawn at its start, as
    in the split phase-shift scheme), added to the nonlinear term of every stage:
    the stage slopes are N_i + O.
    """
    h = 0.5 * dt
    e = model.E(h)
    z = model.zero
    o = 0.0 if forcing is None else forcing
    n0 = model.nl(s0, z) + o
    sa = e * (s0 + h * n0)
    n1 = model.nl(sa, z) + o
    sb = e * s0 + h * n1
    n2 = model.nl(sb, z) + o
    sc = e * e * s0 + dt * e * n2
    n3 = model.nl(sc, z) + o
    return e * e * s0 + (dt / 6.0) * (e * e * n0 + 2.0 * e * n1 + 2.0 * e * n2 + n3)


def beta_of(alpha):
    """Second-stage shift: each component differs from alpha by half a cell, taken mod 1."""
    return tuple((float(a) + 0.5) % 1.0 for a in np.atleast_1d(alpha))


def ps_heun(model, s0, dt, alpha, beta=None, forcing=None):
    """RK2 phase-shift approx / random (Heun, Rogallo 1981), optional split forcing.

    alpha: first-stage shift (zero for "approx", random per step for "random");
    beta defaults to alpha + 1/2 per component (mod 1).  forcing: O added to both
    stages (O0 = O1 = O).
    """
    if beta is None:
        beta = beta_of(alpha)
    o = 0.0 if forcing is None else forcing
    n0 = model.nl(s0, alpha)
    edt = model.E(dt)
    s1 = edt * (s0 + dt * (n0 + o))
    n1 = model.nl(s1, beta)
    return edt * s0 + 0.5 * dt * model.E(0.5 * dt) * (n0 + n1 + 2.0 * o)


# --------------------------------------------------------------------------- adjoints
def ps_heun_vjp(model, s0, lam, dt, alpha, beta=None, forcing=None, forcing_vjp=None):
    """Transpose of the linearised Heun step at S0 applied to lam = dJ/dS_new.

    S1 = E_dt(S0 + dt (N_a(S0) + O)), S_new = E_dt S0 + dt/2 E_h (N_a(S0) + N_b(S1) + 2 O),
    so mu1 = dJ/dS1 = dt/2 dN_b[S1]^T (E_h lam) and
    dJ/dS0 = E_dt (lam + mu1) + dN_a[S0]^T (dt/2 E_h lam + dt E_dt mu1).
    forcing: the O of the forward step (None: unforced).  When O depends on S0,
    forcing_vjp maps mu_O = dJ/dO = dt (E_h lam + E_dt mu1) to its contribution
    (dO/dS0)^T mu_O, which is added.
    """
    if beta is None:
        beta = beta_of(alpha)
    o = 0.0 if forcing is None else forcing
    edt = model.E(dt)
    eh = model.E(0.5 * dt)
    s1 = edt * (s0 + dt * (model.nl(s0, alpha) + o))
    mu1 = 0.5 * dt * model.nl_vjp(s1, eh * lam, beta)
    out = edt * (lam + mu1) + model.nl_vjp(s0, 0.5 * dt * eh * lam + dt * edt * mu1, alpha)
    if forcing_vjp is not None:
        out = out + forcing_vjp(dt * (eh * lam + edt * mu1))
    return out


def ps_exact_vjp(model, s0, lam, dt):
    """Transpose of the linearised PS-exact step, A = 1/2 (N(.;0) + N(.;half)):
    S_h = E_h(S0 + h A(S0)), S_new = E_dt S0 + dt E_h A(S_h)."""
    h = 0.5 * dt
    eh = model.E(h)

    def a(s):
        return 0.5 * (model.nl(s, model.zero) + model.nl(s, model.half))

    def a_vjp(s, l):
        return 0.5 * (model.nl_vjp(s, l, model.zero) + model.nl_vjp(s, l, model.half))

    sh = eh * (s0 + h * a(s0))
    mu = dt * a_vjp(sh, eh * lam)
    return model.E(dt) * lam + eh * mu + h * a_vjp(s0, eh * mu)
