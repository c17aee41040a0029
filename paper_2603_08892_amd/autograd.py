"""Differentiable phase-shift RK2 time stepping: torch.autograd.Function over the
library's forward steps and its hand-written step adjoint (ns_vjp_rk2_phaseshift).

Forward keeps a copy of the state every `checkpoint_every` steps; backward walks
the segments in reverse, recomputes the states of each segment from its
checkpoint (keeping each recomputed Heun step's first-stage state, which its
adjoint then does not evaluate again), and applies the step adjoints in reverse
order.

Gradient convention: torch's gradient of a real loss with respect to a complex
tensor is dL/dRe + i dL/dIm with every stored entry an independent variable.
The library's adjoint works with the Parseval inner product
<a, b> = sum_k w Re(conj(a).b) (w = 1 on the k_z = 0 and N/2 planes, 2 elsewhere),
so the incoming gradient is divided by w and the outgoing one multiplied by w.
For perturbations that are transforms of real fields the two agree.
"""

import numpy as np
import torch

from . import ns


def hermitian_weight(n, device, dtype):
    w = torch.full((n // 2 + 1,), 2.0, dtype=dtype, device=device)
    w[0] = 1.0
    if n % 2 == 0:
        w[-1] = 1.0
    return w


class PSRK2Function(torch.autograd.Function):
    """u_T = PSRK2Function.apply(u0, solver, dt, nsteps, variant, alphas, checkpoint_every[, forcing]).

    forcing: None, or dict(seed=..., injection=...) for the split forcing of the Heun
    variants, step i drawing with key i (the gradient includes the dependence of the
    forcing amplitude on the state)."""

    @staticmethod
    def forward(ctx, u0, solver, dt, nsteps, variant, alphas, checkpoint_every, forcing=None):
        if variant == "random" and alphas is None:
            raise ValueError("the random variant needs explicit per-step shifts (alphas [nsteps, 3])")
        al = None if alphas is None else np.asarray(alphas, dtype=np.float64).reshape(nsteps, 3)
        u = u0.detach().clone().contiguous()
        ckpts = []
        for i in range(0, nsteps, checkpoint_every):
            ckpts.append(u.clone())
            k = min(checkpoint_every, nsteps - i)  # a segment in one call (same results as k calls)
            solver.step_ps(u, dt, k, variant, alphas=None if al is None else al[i:i + k], forcing=forcing,
                           step0=i)
        ctx.solver, ctx.dt, ctx.nsteps, ctx.variant, ctx.forcing = solver, dt, nsteps, variant, forcing
        ctx.alphas, ctx.every, ctx.ckpts = al, checkpoint_every, ckpts
        return u

    @staticmethod
    def backward(ctx, grad):
        s, dt, nsteps, every, al = ctx.solver, ctx.dt, ctx.nsteps, ctx.every, ctx.alphas
        real = torch.float32 if grad.dtype == torch.complex64 else torch.float64
        w = hermitian_weight(s.n, grad.device, real)
        lam = (grad / w).contiguous()
        nseg = len(ctx.ckpts)
        heun = ctx.variant in ("approx", "random")
        for seg in reversed(range(nseg)):
            start = seg * every
            end = min(start + every, nsteps)
            states = [ctx.ckpts[seg]]
            stage1 = []   # the first-stage states of the recomputed steps (Heun variants)
            u = ctx.ckpts[seg].clone()
            for i in range(start, end - 1):
                s1 = s.empty() if heun else None
                s.step_ps(u, dt, 1, ctx.variant, alphas=None if al is None else al[i:i + 1], forcing=ctx.forcing,
                          step0=i, stage1=s1)
                states.append(u.clone())
                stage1.append(s1)
            stage1.append(None)   # the segment's last step is not recomputed: its adjoint evaluates S1
            for i in reversed(range(start, end)):
                s.vjp_ps(states[i - start], lam, dt, ctx.variant, alpha=None if al is None else al[i],
                         forcing=ctx.forcing, step=i, stage1=stage1[i - start])
        ctx.ckpts = None
        return lam * w, None, None, None, None, None, None, None


def final_energy(u):
    """J = (1/2) sum_k w |u_hat|^2, the kinetic energy of a spectral state."""
    real = torch.float32 if u.dtype == torch.complex64 else torch.float64
    w = hermitian_weight(u.shape[-2], u.device, real)
    return 0.5 * (w * (u.real ** 2 + u.imag ** 2)).sum()
