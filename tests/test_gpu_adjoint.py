"""GPU adjoint of the phase-shift RK2 step against the oracle's adjoint, a
dot-product test against finite differences of the GPU step, and the
checkpointed torch.autograd.Function against central finite differences.

Tolerances: FP64 instantiation vs the oracle 1e-11 relative L2; FP32 vs the FP64
oracle 1e-4 relative L2 (the stated adjoint tolerance); FP64 dot products vs
Richardson-extrapolated central differences 1e-9 (the step is a polynomial of
degree 4 in S0, so the extrapolation removes the truncation error); FP32
gradients vs FP32 central differences 1e-3 relative (differences of FP32 states
lose about half the digits).
"""

import numpy as np
import pytest

from oracle import grid, schemes, spectra
from oracle import nonlinear as onl
from paper_2603_08892_amd import inputs

pytestmark = pytest.mark.gpu


def _solver(n, ct, prec, nu):
    from paper_2603_08892_amd import ns
    return ns.Solver(n, nu, ct, precision=prec, seed=5)


def _rep(a, prec):
    return a.astype(np.complex64).astype(np.complex128) if prec == "fp32" else a


def _host(t):
    return t.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("n,ct,prec", [(16, 1.0, "fp64"), (24, 2 / 3, "fp64"), (32, 1.0, "fp32"), (48, 0.9, "fp32")])
@pytest.mark.parametrize("variant", ["approx", "random", "exact"])
def test_vjp_matches_oracle(n, ct, prec, variant):
    print(f"[vjp] n={n} ct={ct:.3f} {prec} {variant}", flush=True)
    nu, dt = 0.02, 0.01
    s = _solver(n, ct, prec, nu)
    m = grid.mask(n, ct)
    model = onl.NSModel(n, nu, m)
    k2 = grid.sphere_k2max(n, ct)
    u0 = _rep(inputs.random_solenoidal(n, 300 + n, k2, energy=0.5), prec)
    lam = _rep(inputs.random_solenoidal(n, 400 + n, k2), prec)
    alpha = (0.31, 0.77, 0.05)
    ud, ld = s.to_device(u0), s.to_device(lam)
    s.vjp_ps(ud, ld, dt, variant, alpha=alpha if variant == "random" else None)
    if variant == "exact":
        want = schemes.ps_exact_vjp(model, u0, lam, dt)
    else:
        want = schemes.ps_heun_vjp(model, u0, lam, dt, alpha if variant == "random" else (0, 0, 0))
    got = _host(ld)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel < (1e-11 if prec == "fp64" else 1e-4), rel
    assert np.array_equal(_host(ud), u0)            # the state is not modified


def test_vjp_dot_product_with_gpu_steps_fp64():
    """<lam, J v> with J v from central differences of the GPU step equals <J^T lam, v>."""
    n, ct, nu, dt = 24, 1.0, 0.01, 0.02
    s = _solver(n, ct, "fp64", nu)
    k2 = grid.sphere_k2max(n, ct)
    u0 = inputs.random_solenoidal(n, 7, k2, energy=0.5)
    lam = inputs.random_solenoidal(n, 8, k2)
    alpha = np.array([[0.12, 0.56, 0.93]])
    for variant in ("random", "exact"):
        ld = s.to_device(lam)
        s.vjp_ps(s.to_device(u0), ld, dt, variant, alpha=alpha[0] if variant == "random" else None)
        g = _host(ld)
        for seed in (1, 2):
            v = inputs.random_solenoidal(n, 50 + seed, k2)

            def step(x):
                xd = s.to_device(x)
                s.step_ps(xd, dt, 1, variant, alphas=alpha if variant == "random" else None)
                return _host(xd)

            d = [(step(u0 + e * v) - step(u0 - e * v)) / (2 * e) for e in (1e-3, 5e-4)]
            jv = (4 * d[1] - d[0]) / 3
            lhs, rhs = spectra.inner(lam, jv), spectra.inner(g, v)
            assert abs(lhs - rhs) <= 1e-9 * abs(lhs), (variant, lhs, rhs)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autograd_checkpointed_gradient(prec):
    """Gradient of the final kinetic energy after 12 random-shift steps (checkpoint every 5)
    w.r.t. the initial field, Taylor-Green plus a 1e-2 perturbation, against central
    differences along seeded directions."""
    import torch
    from paper_2603_08892_amd.autograd import PSRK2Function, final_energy
    n, ct, nu, dt, steps = 32, 1.0, 1 / 1600, 2e-3, 12
    s = _solver(n, ct, prec, nu)
    k2 = grid.sphere_k2max(n, ct)
    u0 = s.to_device(_rep(inputs.tg_perturbed(n, 3, k2), prec))
    al = inputs.random_shifts(9, steps)
    x = u0.clone().requires_grad_(True)
    J = final_energy(PSRK2Function.apply(x, s, dt, steps, "random", al, 5))
    J.backward()
    g = x.grad.detach()

    def run(y):
        with torch.no_grad():
            return final_energy(PSRK2Function.apply(y, s, dt, steps, "random", al, 5)).item()

    eps = 1e-6 if prec == "fp64" else 1e-3 * float(torch.linalg.vector_norm(u0))
    tol = 1e-7 if prec == "fp64" else 1e-3
    for seed in range(4):
        v = s.to_device(inputs.random_solenoidal(n, 90 + seed, k2))
        v = v / torch.linalg.vector_norm(v) + 0.5 * u0 / torch.linalg.vector_norm(u0)
        fd = (run(u0 + eps * v) - run(u0 - eps * v)) / (2 * eps)
        ad = float((g.conj() * v).real.sum())
        assert abs(fd - ad) <= tol * max(abs(fd), 1e-3 * float(torch.linalg.vector_norm(g))), (seed, fd, ad)


@pytest.mark.parametrize("n,ct,mask", [(64, 1.0, "sphere"), (64, 2 / 3, "sphere"), (64, 1.0, "no_multiple_aliases"),
                                       (128, 1.0, "sphere")])
@pytest.mark.parametrize("variant", ["approx", "random", "exact"])
def test_vjp_specialised_passes_match_oracle(n, ct, mask, variant):
    """The specialised FP32 adjoint passes (N = 64, 128) against the FP64 oracle's adjoint."""
    from paper_2603_08892_amd import ns
    print(f"[vjp fast] n={n} ct={ct:.3f} {mask} {variant}", flush=True)
    nu, dt = 0.02, 0.01
    s = ns.Solver(n, nu, ct, mask=mask, precision="fp32", seed=5)
    m = grid.mask(n, ct, mask)
    model = onl.NSModel(n, nu, m)
    k2 = grid.sphere_k2max(n, ct)
    u0 = _rep(inputs.random_solenoidal(n, 300 + n, k2, energy=0.5) * m, "fp32")
    lam = _rep(inputs.random_solenoidal(n, 400 + n, k2) * m, "fp32")
    alpha = (0.31, 0.77, 0.05)
    ud, ld = s.to_device(u0), s.to_device(lam)
    s.vjp_ps(ud, ld, dt, variant, alpha=alpha if variant == "random" else None)
    if variant == "exact":
        want = schemes.ps_exact_vjp(model, u0, lam, dt)
    else:
        want = schemes.ps_heun_vjp(model, u0, lam, dt, alpha if variant == "random" else (0, 0, 0))
    rel = np.linalg.norm(_host(ld) - want) / np.linalg.norm(want)
    assert rel < 1e-4, rel


@pytest.mark.parametrize("n,ct", [(128, 2 / 3), (192, 2 / 3), (256, 1.0), (216, 1.0), (324, 2 / 3),
                                  (384, 512 / 3 / 192), (512, 2 / 3), (144, 1.0), (160, 0.8), (240, 0.9),
                                  (270, 0.8), (360, 512 / 3 / 180)])
def test_vjp_specialised_passes_match_generic(n, ct):
    """Specialised and size-generic adjoint passes agree to FP32 round-off."""
    from paper_2603_08892_amd import ns
    print(f"[vjp fast-vs-generic] n={n} ct={ct:.3f}", flush=True)
    nu, dt = 1 / 1600, 2e-3
    fast = ns.Solver(n, nu, ct, precision="fp32", seed=5)
    gen = ns.Solver(n, nu, ct, precision="fp32", seed=5, generic=True)
    k2 = grid.sphere_k2max(n, ct)
    u0 = _rep(inputs.random_solenoidal(n, 11, k2, energy=0.5), "fp32")
    lam = _rep(inputs.random_solenoidal(n, 12, k2), "fp32")
    for variant in ("approx", "random", "exact"):
        al = (0.4, 0.15, 0.9) if variant == "random" else None
        a, b = fast.to_device(lam), gen.to_device(lam)
        fast.vjp_ps(fast.to_device(u0), a, dt, variant, alpha=al)
        gen.vjp_ps(gen.to_device(u0), b, dt, variant, alpha=al)
        ga, gb = _host(a), _host(b)
        assert np.linalg.norm(ga - gb) / np.linalg.norm(gb) < 1e-5, variant


@pytest.mark.parametrize("n,prec,forced", [(32, "fp32", False), (64, "fp32", True), (24, "fp64", True),
                                           (128, "fp32", True)])
def test_vjp_with_kept_first_stage_is_identical(n, prec, forced):
    """A Heun step that keeps its first-stage state gives the same next state, and the
    adjoint given that state the same result, bit for bit, as without it."""
    import torch
    nu, dt, ct = 0.02, 0.01, 1.0
    print(f"[vjp stage1] n={n} {prec} forced={forced}", flush=True)
    s = _solver(n, ct, prec, nu)
    k2 = grid.sphere_k2max(n, ct)
    u0 = _rep(inputs.hit_initial(n, 91, k2), prec)
    lam = _rep(inputs.random_solenoidal(n, 92, k2), prec)
    fo = {"seed": 13, "injection": 1.0} if forced else None
    alpha = [(0.41, 0.07, 0.66)]
    a, b = s.to_device(u0), s.to_device(u0)
    s1 = s.empty()
    s.step_ps(a, dt, 1, "random", alphas=alpha, forcing=fo, step0=5)
    s.step_ps(b, dt, 1, "random", alphas=alpha, forcing=fo, step0=5, stage1=s1)
    assert torch.equal(a, b)
    la, lb = s.to_device(lam), s.to_device(lam)
    s.vjp_ps(s.to_device(u0), la, dt, "random", alpha=alpha[0], forcing=fo, step=5)
    s.vjp_ps(s.to_device(u0), lb, dt, "random", alpha=alpha[0], forcing=fo, step=5, stage1=s1)
    assert torch.equal(la, lb)
