"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same
seeded inputs.

Tolerances: FP64 instantiation 1e-12 (relative L2 and relative to the largest
entry).  FP32 fields: 1e-5 relative L2 per evaluation or per step (the stated
FP32 field tolerance; FP32 round-off of ~log2(N^3) butterfly stages and one
product gives 2e-6 to 5e-6 here), and 3e-4 relative to the largest entry: the
projection removes the gradient part of u x omega, which on some high-|k|
modes is one to two orders of magnitude larger than the solenoidal remainder,
so the per-mode FP32 error is amplified there by |FFT(u x omega)| / |N|.
The FP64 reference is computed from the same FP32-representable input.  FP64
spectra: 1e-10 per bin (bins above 1e-30 of the total).
"""

import numpy as np
import pytest

from oracle import forcing as oforcing
from oracle import grid, schemes, spectra
from oracle import nonlinear as onl
from paper_2603_08892_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-12), "fp32": (1e-5, 3e-4)}


def _solver(n, ct, mask="sphere", prec="fp32", nu=0.01, seed=0, generic=False):
    from paper_2603_08892_amd import ns
    return ns.Solver(n, nu, ct, mask=mask, precision=prec, seed=seed, generic=generic)


def _rep(a, prec):
    """The input as the device holds it (FP32 rounding for fp32), in complex128."""
    return a.astype(np.complex64).astype(np.complex128) if prec == "fp32" else a.astype(np.complex128)


def _host(t):
    return t.cpu().numpy().astype(np.complex128)


def _check(got, want, prec, what=""):
    l2 = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)
    mx = np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)
    aw = np.abs(want)
    big = aw > 1e-3 * aw.max()
    per_mode = float((np.abs(got - want)[big] / aw[big]).max()) if big.any() else 0.0
    print(f"[parity] {what} {got.shape[-2]}^3 {prec}: rel L2 {l2:.2e} max/max {mx:.2e} "
          f"per-mode (>1e-3 max) {per_mode:.2e}", flush=True)
    tl2, tmx = TOL[prec]
    assert l2 <= tl2 and mx <= tmx, f"{what}: rel L2 {l2:.3e} rel max {mx:.3e}"


def _field(n, ct, mask, seed, energy=None):
    k2 = 3 * grid.cube_kmax(n, ct) ** 2 if mask in ("cube", "rogallo") else grid.sphere_k2max(n, ct)
    u = inputs.random_solenoidal(n, seed, k2, energy=energy)
    return u * grid.mask(n, ct, mask)


NL_CASES = [
    (8, 1.0, "sphere", "fp64"), (12, 1.0, "sphere", "fp64"), (16, 2 / 3, "sphere", "fp64"),
    (24, 1.0, "cube", "fp64"), (32, 2 / 3, "sphere", "fp64"), (40, 0.9, "sphere", "fp64"),
    (48, 1.0, "sphere", "fp32"), (32, 1.0, "sphere", "fp32"), (60, 2 / 3, "cube", "fp32"),
    (64, 1.0, "sphere", "fp32"), (96, 2 / 3, "sphere", "fp32"), (128, 1.0, "sphere", "fp32"),
    (128, 2 / 3, "cube", "fp32"), (192, 2 / 3, "sphere", "fp32"), (256, 1.0, "sphere", "fp32"),
    (16, 1.0, "no_multiple_aliases", "fp64"), (24, 0.97, "no_multiple_aliases", "fp64"),
    (64, 1.0, "no_multiple_aliases", "fp32"), (128, 1.0, "no_multiple_aliases", "fp32"),
    (24, 1.0, "rogallo", "fp64"), (30, 0.9, "rogallo", "fp64"), (64, 1.0, "rogallo", "fp32"),
    (128, 1.0, "rogallo", "fp32"), (192, 1.0, "rogallo", "fp32"), (216, 1.0, "sphere", "fp32"),
]


@pytest.mark.parametrize("n,ct,mask,prec", NL_CASES)
def test_nonlinear_parity(n, ct, mask, prec):
    """ns_nonlinear for unshifted, half-cell, random shifts and the two-shift average."""
    print(f"[nonlinear] n={n} ct={ct:.4f} mask={mask} prec={prec}", flush=True)
    s = _solver(n, ct, mask, prec)
    m = grid.mask(n, ct, mask)
    u = _rep(_field(n, ct, mask, 1000 + n), prec)
    ud = s.to_device(u)
    for shift in [None, (0.5, 0.5, 0.5), (0.137, 0.71, 0.402)]:
        got = _host(s.nonlinear(ud, shift=shift))
        _check(got, onl.nonlinear(u, m, shift), prec, f"shift {shift}")
    got = _host(s.nonlinear(ud, ps_avg=True))
    _check(got, onl.nonlinear_ps(u, m), prec, "ps_avg")


def test_nonlinear_ignores_modes_outside_mask():
    """Entries outside the retained set are ignored on input and zero on output."""
    n, ct = 32, 2 / 3
    s = _solver(n, ct, "sphere", "fp64")
    m = grid.mask(n, ct)
    u = inputs.random_solenoidal(n, 5, 3 * (n // 2) ** 2)      # fills every mode
    got = _host(s.nonlinear(s.to_device(u)))
    _check(got, onl.nonlinear(u, m), "fp64")
    assert np.all(got[:, ~m] == 0)


@pytest.mark.parametrize("n,ct,mask", [(24, 1.0, "no_multiple_aliases"), (30, 0.98, "no_multiple_aliases"),
                                       (24, 1.0, "rogallo"), (30, 0.9, "rogallo")])
def test_pair_rule_masks_pair_average_is_clean(n, ct, mask):
    """With the "no_multiple_aliases" and Rogallo truncations the GPU's isotropic pair
    average is the alias-free (padded) product of the oracle, and the output is zero
    outside the mask even for an input that fills every mode."""
    s = _solver(n, ct, mask, "fp64")
    m = grid.mask(n, ct, mask)
    u = _field(n, ct, mask, 300 + n)
    _check(_host(s.nonlinear(s.to_device(u), ps_avg=True)), onl.nonlinear_pad(u, m), "fp64", "clean")
    full = inputs.random_solenoidal(n, 9, 3 * (n // 2) ** 2)
    got = _host(s.nonlinear(s.to_device(full)))
    _check(got, onl.nonlinear(full, m), "fp64", "full input")
    assert np.all(got[:, ~m] == 0)


@pytest.mark.parametrize("mask", ["no_multiple_aliases", "rogallo"])
@pytest.mark.parametrize("scheme", ["rk4", "exact", "random"])
def test_pair_rule_masks_step(scheme, mask):
    n, ct, nu, dt = 32, 1.0, 0.02, 0.01
    s = _solver(n, ct, mask, "fp64", nu=nu, seed=12)
    m = grid.mask(n, ct, mask)
    model = onl.NSModel(n, nu, m)
    u = _field(n, ct, mask, 41, energy=0.5)
    ud = s.to_device(u)
    if scheme == "rk4":
        s.step_rk4(ud, dt, 1)
    else:
        s.step_ps(ud, dt, 1, scheme, step0=2)
    want = _oracle_step(model, u, dt, "heun" if scheme == "random" else scheme,
                        alpha=oforcing.random_shift(12, 2))
    _check(_host(ud), want, "fp64", scheme)


def test_nonlinear_deterministic():
    n = 64
    s = _solver(n, 1.0)
    ud = s.to_device(_field(n, 1.0, "sphere", 3))
    a = _host(s.nonlinear(ud, shift=(0.3, 0.2, 0.9)))
    b = _host(s.nonlinear(ud, shift=(0.3, 0.2, 0.9)))
    assert np.array_equal(a, b)


def test_taylor_green_closed_form_on_gpu():
    """The GPU nonlinear term of the Taylor-Green field (Eq. T-G-init) is the
    hand-derived one: -(1/8)(sin2x cos2z, sin2y cos2z, -(cos2x+cos2y) sin2z)."""
    n = 32
    s = _solver(n, 2 / 3, prec="fp64")
    got = _host(s.nonlinear(s.to_device(inputs.taylor_green(n))))
    want = np.zeros_like(got)
    for (kx, kz, val) in [(2, 2, 1j / 32), (-2, 2, -1j / 32)]:
        want[0, kx % n, 0, kz] = val
        want[1, 0, kx % n, kz] = val
    for kx in (2, -2):
        want[2, kx % n, 0, 2] = -1j / 32
        want[2, 0, kx % n, 2] = -1j / 32
    assert np.abs(got - want).max() < 1e-15


def _oracle_step(model, u, dt, scheme, alpha=None, force=None):
    plain = {"rk4": schemes.rk4, "exact": schemes.ps_exact, "rk2": schemes.rk2, "euler": schemes.euler,
             "euler_ps": schemes.euler_ps, "exact8": schemes.ps_exact8}
    if scheme in plain:
        return plain[scheme](model, u, dt)
    return schemes.ps_heun(model, u, dt, alpha, forcing=force)


STEP_CASES = [(16, 1.0, "fp64"), (24, 2 / 3, "fp64"), (32, 1.0, "fp32"), (48, 0.9, "fp32"), (64, 2 / 3, "fp32")]


@pytest.mark.parametrize("n,ct,prec", STEP_CASES)
@pytest.mark.parametrize("scheme", ["rk4", "exact", "approx", "random", "rk2", "euler", "euler_ps", "exact8"])
def test_one_step_parity(n, ct, prec, scheme):
    print(f"[step] n={n} ct={ct:.4f} prec={prec} scheme={scheme}", flush=True)
    nu, dt = 0.02, 0.01
    s = _solver(n, ct, prec=prec, nu=nu, seed=77)
    m = grid.mask(n, ct)
    model = onl.NSModel(n, nu, m)
    u = _rep(_field(n, ct, "sphere", 2000 + n, energy=0.5), prec)
    ud = s.to_device(u)
    if scheme == "rk4":
        s.step_rk4(ud, dt, 1)
        want = _oracle_step(model, u, dt, "rk4")
    elif scheme == "exact":
        s.step_ps(ud, dt, 1, "exact")
        want = _oracle_step(model, u, dt, "exact")
    elif scheme == "approx":
        s.step_ps(ud, dt, 1, "approx")
        want = _oracle_step(model, u, dt, "heun", alpha=(0, 0, 0))
    elif scheme != "random":
        s.step_ps(ud, dt, 1, scheme)
        want = _oracle_step(model, u, dt, scheme)
    else:
        s.step_ps(ud, dt, 1, "random", step0=5)            # alpha from SplitMix64(seed, 5)
        want = _oracle_step(model, u, dt, "heun", alpha=oforcing.random_shift(77, 5))
    got = _host(ud)
    _check(got, want, prec, scheme)
    if prec == "fp64":  # the increment S_new - E S0 itself, which carries the nonlinear term
        lin = model.E(dt) * u
        _check(got - lin, want - lin, prec, scheme + " increment")


def test_random_shifts_given_explicitly():
    n, ct, nu, dt = 24, 1.0, 0.02, 0.01
    s = _solver(n, ct, prec="fp64", nu=nu)
    m = grid.mask(n, ct)
    model = onl.NSModel(n, nu, m)
    u = _field(n, ct, "sphere", 9, energy=0.5)
    al = inputs.random_shifts(4, 3)
    ud = s.to_device(u)
    s.step_ps(ud, dt, 3, "random", alphas=al)
    want = u
    for i in range(3):
        want = schemes.ps_heun(model, want, dt, tuple(al[i]))
    _check(_host(ud), want, "fp64", "random explicit")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_split_forcing_parity(prec):
    """RK2 phase-shift random split with the shell forcing (Eq. forcing-eq)."""
    n, ct, nu, dt = 32, 1.0, 0.01, 0.005
    s = _solver(n, ct, prec=prec, nu=nu, seed=3)
    m = grid.mask(n, ct)
    model = onl.NSModel(n, nu, m)
    u = _rep(inputs.hit_initial(n, 8, grid.sphere_k2max(n, ct)), prec)
    ud = s.to_device(u)
    s.step_ps(ud, dt, 2, "random", forcing={"seed": 11, "injection": 1.0}, step0=4)
    want = u
    for i in range(2):
        o = oforcing.forcing(want, dt, 11, 4 + i)
        want = schemes.ps_heun(model, want, dt, oforcing.random_shift(3, 4 + i), forcing=o)
    _check(_host(ud), want, prec, "split forcing")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_taylor_green_config_small(prec):
    """Taylor-Green, N = 32, nu = 1/1600, dt = 1e-3, 10 steps of RK4 (C_t = 2/3) and of
    RK2 phase-shift exact (C_t = 1): the small Taylor-Green workload."""
    n, nu, dt = 32, 1 / 1600, 1e-3
    u0 = inputs.taylor_green(n)
    for scheme, ct in (("rk4", 2 / 3), ("exact", 1.0)):
        s = _solver(n, ct, prec=prec, nu=nu)
        model = onl.NSModel(n, nu, grid.mask(n, ct))
        ud = s.to_device(u0)
        want = u0
        for _ in range(10):
            want = _oracle_step(model, want, dt, scheme)
        if scheme == "rk4":
            s.step_rk4(ud, dt, 10)
        else:
            s.step_ps(ud, dt, 10, "exact")
        tol = 1e-12 if prec == "fp64" else 1e-5
        got = _host(ud)
        assert np.linalg.norm(got - want) / np.linalg.norm(want) < tol, scheme


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spectra_parity(prec):
    n, ct, nu = 32, 1.0, 0.013
    s = _solver(n, ct, prec=prec, nu=nu)
    m = grid.mask(n, ct)
    u = _rep(_field(n, ct, "sphere", 31, energy=0.7), prec)
    ud = s.to_device(u)
    nh = s.nonlinear(ud, ps_avg=True)
    nh_h = _host(nh)
    got = s.spectra(ud, nh)
    want = spectra.spectra(u, nu, nh_h)
    for key in ("e_shell", "d_shell", "t_shell", "e_1d"):
        g, w = got[key], want[key]
        big = np.abs(w) > 1e-30 * np.abs(w).sum()
        assert np.all(np.abs(g[big] - w[big]) <= 1e-10 * np.abs(w[big]) + 1e-14 * np.abs(w).max()), key
    gt, wt = got["totals"], want["totals"]
    assert np.allclose(gt[:3], wt[:3], rtol=1e-10, atol=0)
    assert abs(gt[3] - wt[3]) <= 1e-10 * np.sqrt(spectra.inner(u, u) * spectra.inner(nh_h, nh_h))
    assert gt[4] == 0


def test_spectra_flags_nonfinite():
    from paper_2603_08892_amd import ns
    n = 16
    s = _solver(n, 1.0, prec="fp64")
    u = _field(n, 1.0, "sphere", 1)
    u[1, 2, 3, 1] = np.nan
    with pytest.raises(ns.NSError) as e:
        s.spectra(s.to_device(u))
    assert e.value.status == ns.NS_ERR_NONFINITE
    out = s.spectra(s.to_device(u), check_finite=False)
    assert out["totals"][4] == 1


def test_zero_steps_and_argument_errors():
    from paper_2603_08892_amd import ns
    n = 16
    s = _solver(n, 1.0, prec="fp64")
    u = _field(n, 1.0, "sphere", 2)
    ud = s.to_device(u)
    s.step_rk4(ud, 0.1, 0)
    s.step_ps(ud, 0.1, 0, "random")
    assert np.array_equal(_host(ud), u)
    with pytest.raises(ns.NSError):
        s.step_rk4(ud, -0.1, 1)
    with pytest.raises(ns.NSError):
        s.step_ps(ud, 0.1, 1, "exact", forcing={"seed": 1})
    lam = s.to_device(u)
    for v in ("rk2", "euler", "euler_ps", "exact8"):    # forcing and the adjoint: Heun/PS variants only
        with pytest.raises(ns.NSError):
            s.step_ps(ud, 0.1, 1, v, forcing={"seed": 1})
        with pytest.raises(ns.NSError):
            s.vjp_ps(ud, lam, 0.1, v)
    for bad in (-1, 7):
        assert ns.lib().ns_step_rk2_phaseshift(s.ctx, s._field(ud, "u"), 0.1, 1, bad, None, None, 0, None) == ns.NS_ERR_ARG
    assert np.array_equal(_host(ud), u)
    with pytest.raises(ns.NSError):
        s.nonlinear(ud, out=ud)


def test_energy_conservation_on_gpu():
    """Sum w Re(conj(u).N) = 0 for every shift (u.(u x omega) = 0 on any grid)."""
    n = 64
    s = _solver(n, 1.0, prec="fp32")
    u = _rep(_field(n, 1.0, "sphere", 12), "fp32")
    ud = s.to_device(u)
    for shift in [None, (0.5, 0.5, 0.5), (0.2, 0.6, 0.1)]:
        nh = _host(s.nonlinear(ud, shift=shift))
        scale = np.sqrt(spectra.inner(u, u) * spectra.inner(nh, nh))
        assert abs(spectra.inner(u, nh)) <= 1e-6 * scale


@pytest.mark.parametrize("n,ct,mask", [(64, 1.0, "sphere"), (128, 1.0, "sphere"), (128, 2 / 3, "sphere"),
                                       (192, 2 / 3, "sphere"), (256, 1.0, "sphere"),
                                       (128, 1.0, "no_multiple_aliases"), (128, 2 / 3, "cube"),
                                       (192, 1.0, "rogallo"), (216, 1.0, "sphere"), (324, 2 / 3, "sphere"),
                                       (384, 512 / 3 / 192, "sphere"), (512, 2 / 3, "sphere"),
                                       (144, 128 / 144, "sphere"), (160, 0.8, "sphere"), (160, 2 / 3, "cube"),
                                       (240, 0.9, "sphere"), (240, 1.0, "no_multiple_aliases"),
                                       (270, 0.8, "sphere"), (360, 512 / 3 / 180, "sphere"),
                                       # few retained modes: one k_z tile, most rows pruned
                                       (160, 0.1, "sphere"), (270, 0.05, "sphere"), (360, 0.02, "cube"),
                                       (144, 1.0, "rogallo"),
                                       # the sizes whose y-inverse pass forms the curl, other truncations
                                       (256, 1.0, "no_multiple_aliases"), (256, 2 / 3, "cube"),
                                       (270, 1.0, "cube"), (144, 0.5, "no_multiple_aliases")])
def test_specialised_passes_match_generic(n, ct, mask):
    """The compile-time FP32 passes (N = 64, 128, 144, 160, 192, 216, 240, 256, 270,
    324, 360, 384, 512; at 160, 240, 270 and 360 some butterflies of a stage are
    predicated off; at 128, 144, 256 and 270 the x-inverse passes store five fields
    and the y-inverse pass forms the vorticity, where the generic passes store six)
    and the size-generic passes agree to FP32 round-off (each is within ~5e-6 of the
    FP64 oracle), for the nonlinear term and two steps of every scheme."""
    print(f"[fast-vs-generic] n={n} ct={ct:.4f} mask={mask}", flush=True)
    nu, dt = 1 / 1600, 2e-3
    fast = _solver(n, ct, mask, nu=nu, seed=4)
    gen = _solver(n, ct, mask, nu=nu, seed=4, generic=True)
    u = _rep(_field(n, ct, mask, 77, energy=0.5), "fp32")
    for shift in [None, (0.5, 0.5, 0.5), (0.3, 0.8, 0.45)]:
        a = _host(fast.nonlinear(fast.to_device(u), shift=shift))
        b = _host(gen.nonlinear(gen.to_device(u), shift=shift))
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-5, shift
    for scheme in ("rk4", "exact", "approx", "random", "rk2", "euler", "euler_ps", "exact8"):
        ua, ub = fast.to_device(u), gen.to_device(u)
        for s_, ud in ((fast, ua), (gen, ub)):
            if scheme == "rk4":
                s_.step_rk4(ud, dt, 2)
            else:
                s_.step_ps(ud, dt, 2, scheme)
        a, b = _host(ua), _host(ub)
        # two FP32 paths, each within ~2e-6 of the FP64 oracle after two steps: on
        # the 270^3 cube field at C_t = 1 (every mode retained, Nyquist rows
        # included) rk2 measured 1.88e-6 (specialised) and 1.86e-6 (generic)
        # against the oracle and 2.5e-6 between them
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 3e-6, scheme


@pytest.mark.parametrize("n,ct,prec,variant,forced", [
    (24, 1.0, "fp64", "random", True), (24, 1.0, "fp64", "approx", False), (24, 1.0, "fp64", "exact", False),
    (24, 1.0, "fp64", "rk2", False), (24, 1.0, "fp64", "euler", False), (24, 1.0, "fp64", "euler_ps", False),
    (24, 1.0, "fp64", "exact8", False), (128, 1.0, "fp32", "random", True), (128, 1.0, "fp32", "approx", False),
    (128, 1.0, "fp32", "exact", False), (192, 2 / 3, "fp32", "random", False), (64, 1.0, "fp32", "exact8", False),
    # streaming stores into the scratch fields and the compact stage buffers
    (256, 1.0, "fp32", "random", True), (240, 1.0, "fp32", "exact", False), (270, 0.8, "fp32", "approx", False)])
def test_multi_step_call_equals_single_steps(n, ct, prec, variant, forced):
    """k steps in one call (the state stays in the workspace between them) are
    bit-identical to k calls of one step, and both match the oracle (N <= 24)."""
    print(f"[multi-step] n={n} {prec} {variant} forced={forced}", flush=True)
    nu, dt, k = 0.01, 2e-3, 4
    s = _solver(n, ct, prec=prec, nu=nu, seed=31)
    u = _rep(_field(n, ct, "sphere", 500 + n, energy=0.5), prec)
    fo = {"seed": 3, "injection": 1.0} if forced else None
    a, b = s.to_device(u), s.to_device(u)
    s.step_ps(a, dt, k, variant, forcing=fo, step0=9)
    for i in range(k):
        s.step_ps(b, dt, 1, variant, forcing=fo, step0=9 + i)
    ga, gb = _host(a), _host(b)
    assert np.array_equal(ga, gb)
    if n <= 24:
        model = onl.NSModel(n, nu, grid.mask(n, ct))
        want = u
        for i in range(k):
            if variant in ("random", "approx"):
                al = oforcing.random_shift(31, 9 + i) if variant == "random" else (0, 0, 0)
                o = oforcing.forcing(want, dt, 3, 9 + i) if forced else None
                want = schemes.ps_heun(model, want, dt, al, forcing=o)
            else:
                want = _oracle_step(model, want, dt, variant)
        _check(ga, want, prec, "multi-step")


@pytest.mark.parametrize("n,ct,prec", [(24, 2 / 3, "fp64"), (192, 2 / 3, "fp32")])
def test_multi_step_rk4_call_equals_single_steps(n, ct, prec):
    print(f"[multi-step rk4] n={n} {prec}", flush=True)
    nu, dt, k = 0.01, 2e-3, 3
    s = _solver(n, ct, prec=prec, nu=nu, seed=31)
    u = _rep(_field(n, ct, "sphere", 700 + n, energy=0.5), prec)
    a, b = s.to_device(u), s.to_device(u)
    s.step_rk4(a, dt, k)
    for _ in range(k):
        s.step_rk4(b, dt, 1)
    assert np.array_equal(_host(a), _host(b))
    if n <= 24:
        model = onl.NSModel(n, nu, grid.mask(n, ct))
        want = u
        for _ in range(k):
            want = schemes.rk4(model, want, dt)
        _check(_host(a), want, prec, "multi-step rk4")


def test_spectra_async_sees_the_state_at_enqueue():
    """ns_spectra_async reduces the state as it is at that point of the stream, even
    with steps enqueued before ns_spectra_wait; waiting with nothing in flight is an
    error.  The reduction adds in a fixed order, so both results agree bit for bit."""
    from paper_2603_08892_amd import ns
    n = 32
    s = _solver(n, 1.0, prec="fp64", nu=0.01)
    u = _field(n, 1.0, "sphere", 77, energy=0.5)
    ud = s.to_device(u)
    want = s.spectra(ud)
    s.spectra_async(ud)
    s.step_ps(ud, 1e-2, 5, "random")
    got = s.spectra_wait()
    for key in want:
        assert np.array_equal(got[key], want[key]), key
    assert not np.allclose(s.spectra(ud)["totals"][:2], want["totals"][:2], rtol=1e-6)
    with pytest.raises(ns.NSError) as e:
        s.spectra_wait()
    assert e.value.status == ns.NS_ERR_STATE


@pytest.mark.parametrize("mask,ct", [("cube", 2 / 3), ("no_multiple_aliases", 1.0), ("rogallo", 1.0)])
@pytest.mark.parametrize("scheme", ["random", "exact", "rk4"])
def test_chained_steps_every_mask(mask, ct, scheme):
    """Chained evaluations (specialised 64^3 passes) with the other truncations: three
    steps in one call are bit-identical to one-step calls and match the oracle."""
    print(f"[chained] {mask} ct={ct:.3f} {scheme}", flush=True)
    n, nu, dt, k = 64, 0.01, 2e-3, 3
    s = _solver(n, ct, mask, "fp32", nu=nu, seed=17)
    m = grid.mask(n, ct, mask)
    u = _rep(_field(n, ct, mask, 808, energy=0.5), "fp32")
    a, b = s.to_device(u), s.to_device(u)
    if scheme == "rk4":
        s.step_rk4(a, dt, k)
        for _ in range(k):
            s.step_rk4(b, dt, 1)
    else:
        s.step_ps(a, dt, k, scheme, step0=4)
        for i in range(k):
            s.step_ps(b, dt, 1, scheme, step0=4 + i)
    ga = _host(a)
    assert np.array_equal(ga, _host(b))
    model = onl.NSModel(n, nu, m)
    want = u
    for i in range(k):
        al = oforcing.random_shift(17, 4 + i) if scheme == "random" else None
        want = _oracle_step(model, want, dt, "heun" if scheme == "random" else scheme, alpha=al)
    _check(ga, want, "fp32", f"{mask} {scheme}")


@pytest.mark.parametrize("n,prec", [(128, "fp32"), (48, "fp64"), (256, "fp32")])
def test_spectra_bitwise_reproducible(n, prec):
    """The FP64 spectra of one state (with a transfer field) are identical bit for bit
    across calls: every bin is summed in a fixed order."""
    print(f"[spectra determinism] n={n} {prec}", flush=True)
    s = _solver(n, 1.0, prec=prec, nu=0.01)
    u = _rep(_field(n, 1.0, "sphere", 61, energy=0.5), prec)
    ud = s.to_device(u)
    nh = s.nonlinear(ud)
    a, b = s.spectra(ud, nh), s.spectra(ud, nh)
    for key in a:
        assert np.array_equal(a[key], b[key]), key
