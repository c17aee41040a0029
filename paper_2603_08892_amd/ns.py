"""Thin ctypes binding of libns.so (include/ns.h); argument marshalling only.

Every computation runs in the library's HIP kernels.  PyTorch provides device
memory (the caller's field tensors and the workspace) and the stream.  If the
library is missing the binding raises; there is no fallback.

Field tensors: complex64 (FP32 contexts) or complex128 (FP64 contexts), shape
[3, N, N, N//2+1], contiguous, on the context's device; layout and conventions
as documented in include/ns.h.
"""

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libns.so")

NS_OK, NS_ERR_ARG, NS_ERR_SIZE, NS_ERR_HIP, NS_ERR_STATE, NS_ERR_NONFINITE = range(6)
NS_FP32, NS_FP64 = 0, 1
NS_MASK_SPHERE, NS_MASK_CUBE, NS_MASK_NO_MULTIPLE_ALIASES, NS_MASK_ROGALLO = 0, 1, 2, 3
MASKS = {"sphere": NS_MASK_SPHERE, "cube": NS_MASK_CUBE, "no_multiple_aliases": NS_MASK_NO_MULTIPLE_ALIASES,
         "rogallo": NS_MASK_ROGALLO}
NS_PS_EXACT, NS_PS_APPROX, NS_PS_RANDOM, NS_RK2, NS_EULER, NS_EULER_PS, NS_PS_EXACT8 = range(7)
NS_NL_PS_AVG = 1
VARIANTS = {"exact": NS_PS_EXACT, "approx": NS_PS_APPROX, "random": NS_PS_RANDOM, "rk2": NS_RK2,
            "euler": NS_EULER, "euler_ps": NS_EULER_PS, "exact8": NS_PS_EXACT8}

# every function declared in include/ns.h
ABI_FUNCTIONS = ("ns_workspace_bytes", "ns_num_shells", "ns_retained_bound", "ns_init", "ns_destroy",
                 "ns_last_error", "ns_set_stream", "ns_nonlinear", "ns_step_rk4_trunc",
                 "ns_step_rk2_phaseshift", "ns_spectra", "ns_vjp_rk2_phaseshift", "ns_timing_enable",
                 "ns_timing_read", "ns1d_nonlinear", "ns1d_step", "ns_spectra_async", "ns_spectra_wait",
                 "ns_budget_start", "ns_budget_stop", "ns_budget_read", "ns_spectra_static")
NS_BUDGET_LEN = 8
BUDGET_NAMES = ("t", "E", "eps", "E0", "int_eps", "int_p", "p_last", "residual")
PASS_NAMES = ("x_inverse", "y_inverse", "z_fused", "y_forward", "x_forward_epilogue", "x_forward_inverse")


class NSConfig(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("precision", ctypes.c_int32), ("mask", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("nu", ctypes.c_double), ("ct", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("stream", ctypes.c_void_p)]


class NSForcing(ctypes.Structure):
    _fields_ = [("k2_lo", ctypes.c_int32), ("k2_hi", ctypes.c_int32), ("injection", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class NSSpectraOut(ctypes.Structure):
    _fields_ = [("e_shell", ctypes.c_void_p), ("d_shell", ctypes.c_void_p), ("t_shell", ctypes.c_void_p),
                ("e_1d", ctypes.c_void_p), ("totals", ctypes.c_void_p)]


class NSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libns status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libns.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_08892_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, S = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    cfgp = ctypes.POINTER(NSConfig)
    sig = {
        "ns_workspace_bytes": (S, [cfgp]),
        "ns_num_shells": (I32, [I32]),
        "ns_retained_bound": (I64, [cfgp]),
        "ns_init": (I32, [cfgp, P, S, ctypes.POINTER(P)]),
        "ns_destroy": (I32, [P]),
        "ns_last_error": (ctypes.c_char_p, [P]),
        "ns_set_stream": (I32, [P, P]),
        "ns_nonlinear": (I32, [P, P, P, P, I32]),
        "ns_step_rk4_trunc": (I32, [P, P, D, I32, ctypes.POINTER(NSForcing), I64]),
        "ns_step_rk2_phaseshift": (I32, [P, P, D, I32, I32, P, ctypes.POINTER(NSForcing), I64, P]),
        "ns_spectra": (I32, [P, P, P, ctypes.POINTER(NSSpectraOut)]),
        "ns_vjp_rk2_phaseshift": (I32, [P, P, P, D, I32, P, ctypes.POINTER(NSForcing), I64, P]),
        "ns_budget_start": (I32, [P, P]),
        "ns_budget_stop": (I32, [P]),
        "ns_budget_read": (I32, [P, P]),
        "ns_spectra_static": (I32, [I32, I32, D, P, P, P, ctypes.POINTER(NSSpectraOut)]),
        "ns_timing_enable": (I32, [P, I32]),
        "ns_timing_read": (I32, [P, P, P]),
        "ns_spectra_async": (I32, [P, P, P]),
        "ns_spectra_wait": (I32, [P, ctypes.POINTER(NSSpectraOut)]),
        "ns1d_nonlinear": (I32, [P, P, I32, D, I32, D, P]),
        "ns1d_step": (I32, [P, I32, D, I32, D, I32, I32, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    _lib = L
    return L


NS_CFG_GENERIC_PASSES = 1


def make_config(n, nu, ct, mask="sphere", precision="fp32", seed=0, stream=None, generic=False):
    return NSConfig(int(n), NS_FP32 if precision == "fp32" else NS_FP64,
                    MASKS[mask],
                    NS_CFG_GENERIC_PASSES if generic else 0, float(nu), float(ct), int(seed), stream)


def workspace_bytes(n, nu, ct, mask="sphere", precision="fp32"):
    return int(lib().ns_workspace_bytes(ctypes.byref(make_config(n, nu, ct, mask, precision))))


def retained_bound(n, ct, mask="sphere"):
    return int(lib().ns_retained_bound(ctypes.byref(make_config(n, 0.0, ct, mask))))


def num_shells(n):
    return int(lib().ns_num_shells(int(n)))


def _forcing(f):
    """ns_forcing from dict(seed=..., injection=1.0) (the shell 4 <= |k|^2 <= 9), or NULL."""
    if f is None:
        return None
    return ctypes.byref(NSForcing(4, 9, float(f.get("injection", 1.0)), int(f["seed"])))


def _dbl3(v):
    if v is None:
        return None
    a = (ctypes.c_double * 3)(*[float(x) for x in v])
    return a


class Solver:
    """One library context on a CUDA (HIP) device with its workspace tensor."""

    def __init__(self, n, nu, ct, mask="sphere", precision="fp32", seed=0, device="cuda:0", generic=False):
        import torch
        self.torch = torch
        self.n, self.nu, self.ct, self.mask, self.precision = n, nu, ct, mask, precision
        self.device = torch.device(device)
        self.dtype = torch.complex64 if precision == "fp32" else torch.complex128
        self.stream = torch.cuda.current_stream(self.device)
        cfg = make_config(n, nu, ct, mask, precision, seed, ctypes.c_void_p(self.stream.cuda_stream), generic)
        L = lib()
        nbytes = L.ns_workspace_bytes(ctypes.byref(cfg))
        if nbytes == 0:
            raise NSError(NS_ERR_ARG, L.ns_last_error(None).decode())
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        ctx = ctypes.c_void_p()
        st = L.ns_init(ctypes.byref(cfg), ctypes.c_void_p(base + off), nbytes, ctypes.byref(ctx))
        if st != NS_OK:
            raise NSError(st, L.ns_last_error(None).decode())
        self.ctx = ctx
        self.nshells = int(L.ns_num_shells(n))
        self.bound = int(L.ns_retained_bound(ctypes.byref(cfg)))

    def __del__(self):
        if getattr(self, "ctx", None) is not None and _lib is not None:
            _lib.ns_destroy(self.ctx)
            self.ctx = None

    def _check(self, st):
        if st != NS_OK:
            raise NSError(st, lib().ns_last_error(self.ctx).decode())

    def _field(self, t, name):
        shape = (3, self.n, self.n, self.n // 2 + 1)
        if t.dtype != self.dtype or tuple(t.shape) != shape or not t.is_contiguous() or t.device != self.device:
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of shape {shape} on {self.device}")
        return ctypes.c_void_p(t.data_ptr())

    def _sync_stream(self):
        """Follow torch's current stream.  The workspace is shared by every call, so the
        new stream first waits for the work already enqueued on the old one."""
        cur = self.torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.wait_stream(self.stream)
            self.stream = cur
            self._check(lib().ns_set_stream(self.ctx, ctypes.c_void_p(cur.cuda_stream)))

    def empty(self):
        return self.torch.zeros((3, self.n, self.n, self.n // 2 + 1), dtype=self.dtype, device=self.device)

    def to_device(self, a):
        """Copy a host complex array [3, N, N, N/2+1] into a new field tensor."""
        t = self.torch.from_numpy(np.ascontiguousarray(a).astype(
            np.complex64 if self.precision == "fp32" else np.complex128))
        return t.to(self.device)

    def nonlinear(self, u, out=None, shift=None, ps_avg=False):
        self._sync_stream()
        out = self.empty() if out is None else out
        self._check(lib().ns_nonlinear(self.ctx, self._field(u, "u"), self._field(out, "out"),
                                       _dbl3(shift), NS_NL_PS_AVG if ps_avg else 0))
        return out

    def step_rk4(self, u, dt, nsteps=1, forcing=None, step0=0):
        """Lawson RK4 steps in place; forcing: dict(seed=..., injection=1.0) or None."""
        self._sync_stream()
        self._check(lib().ns_step_rk4_trunc(self.ctx, self._field(u, "u"), float(dt), int(nsteps),
                                            _forcing(forcing), int(step0)))
        return u

    def step_ps(self, u, dt, nsteps=1, variant="random", alphas=None, forcing=None, step0=0, stage1=None):
        """Steps in place of one of VARIANTS: the phase-shift RK2 schemes ("exact", "approx",
        "random"), midpoint RK2 and Euler without shifts ("rk2", "euler"), Euler with the
        two-shift average ("euler_ps") and the eight-shift exact RK2 ("exact8").
        alphas: array [nsteps, 3] (random variant) or None; forcing: dict(seed=...,
        injection=1.0) or None (Heun variants only); stage1: a field tensor that receives
        the first-stage state of a single Heun step (for vjp_ps)."""
        self._sync_stream()
        ap = None
        if alphas is not None:
            a = np.ascontiguousarray(np.asarray(alphas, dtype=np.float64).reshape(-1))
            if a.size != 3 * int(nsteps):
                raise ValueError("alphas must have shape [nsteps, 3]")
            ap = a.ctypes.data_as(ctypes.c_void_p)
        self._check(lib().ns_step_rk2_phaseshift(self.ctx, self._field(u, "u"), float(dt), int(nsteps),
                                                 VARIANTS[variant], ap, _forcing(forcing), int(step0),
                                                 None if stage1 is None else self._field(stage1, "stage1")))
        return u

    def _spectra_out(self):
        nsh, h = self.nshells, self.n // 2 + 1
        out = {"e_shell": np.zeros(nsh), "d_shell": np.zeros(nsh), "t_shell": np.zeros(nsh),
               "e_1d": np.zeros((3, h)), "totals": np.zeros(5)}
        so = NSSpectraOut(*[out[k].ctypes.data_as(ctypes.c_void_p) for k in
                            ("e_shell", "d_shell", "t_shell", "e_1d", "totals")])
        return out, so

    def _spectra_status(self, st, out, check_finite):
        if st == NS_ERR_NONFINITE and not check_finite:
            return out
        self._check(st)
        return out

    def spectra(self, u, n_hat=None, check_finite=True):
        self._sync_stream()
        out, so = self._spectra_out()
        st = lib().ns_spectra(self.ctx, self._field(u, "u"),
                              None if n_hat is None else self._field(n_hat, "n_hat"), ctypes.byref(so))
        return self._spectra_status(st, out, check_finite)

    def spectra_async(self, u, n_hat=None):
        """Enqueue the spectra of u (as it is at this point of the stream); spectra_wait returns them."""
        self._sync_stream()
        self._check(lib().ns_spectra_async(self.ctx, self._field(u, "u"),
                                           None if n_hat is None else self._field(n_hat, "n_hat")))

    def spectra_wait(self, check_finite=True):
        out, so = self._spectra_out()
        return self._spectra_status(lib().ns_spectra_wait(self.ctx, ctypes.byref(so)), out, check_finite)

    def vjp_ps(self, u0, lam, dt, variant="random", alpha=None, forcing=None, step=0, stage1=None):
        """In place: lam <- (dS_new/dS_0)^T lam for one phase-shift RK2 step at u0 (forced with
        the draw of `step` when forcing is a dict(seed=..., injection=...)); stage1: the
        step's first-stage state kept by step_ps, which saves one evaluation."""
        self._sync_stream()
        self._check(lib().ns_vjp_rk2_phaseshift(self.ctx, self._field(u0, "u0"), self._field(lam, "lam"),
                                                float(dt), VARIANTS[variant], _dbl3(alpha), _forcing(forcing),
                                                int(step), None if stage1 is None else self._field(stage1, "stage1")))
        return lam

    def budget_start(self, u):
        """Start the FP64 energy budget at state u; every later step updates it on the device."""
        self._sync_stream()
        self._check(lib().ns_budget_start(self.ctx, self._field(u, "u")))

    def budget_stop(self):
        self._check(lib().ns_budget_stop(self.ctx))

    def budget_read(self):
        """{t, E, eps, E0, int_eps, int_p, p_last, residual} (waits for the stream)."""
        self._sync_stream()
        out = np.zeros(NS_BUDGET_LEN)
        self._check(lib().ns_budget_read(self.ctx, out.ctypes.data_as(ctypes.c_void_p)))
        return {k: float(out[i]) for i, k in enumerate(BUDGET_NAMES)}

    def timing(self, enable):
        """Enable or disable per-pass event timing on this context."""
        self._check(lib().ns_timing_enable(self.ctx, 1 if enable else 0))

    def timing_read(self):
        """Per-pass {name: (total ms, launches)} since the previous read (waits for the stream)."""
        ms = np.zeros(len(PASS_NAMES))
        cnt = np.zeros(len(PASS_NAMES), dtype=np.int64)
        self._check(lib().ns_timing_read(self.ctx, ms.ctypes.data_as(ctypes.c_void_p),
                                         cnt.ctypes.data_as(ctypes.c_void_p)))
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(PASS_NAMES)}


def spectra_static(u, n, nu, n_hat=None, check_finite=True):
    """ns_spectra_static: the spectra of u (a [3, N, N, N/2+1] complex64 or complex128 CUDA
    tensor) without a context and without allocating, on torch's current stream."""
    import torch
    prec = NS_FP32 if u.dtype == torch.complex64 else NS_FP64
    shape = (3, n, n, n // 2 + 1)
    for t, name in ((u, "u"), (n_hat, "n_hat")):
        if t is not None and (tuple(t.shape) != shape or not t.is_contiguous() or t.device.type != "cuda"
                              or t.dtype != u.dtype):
            raise ValueError(f"{name} must be a contiguous {u.dtype} CUDA tensor of shape {shape}")
    nsh, h = num_shells(n), n // 2 + 1
    out = {"e_shell": np.zeros(nsh), "d_shell": np.zeros(nsh), "t_shell": np.zeros(nsh),
           "e_1d": np.zeros((3, h)), "totals": np.zeros(5)}
    so = NSSpectraOut(*[out[k].ctypes.data_as(ctypes.c_void_p) for k in
                        ("e_shell", "d_shell", "t_shell", "e_1d", "totals")])
    st = lib().ns_spectra_static(int(n), prec, float(nu), ctypes.c_void_p(u.data_ptr()),
                                 None if n_hat is None else ctypes.c_void_p(n_hat.data_ptr()),
                                 ctypes.c_void_p(torch.cuda.current_stream(u.device).cuda_stream), ctypes.byref(so))
    if st == NS_ERR_NONFINITE and not check_finite:
        return out
    if st != NS_OK:
        raise NSError(st, lib().ns_last_error(None).decode())
    return out


# ---------------------------------------------------------------- the 1D model
SCHEMES_1D = {"euler": 0, "euler_ps": 1, "rk2": 2, "ps_exact": 3, "ps_approx": 4, "rk4": 5}


def _spectra_1d(s, n, name):
    import torch
    h = n // 2 + 1
    if (s.dtype != torch.complex128 or s.dim() != 2 or s.shape[1] != h or not s.is_contiguous()
            or s.device.type != "cuda"):
        raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor of shape [batch, {h}]")
    return ctypes.c_void_p(s.data_ptr()), int(s.shape[0])


def _check1d(st):
    if st != NS_OK:
        raise NSError(st, lib().ns_last_error(None).decode())


def _stream1d(s):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(s.device).cuda_stream)


def model1d_nonlinear(s, n, ct, shift=0.0, out=None):
    """N(S; shift) of the 1D model dS/dt = -S^2 for a batch of spectra s [batch, n/2 + 1]."""
    import torch
    p, b = _spectra_1d(s, n, "s")
    out = torch.empty_like(s) if out is None else out
    q, bo = _spectra_1d(out, n, "out")
    if bo != b:
        raise ValueError("out must have the batch size of s")
    _check1d(lib().ns1d_nonlinear(p, q, int(n), float(ct), b, float(shift), _stream1d(s)))
    return out


def model1d_step(s, n, ct, dt, nsteps=1, scheme="ps_exact"):
    """nsteps steps of one of SCHEMES_1D on a batch of spectra s [batch, n/2 + 1], in place."""
    p, b = _spectra_1d(s, n, "s")
    _check1d(lib().ns1d_step(p, int(n), float(ct), b, float(dt), int(nsteps), SCHEMES_1D[scheme], _stream1d(s)))
    return s
