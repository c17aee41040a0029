"""Accuracy against cost on the GPU: Taylor-Green runs of each scheme at matched
k_max, their 1D energy spectra through the transition, and the spectral error
index of Sec. "Performance and accuracy for a decaying flow" (Eq. quality; its
discrete form in the appendix, with the wavenumber sum starting at k = 1)
against a dealiased reference run.

    python -m paper_2603_08892_amd.quality [--t-start 7 --t-end 12 --every 0.1] [--sweep] [--kmax 108]

prints one JSON object: per run the grid, truncation, error index (percent),
wall time and speedup over the reference (at equal dt, and under the paper's
CFL protocol: CFL 0.4 for the RK2 schemes and 1.0 for RK4, dt proportional to
the grid spacing; the eight-shift scheme is costed with the RK2 CFL number);
and the run's dissipation diagnostics (Sec. "Numerical methods and overview",
Sec. "3D flow: Taylor-Green vortices", Fig. 4): the largest dissipation eps_max
and its time, the Kolmogorov length eta~ = (nu^3 / eps_max)^(1/4) and k_max eta~,
and at the time of eps_max the nonlinear energy flux Pi(k) = sum_{k' > k} T(k')
(T of the run's own dealiased nonlinear term) and the cumulative dissipation
sum_{k' <= k} D(k') / eps, from the FP64 spectra of the library.
"""

import argparse
import json
import sys
import time

import numpy as np

from . import inputs, ns

NU, DT = 1.0 / 1600.0, 2e-3
KMAX = 63                      # largest |k_i| retained with k^2 <= 4095

# name: (scheme, N, C_t, CFL number of the scheme, mask); every run keeps k^2 <= 4095
RUNS = {
    "rk4_192_reference": ("rk4", 192, 2.0 / 3.0, 1.0, "sphere"),
    "ps_random_128": ("random", 128, 1.0, 0.4, "sphere"),
    "ps_approx_128": ("approx", 128, 1.0, 0.4, "sphere"),
    "ps_exact_128": ("exact", 128, 1.0, 0.4, "sphere"),
    "rk4_128_aliased": ("rk4", 128, 1.0, 1.0, "sphere"),
}
# the truncation sweep at the same k_max (the grids of Table S1 scaled to k_max = 64):
# C_t = 128 / N, and the "no_multiple_aliases" truncation at C_t = 1 (Fig. 7b); plain
# midpoint RK2 with 2/3 truncation (the fourth scheme the paper compares) and the
# eight-shift exact RK2 at C_t = 1 (alias-free for every truncation, eight evaluations)
SWEEP = {
    "rk2_192": ("rk2", 192, 2.0 / 3.0, 0.4, "sphere"),
    "ps_exact8_128": ("exact8", 128, 1.0, 0.4, "sphere"),
    "ps_random_128_nma": ("random", 128, 1.0, 0.4, "no_multiple_aliases"),
    "ps_exact_128_nma": ("exact", 128, 1.0, 0.4, "no_multiple_aliases"),
    "ps_random_144": ("random", 144, 128 / 144, 0.4, "sphere"),
    "ps_exact_144": ("exact", 144, 128 / 144, 0.4, "sphere"),
    "ps_random_160": ("random", 160, 0.8, 0.4, "sphere"),
    "ps_exact_160": ("exact", 160, 0.8, 0.4, "sphere"),
}
REFERENCE = "rk4_192_reference"

# k_max = 108 (k^2 <= 11663), the resolution of Table S1: RK4 on 324^3 with 2/3
# truncation as the reference; the grids of the table that are 2^a 3^b 5^c
# (216 at C_t = 1, 240 at 0.9; 270 at 0.8 beside them) and 256 at C_t = 27/32.
# Every grid here runs the specialised passes.
KMAX108 = 107
RUNS108 = {
    "rk4_324_reference": ("rk4", 324, 2.0 / 3.0, 1.0, "sphere"),
    "ps_random_216": ("random", 216, 1.0, 0.4, "sphere"),
    "ps_exact_216": ("exact", 216, 1.0, 0.4, "sphere"),
    "ps_random_240": ("random", 240, 0.9, 0.4, "sphere"),
    "ps_exact_240": ("exact", 240, 0.9, 0.4, "sphere"),
    "ps_random_270": ("random", 270, 0.8, 0.4, "sphere"),
    "ps_random_256": ("random", 256, 216 / 256, 0.4, "sphere"),
    "ps_exact_256": ("exact", 256, 216 / 256, 0.4, "sphere"),
    "rk2_324": ("rk2", 324, 2.0 / 3.0, 0.4, "sphere"),
}
REFERENCE108 = "rk4_324_reference"


def error_index(e1d, e1d_ref, kmax):
    """Mean over the three directions of the time- and 1/k-weighted mean of
    100 |E_ref - E| / E_ref over the 1D wavenumbers 1..kmax.
    e1d, e1d_ref: arrays [samples, 3, >= kmax + 1]."""
    e = np.asarray(e1d, dtype=np.float64)[:, :, 1:kmax + 1]
    r = np.asarray(e1d_ref, dtype=np.float64)[:, :, 1:kmax + 1]
    if e.shape != r.shape or e.shape[0] == 0:
        raise ValueError("need the same, non-zero number of samples in both runs")
    if not np.all(r > 0):
        raise ValueError("the reference spectra have empty bins in 1..kmax")
    w = 1.0 / np.arange(1, kmax + 1)
    rel = 100.0 * np.abs(r - e) / r
    per_dir = (rel * w).sum(axis=(0, 2)) / (e.shape[0] * w.sum())
    return float(per_dir.mean()), per_dir.tolist()


def run_taylor_green(scheme, n, ct, t_start, t_end, every, nu=NU, dt=DT, seed=2026, kmax=KMAX, mask="sphere",
                     diagnostics=None):
    """Time-step the Taylor-Green field to t_end; returns the sample times, the 1D
    spectra [samples, 3, kmax + 1] taken every `every` time units from t_start, and
    the wall time of the whole run (stepping and sampling).  With a dict as
    `diagnostics`, it also receives the dissipation diagnostics of the run at the
    sample of largest eps (dissipation_diagnostics)."""
    import torch
    s = ns.Solver(n, nu, ct, mask=mask, precision="fp32", seed=seed)
    u = s.to_device(inputs.taylor_green(n))
    nsteps = int(round(t_end / dt))
    first, stride = int(round(t_start / dt)), max(1, int(round(every / dt)))
    times, spec, eps = [], [], []
    # with diagnostics: the state at every sample goes into one of two buffers; once
    # the sample's eps is known (one sample later) the state of the largest eps is kept
    bufs = [s.empty(), s.empty()] if diagnostics is not None else None
    best = s.empty() if diagnostics is not None else None

    def advance(i, k):
        if scheme == "rk4":
            s.step_rk4(u, dt, k)
        elif scheme == "random":
            s.step_ps(u, dt, k, "random", step0=i)
        else:
            s.step_ps(u, dt, k, scheme)

    def collect():
        sp = s.spectra_wait()
        spec.append(sp["e_1d"][:, :kmax + 1].copy())
        eps.append(float(sp["totals"][1]))
        j = len(eps) - 1
        if bufs is not None and eps[j] == max(eps):
            best.copy_(bufs[j % 2])

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # the steps up to the next sample in one call; each sample is collected once the
    # following steps are queued behind it
    k, pending = 0, False
    while k < nsteps:
        nxt = first if k < first else first + ((k - first) // stride + 1) * stride
        nxt = min(max(nxt, k + 1), nsteps)
        advance(k, nxt - k)
        k = nxt
        if pending:
            collect()
            pending = False
        if k >= first and (k - first) % stride == 0:
            s.spectra_async(u)
            if bufs is not None:
                bufs[len(times) % 2].copy_(u)
            times.append(k * dt)
            pending = True
    if pending:
        collect()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if diagnostics is not None and eps:
        jmax = int(np.argmax(eps))
        diagnostics.update(dissipation_diagnostics(s, best, scheme, nu, ct * n / 2.0))
        diagnostics["t_eps_max"] = float(times[jmax])
    return np.array(times), np.array(spec), wall


def dissipation_diagnostics(s, u, scheme, nu, kmax):
    """eps, eta~ = (nu^3 / eps)^(1/4) and k_max eta~ of the state u, the nonlinear
    energy flux through each shell Pi(n) = sum_{n' > n} T(n') and the cumulative
    dissipation C(n) = sum_{n' <= n} D(n') / eps (Fig. 4b), where T is the transfer of
    the scheme's own dealiased nonlinear term (the two-shift average for the phase-shift
    schemes, the truncated product otherwise) and D the dissipation spectrum."""
    nh = s.nonlinear(u, ps_avg=scheme in ("random", "approx", "exact", "exact8", "euler_ps"))
    sp = s.spectra(u, nh)
    e = float(sp["totals"][1])
    t = sp["t_shell"]
    flux = np.concatenate([np.cumsum(t[::-1])[::-1][1:], [0.0]])
    eta = (nu ** 3 / e) ** 0.25
    return {"eps_max": e, "eta_tilde": eta, "kmax_eta": kmax * eta, "flux": flux.tolist(),
            "cum_dissipation": (np.cumsum(sp["d_shell"]) / e).tolist(), "transfer_total": float(sp["totals"][3])}


def compare(t_start, t_end, every, runs=None, log=sys.stderr, table=None, reference=REFERENCE, kmax=KMAX):
    table = {**RUNS, **SWEEP} if table is None else table
    runs = list(RUNS) if runs is None else runs
    if reference not in runs:
        runs = [reference] + runs
    out = {}
    for name in runs:
        scheme, n, ct, _, mask = table[name]
        diag = {}
        tt, sp, wall = run_taylor_green(scheme, n, ct, t_start, t_end, every, mask=mask, kmax=kmax,
                                        diagnostics=diag)
        out[name] = {"scheme": scheme, "n": n, "ct": round(ct, 6), "mask": mask, "wall_s": wall, "times": tt,
                     "spec": sp, "diag": diag}
        print(f"[quality] {name}: {len(tt)} samples, {wall:.2f} s", file=log, flush=True)
    ref = out[reference]
    _, nr, _, cfl_r, _ = table[reference]
    rows = {}
    for name, r in out.items():
        _, n, _, cfl, _ = table[name]
        err, dirs = error_index(r["spec"], ref["spec"], kmax)
        eq = ref["wall_s"] / r["wall_s"]
        # CFL protocol: dt = CFL dx / U, so the ratio of step counts is (cfl n_ref) / (cfl_ref n)
        rows[name] = {"scheme": r["scheme"], "n": n, "ct": r["ct"], "mask": r["mask"], "error_pct": round(err, 4),
                      "error_pct_xyz": [round(d, 4) for d in dirs], "wall_s": round(r["wall_s"], 4),
                      "speedup_equal_dt": round(eq, 3),
                      "speedup_cfl_protocol": round(eq * (cfl * nr) / (cfl_r * n), 3)}
        d = r["diag"]
        if d:
            rows[name].update({"eps_max": round(d["eps_max"], 8), "t_eps_max": round(d["t_eps_max"], 4),
                               "eta_tilde": round(d["eta_tilde"], 8), "kmax_eta": round(d["kmax_eta"], 4),
                               "flux": [round(v, 8) for v in d["flux"][:kmax + 2]],
                               "cum_dissipation": [round(v, 6) for v in d["cum_dissipation"][:kmax + 2]]})
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--t-start", type=float, default=7.0)
    ap.add_argument("--t-end", type=float, default=12.0)
    ap.add_argument("--every", type=float, default=0.1)
    ap.add_argument("--sweep", action="store_true", help="also the truncation sweep at the same k_max")
    ap.add_argument("--kmax", type=int, default=64, choices=(64, 108), help="k_max of the comparison")
    args = ap.parse_args()
    if args.kmax == 108:
        rows = compare(args.t_start, args.t_end, args.every, list(RUNS108), table=RUNS108,
                       reference=REFERENCE108, kmax=KMAX108)
        ref, k2 = REFERENCE108, 11663
    else:
        rows = compare(args.t_start, args.t_end, args.every, list(RUNS) + (list(SWEEP) if args.sweep else []))
        ref, k2 = REFERENCE, 4095
    print(json.dumps({"workload": f"Taylor-Green nu=1/1600 dt={DT} t in [{args.t_start}, {args.t_end}], "
                                  f"k_max={args.kmax} (k^2 <= {k2}), 1D spectra every {args.every}",
                      "reference": ref, "runs": rows}))


if __name__ == "__main__":
    main()
