"""Benchmark: Taylor-Green transition at matched k_max, one MI355X.

Workload (the 128^3 Taylor-Green configuration): u0 from Eq. T-G-init, nu = 1/1600,
dt = 2e-3, FP32 fields, FP64 spectra every 10 steps.  Phase-shift RK2 (random,
approx, exact) runs on N = 128 with C_t = 1; the 2/3-truncated RK4 baseline runs
on N = 192; both keep exactly the modes |k|^2 <= 4095 (k_max = 64).  A "step" is
one time step of a scheme (every evaluation of the nonlinear term with its
transforms, shifts, product, projection, truncation and Runge-Kutta update,
plus the spectra every 10th step), inputs resident in HBM.  As in a time loop,
the 10 steps between two spectra are one library call.

    python bench.py [--gpus 1] [--steps 200] [--warmup 3] [--no-cpu-baseline] [--no-hit512]

Prints ONE JSON line.  `value` is the PS-RK2 random throughput on its own grid in
Mgridpts*RKsteps/s (N^3 steps / s / 1e6); the other schemes and the matched-k_max
speedups are in `schemes` and `speedup`.  `roofline` is the dominant pass of the
PS-RK2 random step: algorithmic bytes per launch over its average launch time,
from HIP events recorded on the library's stream during a second timed run of
the same steps.  `adjoint` times the gradient workload (50 PS-RK2 steps on 128^3,
checkpoint every 10, hand-written step adjoints).  `hit_512` times the forced-HIT pairing
at k_max = 512/3 (RK4 on 512^3 against PS-RK2 random on 384^3).  `cpu_baseline` times the FP64
oracle on a few steps of the same workload on the host cores.
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mgridpts·RKsteps/s at matched kmax (PS-RK2 vs 2/3-RK4); HBM GB/s % of peak"
HBM_PEAK_GBS = 8000.0
NU, DT = 1.0 / 1600.0, 2e-3
NP, NR = 128, 192
SPEC_EVERY = 10
ELEM = 8  # bytes of one FP32 complex


def geometry(n, k2max):
    """Counts that fix the algorithmic bytes of the pruned passes (sphere k^2 <= k2max)."""
    kmax = int(np.floor(np.sqrt(k2max)))
    kzn = kmax + 1
    i = np.arange(n)
    k = np.where(i < n // 2, i, i - n)
    kz = np.arange(kzn)
    disk = (k[:, None] ** 2 + kz[None, :] ** 2) <= k2max          # (k_y, k_z) lines
    A = int(disk.sum())
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + kz[None, None, :] ** 2
    R = int((k2 <= k2max).sum())                                   # retained half-spectrum modes
    return {"n": n, "kzn": kzn, "lines": A, "retained": R, "h": n // 2 + 1}


def pass_bytes(g):
    """Algorithmic HBM bytes per launch of each pass of the chained PS-RK2 random step.

    x_inverse          reads the 3 retained components, writes 6 fields on the active lines
                       (only the first evaluation of a call runs it on its own)
    y_inverse          reads the 6 fields on the active lines, writes the full (x, y) planes k_z < kzn
    z_fused            reads 6 and writes 3 fields on those planes
    y_forward          reads 3 fields on the planes, writes them on the active lines
    x_forward_epilogue the last stage of a call: reads 3 fields on the active lines and the
                       partial update (retained modes), writes the state's whole half spectrum
    x_forward_inverse  every other stage: reads 3 fields on the active lines and one stage
                       operand, writes one stage output (retained modes; S1 only feeds the
                       next evaluation and is not stored), then the next evaluation's 6
                       fields on the active lines
    """
    n, A, R, kzn, h = g["n"], g["lines"], g["retained"], g["kzn"], g["h"]
    planes = n * n * kzn
    return {
        "x_inverse": (3 * R + 6 * A * n) * ELEM,
        "y_inverse": (6 * A * n + 6 * planes) * ELEM,
        "z_fused": (6 * planes + 3 * planes) * ELEM,
        "y_forward": (3 * planes + 3 * A * n) * ELEM,
        "x_forward_epilogue": (3 * A * n + 3 * R + 3 * n * n * h) * ELEM,
        "x_forward_inverse": (9 * A * n + 6 * R) * ELEM,
    }


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_08892_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def committed_traffic(kernel, workload):
    """HBM traffic per launch from the committed counter summary, if it was taken on
    the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("per_launch_bytes", {}).get(f"{workload}:{kernel}")


def run_scheme(torch, ns, inputs, name, n, ct, steps, warmup, timing=False, nu=NU, dt=DT, u0=None,
               forcing=None):
    """Time `steps` steps of one scheme (after `warmup` untimed ones) from u0 (host array;
    default the Taylor-Green state); forcing applies to the random scheme."""
    s = ns.Solver(n, nu, ct, precision="fp32", seed=2026)
    u0 = s.to_device(inputs.taylor_green(n) if u0 is None else u0)
    u = u0.clone()

    def advance(i, k):
        """k steps from step index i in one library call."""
        if name == "rk4":
            s.step_rk4(u, dt, k)
        elif name == "exact":
            s.step_ps(u, dt, k, "exact")
        elif name == "approx":
            s.step_ps(u, dt, k, "approx")
        else:
            s.step_ps(u, dt, k, "random", forcing=forcing, step0=i)

    def run(nsteps):
        # a time loop: the steps between two spectra in one call each; the host collects
        # each spectra result once the next steps are queued behind it
        i, pending = 0, False
        while i < nsteps:
            k = min(SPEC_EVERY - i % SPEC_EVERY, nsteps - i)
            advance(i, k)
            i += k
            if pending:
                s.spectra_wait()
                pending = False
            if i % SPEC_EVERY == 0:
                s.spectra_async(u)
                pending = True
        if pending:
            s.spectra_wait()

    run(warmup)
    u.copy_(u0)
    torch.cuda.synchronize()
    if timing:
        s.timing(True)
        s.timing_read()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    run(steps)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    passes = s.timing_read() if timing else None
    E = s.spectra(u)["totals"][0]
    return ms, passes, float(E)


def adjoint_run(torch, ns, inputs, reps=3):
    """The adjoint workload: gradient of the final kinetic energy after 50 PS-RK2 random
    steps on 128^3 (Taylor-Green plus a 1e-2 seeded perturbation), checkpoint every 10
    steps (forward with checkpoints, then per segment the recomputed states and the step
    adjoints in reverse).  Median wall time of `reps` gradients after one warm-up."""
    from paper_2603_08892_amd.autograd import PSRK2Function, final_energy
    n, steps, every = NP, 50, 10
    s = ns.Solver(n, NU, 1.0, precision="fp32", seed=5)
    u0 = s.to_device(inputs.tg_perturbed(n, 3, ns.retained_bound(n, 1.0)))
    al = inputs.random_shifts(11, steps)

    def forward():
        with torch.no_grad():
            return PSRK2Function.apply(u0, s, DT, steps, "random", al, every)

    def gradient():
        x = u0.clone().requires_grad_(True)
        final_energy(PSRK2Function.apply(x, s, DT, steps, "random", al, every)).backward()
        return x.grad

    def timed(f):
        out = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f()
            torch.cuda.synchronize()
            out.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(out))

    gradient()
    fwd, grad = timed(forward), timed(gradient)
    return {"workload": "adjoint_128: d(final kinetic energy)/d(u0) after 50 PS-RK2 random steps on 128^3 "
                        "Taylor-Green + 1e-2 perturbation, checkpoint every 10 steps",
            "ms_per_gradient": round(grad, 3), "ms_forward_only": round(fwd, 3),
            "gradient_over_forward": round(grad / fwd, 2)}


def hit512_run(torch, ns, inputs, steps, warmup):
    """The forced-HIT pairing at k_max = 512/3 (K2max = 29127): 2/3-truncated RK4 on 512^3
    against PS-RK2 random on 384^3 with C_t = 8/9 (the coarser grid with the same retained
    sphere), from the seeded HIT state E(k) ~ k^4 exp(-2 (k/4)^2), nu from k_max eta = 1 at
    unit injection, dt = 1e-3.  The PS run carries the stochastic shell forcing; the RK4
    step of the library has no forcing term, so its run is unforced (the forcing adds a
    small per-step kernel to the PS side only)."""
    kmax = 512 / 3
    nu, dt = kmax ** (-4.0 / 3.0), 1e-3
    runs = {"rk4_512": ("rk4", 512, 2.0 / 3.0, None), "ps_random_384": ("random", 384, kmax / 192,
                                                                          {"seed": 13, "injection": 1.0})}
    out = {}
    for key, (name, n, ct, fo) in runs.items():
        k2 = ns.retained_bound(n, ct)
        u0 = inputs.hit_initial(n, 21, k2)
        ms, _, _ = run_scheme(torch, ns, inputs, name, n, ct, steps, warmup, nu=nu, dt=dt, u0=u0, forcing=fo)
        del u0
        torch.cuda.empty_cache()
        out[key] = {"n": n, "ct": round(ct, 6), "k2max": k2, "ms_per_step": round(ms / steps, 4),
                    "mgridpts_steps_per_s": round(n ** 3 * steps / (ms * 1e-3) / 1e6, 1)}
        print(f"[bench] hit512 {key}: {ms / steps:.3f} ms/step", file=sys.stderr, flush=True)
    eq = out["rk4_512"]["ms_per_step"] / out["ps_random_384"]["ms_per_step"]
    out["workload"] = ("forced_hit_kmax_512/3: RK4 on 512^3 C_t=2/3 vs PS-RK2 random on 384^3 C_t=8/9 "
                       f"(K2max={out['rk4_512']['k2max']}), nu={nu:.4g}, dt={dt}, spectra every 10 steps")
    out["speedup_ps_random_vs_rk4"] = {"equal_dt": round(eq, 3), "cfl_protocol": round(eq * 0.4 * 512 / 384, 3)}
    return out


def cpu_baseline(budget_s=20.0):
    """The FP64 oracle on the same Taylor-Green state, PS-RK2 random on 128^3: a bounded
    sample of steps (stops once `budget_s` of host time is used)."""
    from oracle import forcing, grid, schemes, transforms
    from oracle import nonlinear as onl
    from paper_2603_08892_amd import inputs
    m = grid.mask(NP, 1.0)
    model = onl.NSModel(NP, NU, m)
    u = inputs.taylor_green(NP)
    t0 = time.perf_counter()
    nsteps = 0
    while True:
        u = schemes.ps_heun(model, u, DT, forcing.random_shift(2026, nsteps))
        nsteps += 1
        if time.perf_counter() - t0 > budget_s or nsteps >= 50:
            break
    dt = time.perf_counter() - t0
    return {"value": NP ** 3 * nsteps / dt / 1e6, "unit": "Mgridpts*RKsteps/s", "cores": transforms.WORKERS,
            "kind": "oracle",
            "sample": f"{nsteps} steps of PS-RK2 random on the 128^3 Taylor-Green state (FP64 NumPy/SciPy, "
                      f"scipy.fft workers={transforms.WORKERS}), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the timing of the adjoint workload")
    ap.add_argument("--schemes", default="random,approx,exact,rk4")
    ap.add_argument("--no-hit512", action="store_true",
                    help="skip the forced-HIT pairing at k_max = 512/3 (RK4 on 512^3, PS-RK2 on 384^3)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first run 3 elementwise copies of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU slab "
              "decomposition is a design, not a build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_08892_amd import inputs, ns
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    ns.lib()
    if args.copy_mb:
        # counter calibration: an elementwise kernel that reads and writes copy_mb MiB once
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    K, W = args.steps, args.warmup
    want = args.schemes.split(",")
    grids = {"random": (NP, 1.0), "approx": (NP, 1.0), "exact": (NP, 1.0), "rk4": (NR, 2.0 / 3.0)}
    results = {}
    for name in want:
        n, ct = grids[name]
        ms, _, E = run_scheme(torch, ns, inputs, name, n, ct, K, W)
        results[name] = {"n": n, "ct": round(ct, 6), "ms_per_step": ms / K,
                         "mgridpts_steps_per_s": n ** 3 * K / (ms * 1e-3) / 1e6, "energy_end": E}
        print(f"[bench] {name}: N={n} {ms / K:.4f} ms/step", file=sys.stderr, flush=True)

    # live per-pass timing of the headline scheme for the roofline
    head = "random" if "random" in want else want[0]
    n, ct = grids[head]
    _, passes, _ = run_scheme(torch, ns, inputs, head, n, ct, K, W, timing=True)
    g = geometry(n, 4095)
    pb = pass_bytes(g)
    per = {}
    for pname, (tot_ms, cnt) in passes.items():
        if cnt:
            avg = tot_ms / cnt
            per[pname] = {"avg_ms": avg, "launches": cnt, "bytes": pb[pname],
                          "gbs": pb[pname] / (avg * 1e-3) / 1e9}
    dom = max(per, key=lambda k: per[k]["avg_ms"] * per[k]["launches"])
    d = per[dom]
    workload = "taylor_green_128_ps_random"
    traffic = committed_traffic(dom, workload)
    roof = {"bound": "hbm", "achieved": round(d["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(d["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
            "bytes_per_launch": d["bytes"], "avg_launch_ms": round(d["avg_ms"], 5),
            "passes": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                       for k, v in per.items()}}

    r = results[head]
    speed = {}
    if "rk4" in results:
        for sname in ("random", "approx", "exact"):
            if sname in results:
                eq = results["rk4"]["ms_per_step"] / results[sname]["ms_per_step"]
                speed[f"ps_{sname}_vs_rk4"] = {"equal_dt": round(eq, 3), "cfl_protocol": round(eq * 0.4 * NR / NP, 3)}
    out = {
        "metric": METRIC, "value": round(r["mgridpts_steps_per_s"], 1), "unit": "Mgridpts*RKsteps/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": round(r["ms_per_step"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "taylor_green_matched_kmax: PS-RK2 on 128^3 C_t=1 vs RK4 on 192^3 C_t=2/3, "
                               "K2max=4095, nu=1/1600, dt=2e-3, spectra every 10 steps",
                   "scheme": f"ps_{head}", "n": r["n"], "k2max": 4095},
        "schemes": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in results.items()},
        "speedup": speed,
        "roofline": roof,
    }
    if not args.no_adjoint:
        out["adjoint"] = adjoint_run(torch, ns, inputs)
    if not args.no_hit512:
        out["hit_512"] = hit512_run(torch, ns, inputs, K, W)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
