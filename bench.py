"""Benchmark of the dealiased nonlinear term inside the Runge-Kutta step, one MI355X.

Workloads (all inputs synthetic and seeded, resident in HBM before the timed region):
  tg128   Taylor-Green at matched k_max = 64 (the headline): u0 from Eq. T-G-init,
          nu = 1/1600, dt = 2e-3, FP32 fields, FP64 spectra every 10 steps;
          PS-RK2 random / approx / exact on 128^3 at C_t = 1 against 2/3-truncated
          RK4 on 192^3 (both keep exactly |k|^2 <= 4095).  `value` is PS-RK2
          random on its own grid in Mgridpts*RKsteps/s.
  hit256  forced HIT on 256^3: seeded field with E(k) ~ k^4 exp(-2 (k/4)^2), E = 1.5,
          shell forcing at unit injection, PS-RK2 random at C_t = 1,
          nu = 128^(-4/3) (k_max eta = 1), dt frozen from CFL 0.4 at t = 0,
          500 steps; FP64 spectra every 10 steps; the FP64 energy budget on the GPU
          in a second run of the same steps.  The `roofline` object is the pass with
          the largest total time of this run (N >= 256: the working set is far beyond
          the 256 MB last-level cache).
  hit512  forced HIT at k_max = 512/3: RK4 on 512^3 at C_t = 2/3 against PS-RK2 random
          on 360^3 at C_t = 0.948 and on 384^3 at C_t = 8/9 (all three keep
          |k|^2 <= 29127), the same initial field and the same seeded forcing, dt
          frozen from CFL (1.0 for RK4, 0.4 for PS-RK2), 200 steps, FP64 spectra every
          10 steps.
  adjoint gradient of the final kinetic energy after 50 PS-RK2 random steps on 128^3,
          checkpoint every 10 (hand-written step adjoints).
  tg32    Taylor-Green 32^3 FP64, 10 steps of RK4 (C_t = 2/3) and PS exact (C_t = 2/3
          and 1): the FP64 oracle's wall time on the host and the GPU's FP64 passes.
A "step" is one time step of a scheme: every evaluation of the nonlinear term with its
transforms, shifts, product, projection, truncation, forcing and Runge-Kutta update.  As
in a time loop, the 10 steps between two spectra are one library call.

    python bench.py [--gpus 1] [--steps 200] [--warmup 3] [--only tg128,hit256,...]
                    [--no-cpu-baseline] [--copy-mb MiB]

Prints ONE JSON line.  `cpu_baseline` times the FP64 oracle on a bounded sample of the
headline workload on the host cores.
"""

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2603_08892_amd.profsum import geometry, pass_bytes, source_hash  # noqa: E402  (the byte model)

METRIC = "Mgridpts·RKsteps/s at matched kmax (PS-RK2 vs 2/3-RK4); HBM GB/s % of peak"
HBM_PEAK_GBS = 8000.0
NU, DT = 1.0 / 1600.0, 2e-3
NP, NR = 128, 192
SPEC_EVERY = 10
WORKLOADS = ("tg128", "hit256", "hit512", "adjoint", "tg32")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)



def committed_traffic(kernel, workload, n):
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
    return rec.get("per_launch_bytes", {}).get(f"{workload}@{n}:{kernel}")


def cfl_dt(u_hat, n, cfl):
    """dt = C dx / max_x (|u_x| + |u_y| + |u_z|) at t = 0 (dx = 2 pi / N), from the
    physical velocity on the N^3 grid (set-up only, on the host)."""
    import scipy.fft as sfft
    workers = len(os.sched_getaffinity(0))
    umax = np.zeros((n, n, n))
    for c in range(3):
        umax += np.abs(sfft.irfftn(u_hat[c], s=(n, n, n), norm="forward", workers=workers))
    return cfl * (2 * np.pi / n) / float(umax.max())


def run_scheme(torch, ns, name, n, ct, steps, warmup, u0, nu=NU, dt=DT, forcing=None, timing=False,
               budget=False, seed=2026):
    """Time `steps` steps of one scheme (after `warmup` untimed ones) from the host state u0,
    the steps between two spectra in one call each (a time loop: the host collects each
    spectra result once the next steps are queued).  Returns ms, per-pass timing (if
    timing), the final energy and the budget record (if budget)."""
    s = ns.Solver(n, nu, ct, precision="fp32", seed=seed)
    start = s.to_device(u0)
    u = start.clone()

    def advance(i, k):
        if name == "rk4":
            s.step_rk4(u, dt, k, forcing=forcing, step0=i)
        else:
            s.step_ps(u, dt, k, name, forcing=forcing if name in ("random", "approx") else None, step0=i)

    def run(nsteps):
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
    u.copy_(start)
    torch.cuda.synchronize()
    if timing:
        s.timing(True)
        s.timing_read()
    if budget:
        s.budget_start(u)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    run(steps)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    passes = s.timing_read() if timing else None
    rec = s.budget_read() if budget else None
    E = s.spectra(u)["totals"][0]
    del s, u, start
    torch.cuda.empty_cache()
    return ms, passes, float(E), rec


def roofline(passes, n, k2max, workload):
    pb = pass_bytes(geometry(n, k2max))
    per = {}
    for pname, (tot_ms, cnt) in passes.items():
        if cnt:
            avg = tot_ms / cnt
            per[pname] = {"avg_ms": avg, "launches": cnt, "bytes": pb[pname],
                          "gbs": pb[pname] / (avg * 1e-3) / 1e9}
    dom = max(per, key=lambda k: per[k]["avg_ms"] * per[k]["launches"])
    d = per[dom]
    return {"bound": "hbm", "achieved": round(d["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(d["gbs"] / HBM_PEAK_GBS, 4), "traffic": committed_traffic(dom, workload, n),
            "kernel": dom, "workload": workload, "bytes_per_launch": d["bytes"],
            "avg_launch_ms": round(d["avg_ms"], 5),
            "passes": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                       for k, v in per.items()}}


def tg128(torch, ns, inputs, K, W, want):
    grids = {"random": (NP, 1.0), "approx": (NP, 1.0), "exact": (NP, 1.0), "rk4": (NR, 2.0 / 3.0)}
    results = {}
    for name in want:
        n, ct = grids[name]
        ms, _, E, _ = run_scheme(torch, ns, name, n, ct, K, W, inputs.taylor_green(n))
        results[name] = {"n": n, "ct": round(ct, 6), "ms_per_step": ms / K,
                         "mgridpts_steps_per_s": n ** 3 * K / (ms * 1e-3) / 1e6, "energy_end": E}
        log(f"tg128 {name}: N={n} {ms / K:.4f} ms/step")
    speed = {}
    if "rk4" in results:
        for sname in ("random", "approx", "exact"):
            if sname in results:
                eq = results["rk4"]["ms_per_step"] / results[sname]["ms_per_step"]
                speed[f"ps_{sname}_vs_rk4"] = {"equal_dt": round(eq, 3), "cfl_protocol": round(eq * 0.4 * NR / NP, 3)}
    roof = None
    if "random" in want:
        _, passes, _, _ = run_scheme(torch, ns, "random", NP, 1.0, K, W, inputs.taylor_green(NP), timing=True)
        roof = roofline(passes, NP, 4095, "taylor_green_128_ps_random")
        roof["note"] = "128^3 working set inside the 256 MB last-level cache: not an HBM figure"
    return results, speed, roof


def hit256(torch, ns, inputs, steps, warmup):
    """Config 3: forced HIT, PS-RK2 random on 256^3, 500 steps."""
    n, ct = 256, 1.0
    nu = (ct * n / 2) ** (-4.0 / 3.0)
    k2 = ns.retained_bound(n, ct)
    u0 = inputs.hit_field(n, 21, k2)
    dt = cfl_dt(u0, n, 0.4)
    fo = {"seed": 13, "injection": 1.0}
    ms, _, E, _ = run_scheme(torch, ns, "random", n, ct, steps, warmup, u0, nu=nu, dt=dt, forcing=fo, seed=8)
    log(f"hit256: {ms / steps:.3f} ms/step")
    msb, _, _, rec = run_scheme(torch, ns, "random", n, ct, steps, warmup, u0, nu=nu, dt=dt, forcing=fo, seed=8,
                                budget=True)
    log(f"hit256 with the energy budget: {msb / steps:.3f} ms/step, residual {rec['residual']:.3e}")
    tsteps = min(steps, 100)
    _, passes, _, _ = run_scheme(torch, ns, "random", n, ct, tsteps, warmup, u0, nu=nu, dt=dt, forcing=fo,
                                 seed=8, timing=True)
    roof = roofline(passes, n, k2, "forced_hit_256_ps_random")
    out = {"workload": f"forced_hit_256: PS-RK2 random split forcing on 256^3 C_t=1 (K2max={k2}), "
                       f"nu={nu:.4g}, dt={dt:.4g} (CFL 0.4 at t=0), unit injection, spectra every 10 steps",
           "n": n, "steps": steps, "dt": dt, "nu": nu, "ms_per_step": round(ms / steps, 4),
           "mgridpts_steps_per_s": round(n ** 3 * steps / (ms * 1e-3) / 1e6, 1),
           "ms_per_step_with_budget": round(msb / steps, 4), "energy_end": E,
           "budget": {k: (round(v, 9) if isinstance(v, float) else v) for k, v in rec.items()},
           "budget_drift_rel": rec["residual"] / (rec["E0"] + rec["int_p"])}
    return out, roof


def hit512(torch, ns, inputs, steps, warmup):
    """RK4 on 512^3 against PS-RK2 random on 360^3 (the coarsest grid of radices 2, 3
    and 5 that holds k_max = 512/3 at C_t <= 1) and on 384^3, all forced with the same
    seeded forcing from the same initial field, dt frozen from CFL."""
    kmax = 512 / 3
    nu = kmax ** (-4.0 / 3.0)
    fo = {"seed": 13, "injection": 1.0}
    runs = {"rk4_512": ("rk4", 512, 2.0 / 3.0, 1.0), "ps_random_360": ("random", 360, kmax / 180, 0.4),
            "ps_random_384": ("random", 384, kmax / 192, 0.4)}
    out = {}
    for key, (name, n, ct, cfl) in runs.items():
        k2 = ns.retained_bound(n, ct)
        u0 = inputs.hit_field(n, 21, k2)
        dt = cfl_dt(u0, n, cfl)
        ms, _, _, _ = run_scheme(torch, ns, name, n, ct, steps, warmup, u0, nu=nu, dt=dt, forcing=fo, seed=8)
        del u0
        out[key] = {"n": n, "ct": round(ct, 6), "k2max": k2, "cfl": cfl, "dt": dt,
                    "ms_per_step": round(ms / steps, 4),
                    "mgridpts_steps_per_s": round(n ** 3 * steps / (ms * 1e-3) / 1e6, 1)}
        log(f"hit512 {key}: {ms / steps:.3f} ms/step, dt {dt:.4g}")
    r = out["rk4_512"]
    out["workload"] = ("forced_hit_kmax_512/3: RK4 on 512^3 C_t=2/3 vs PS-RK2 random on 360^3 C_t=0.948 "
                       f"and on 384^3 C_t=8/9 (K2max={r['k2max']}), same initial field and seeded forcing, "
                       f"nu={nu:.4g}, dt frozen from CFL 1.0 (RK4) and 0.4 (PS-RK2) at t=0, spectra every 10 steps")
    for key in ("ps_random_360", "ps_random_384"):
        p = out[key]
        eq = r["ms_per_step"] / p["ms_per_step"]
        out[f"speedup_{key}_vs_rk4"] = {"equal_dt": round(eq, 3), "cfl_protocol": round(eq * p["dt"] / r["dt"], 3)}
    return out


def adjoint_run(torch, ns, inputs, reps=3):
    """The adjoint workload: gradient of the final kinetic energy after 50 PS-RK2 random
    steps on 128^3 (Taylor-Green plus a 1e-2 seeded perturbation), checkpoint every 10
    steps.  Median wall time of `reps` gradients after one warm-up."""
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


TG32_RUNS = (("rk4_2/3", "rk4", 2.0 / 3.0), ("ps_exact_2/3", "exact", 2.0 / 3.0), ("ps_exact_1", "exact", 1.0))


def tg32(torch, ns, inputs):
    """Config 1 on the GPU: Taylor-Green on 32^3 in FP64, nu = 1/1600, dt = 1e-3, 10 steps
    of RK4 at C_t = 2/3 and of PS exact at C_t = 2/3 and 1 (one call of 10 steps), the FP64
    instantiation of the passes (the oracle's time for the same runs is in cpu_baseline)."""
    n, nu, dt, steps = 32, 1.0 / 1600.0, 1e-3, 10
    out = {"workload": "taylor_green_32_fp64: 10 steps, nu=1/1600, dt=1e-3"}
    for key, name, ct in TG32_RUNS:
        s = ns.Solver(n, nu, ct, precision="fp64")
        d = s.to_device(inputs.taylor_green(n))
        for rep in range(2):            # the first call builds the tables
            d.copy_(s.to_device(inputs.taylor_green(n)))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "rk4":
                s.step_rk4(d, dt, steps)
            else:
                s.step_ps(d, dt, steps, "exact")
            torch.cuda.synchronize()
            t_gpu = time.perf_counter() - t0
        out[key] = {"gpu_fp64_ms": round(t_gpu * 1e3, 3), "energy_end": float(s.spectra(d)["totals"][0])}
        log(f"tg32 {key}: GPU FP64 {t_gpu * 1e3:.2f} ms")
    return out


def cpu_baseline(inputs, budget_s=20.0):
    """The FP64 oracle on the headline workload, PS-RK2 random on 128^3 from the
    Taylor-Green state: a bounded sample of steps (stops once `budget_s` of host time is
    used)."""
    from oracle import forcing, grid, schemes, transforms
    from oracle import nonlinear as onl
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
    out = {"value": NP ** 3 * nsteps / dt / 1e6, "unit": "Mgridpts*RKsteps/s", "cores": transforms.WORKERS,
           "kind": "oracle",
           "sample": f"{nsteps} steps of PS-RK2 random on the 128^3 Taylor-Green state (FP64 NumPy/SciPy, "
                     f"scipy.fft workers={transforms.WORKERS}), {dt:.1f} s"}
    # config 1: the oracle's wall time for the 10-step Taylor-Green runs on 32^3
    cfg1 = {}
    for key, name, ct in TG32_RUNS:
        model = onl.NSModel(32, NU, grid.mask(32, ct))
        v = inputs.taylor_green(32)
        t0 = time.perf_counter()
        for _ in range(10):
            v = schemes.rk4(model, v, 1e-3) if name == "rk4" else schemes.ps_exact(model, v, 1e-3)
        cfg1[key] = {"oracle_s": round(time.perf_counter() - t0, 4)}
    out["taylor_green_32_fp64_oracle"] = cfg1
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--hit256-steps", type=int, default=500)
    ap.add_argument("--only", default=",".join(WORKLOADS), help="comma list of " + ", ".join(WORKLOADS))
    ap.add_argument("--schemes", default="random,approx,exact,rk4", help="schemes of the tg128 workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first run 3 elementwise copies of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU slab "
              "decomposition is a design, not a build", file=sys.stderr)
        sys.exit(2)
    only = args.only.split(",")
    for w in only:
        if w not in WORKLOADS:
            ap.error(f"unknown workload {w}")

    import torch
    from paper_2603_08892_amd import inputs, ns
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    ns.lib()
    if args.copy_mb:
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    K, W = args.steps, args.warmup
    out = {"metric": METRIC, "value": None, "unit": "Mgridpts*RKsteps/s", "n_gpus": 1, "steps": K, "warmup": W,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "taylor_green_matched_kmax: PS-RK2 on 128^3 C_t=1 vs RK4 on 192^3 C_t=2/3, "
                                  "K2max=4095, nu=1/1600, dt=2e-3, spectra every 10 steps",
                      "scheme": "ps_random", "n": NP, "k2max": 4095}}
    roof128 = None
    if "tg128" in only:
        want = args.schemes.split(",")
        results, speed, roof128 = tg128(torch, ns, inputs, K, W, want)
        head = "random" if "random" in results else want[0]
        out["value"] = round(results[head]["mgridpts_steps_per_s"], 1)
        out["ms_per_step"] = round(results[head]["ms_per_step"], 5)
        out["config"]["scheme"] = f"ps_{head}"
        out["schemes"] = {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                          for k, v in results.items()}
        out["speedup"] = speed
    if "hit256" in only:
        out["hit_256"], out["roofline"] = hit256(torch, ns, inputs, args.hit256_steps, W)
    if roof128 is not None:
        out["roofline_128_cache_resident"] = roof128
        out.setdefault("roofline", roof128)
    if "hit512" in only:
        out["hit_512"] = hit512(torch, ns, inputs, K, W)
    if "adjoint" in only:
        out["adjoint"] = adjoint_run(torch, ns, inputs)
    if "tg32" in only:
        out["taylor_green_32"] = tg32(torch, ns, inputs)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inputs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
