"""Per-pass summaries of rocprofv3 output for the library's kernels.

    python -m paper_2603_08892_amd.profsum trace DIR [--k2max K] [--rk4 N,...]
        kernel trace (rocprofv3 --kernel-trace --output-format csv -d DIR -o run):
        launches and mean duration per grid size and pass; with --k2max also the
        algorithmic bytes of each pass (sphere k^2 <= K; the x-forward stage operands
        of RK4 for the sizes after --rk4, of PS-RK2 for the others), GB/s and the
        fraction of the 8 TB/s HBM peak
    python -m paper_2603_08892_amd.profsum traffic FETCH_DIR WRITE_DIR WORKLOAD
        two counter runs (rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE, of a
        bench run with --copy-mb MiB): KiB per dispatch per pass, scaled by what the
        same counters read for the calibration copy (torch.neg over MiB in and out),
        and the JSON block that bench.py reads its roofline traffic from
    python -m paper_2603_08892_amd.profsum sq DIR
        one counter run of the SQ counters SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS
        SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_WAVE_CYCLES SQ_ACTIVE_INST_VALU
        SQ_LDS_BANK_CONFLICT: per pass, instructions per wave, the share of the
        waves' lifetime spent issuing VALU instructions and the LDS bank-conflict
        cycles per LDS instruction

Passes are named as in bench.py: x_inverse, y_inverse, z_fused, y_forward,
x_forward_epilogue (an x-forward pass on its own) and x_forward_inverse (an
x-forward pass that also runs the next evaluation's x-inverse pass); the adjoint
kernels as lam_x, z_adjoint, x_adjoint; everything else by kernel name.
"""

import argparse
import collections
import csv
import hashlib
import json
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")


ELEM = 8           # bytes of one FP32 complex
HBM_PEAK_GBS = 8000.0
# Grid sizes whose step sequences form the vorticity in the y-inverse pass
# (FastCfg YC in csrc/ns_fast.hpp): their x-inverse passes write five fields, not six.
YC_SIZES = frozenset({128, 144, 256, 270})


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


def pass_bytes(g, operands=6.0, yc=None):
    """Algorithmic HBM bytes per launch of each pass of a chained step (operands: stage
    operands read and outputs stored per x-forward stage, in retained-mode fields:
    6 for the PS-RK2 Heun stages (one operand read, one output stored, three
    components each), 7.5 on average over the four Lawson RK4 stages, which read one,
    two, two and one operand and store one output each).  F = 5 fields on the active
    lines between the x-inverse and y-inverse passes where the y-inverse pass forms
    the vorticity (yc; by default for the sizes in YC_SIZES), else 6.

    x_inverse          reads the 3 retained components, writes F fields on the active lines
                       (only the first evaluation of a call runs it on its own)
    y_inverse          reads the F fields on the active lines, writes the 6 full (x, y) planes k_z < kzn
    z_fused            reads 6 and writes 3 fields on those planes
    y_forward          reads 3 fields on the planes, writes them on the active lines
    x_forward_epilogue the last stage of a call: reads 3 fields on the active lines and the
                       partial update (retained modes), writes the state's whole half spectrum
    x_forward_inverse  every other stage: reads 3 fields on the active lines and one stage
                       operand, writes one stage output (retained modes; S1 only feeds the
                       next evaluation and is not stored), then the next evaluation's F
                       fields on the active lines
    """
    n, A, R, kzn, h = g["n"], g["lines"], g["retained"], g["kzn"], g["h"]
    planes = n * n * kzn
    f = 5 if (n in YC_SIZES if yc is None else yc) else 6
    return {
        "x_inverse": (3 * R + f * A * n) * ELEM,
        "y_inverse": (f * A * n + 6 * planes) * ELEM,
        "z_fused": (6 * planes + 3 * planes) * ELEM,
        "y_forward": (3 * planes + 3 * A * n) * ELEM,
        "x_forward_epilogue": (3 * A * n + 3 * R + 3 * n * n * h) * ELEM,
        "x_forward_inverse": int(((3 + f) * A * n + operands * R) * ELEM),
    }


def source_hash():
    """Hash of every kernel source file (names and contents)."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def classify(name):
    """(grid size or None, pass name) of a kernel name as rocprofv3 prints it."""
    m = re.match(r"(?:void )?ns::(\w+)<ns::LinePlan<(\d+),", name)
    if m:
        kern, n = m.group(1), int(m.group(2))
        if kern == "f_xinv":
            return n, "x_inverse"
        if kern == "f_ycurl":
            return n, "y_inverse"
        if kern == "f_ypass":
            return n, "y_inverse" if re.search(r"> >, 1>\(", name) else "y_forward"
        if kern == "f_zcross":
            return n, "z_fused"
        if kern == "f_xfwd":
            feed = re.search(r"> >, -?\d+, (\d+)(?:, (?:true|false))?>\(", name)
            return n, "x_forward_inverse" if feed and feed.group(1) != "0" else "x_forward_epilogue"
        return n, {"f_xlam": "lam_x", "f_zadj": "z_adjoint", "f_xadj": "x_adjoint"}.get(kern, kern)
    m = re.match(r"(?:void )?ns::(k_\w+)<", name) or re.match(r"(?:void )?ns::(k_\w+)\(", name)
    if m:
        kern = m.group(1)
        generic = {"k_xinv": "x_inverse", "k_zcross": "z_fused", "k_xlam": "lam_x", "k_zadj": "z_adjoint",
                   "k_xadj": "x_adjoint"}
        if kern == "k_ypass":
            return None, "y_inverse (generic)" if ", 1>(" in name else "y_forward (generic)"
        if kern in generic:
            return None, generic[kern] + " (generic)"
        if kern == "k_xfwd":
            return None, "x_forward (generic)"
        return None, kern
    return None, None


def _rows(path, fname):
    with open(os.path.join(path, fname)) as fh:
        return list(csv.DictReader(fh))


def trace(path):
    """{(n, pass): [durations in us]} from a kernel-trace directory."""
    out = collections.defaultdict(list)
    for r in _rows(path, "run_kernel_trace.csv"):
        n, p = classify(r["Kernel_Name"])
        if p is None:
            continue
        out[(n, p)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    return out


def counters(path, counter):
    """({(n, pass): [KiB per dispatch]}, calibration KiB of the torch.neg copy or None)."""
    out = collections.defaultdict(list)
    calib = None
    for r in _rows(path, "run_counter_collection.csv"):
        if r["Counter_Name"] != counter:
            continue
        name, v = r["Kernel_Name"], float(r["Counter_Value"])
        if "neg_kernel" in name:
            calib = v if calib is None else max(calib, v)
            continue
        n, p = classify(name)
        if p is not None:
            out[(n, p)].append(v)
    return out, calib


ORDER = ["x_inverse", "y_inverse", "z_fused", "y_forward", "x_forward_epilogue", "x_forward_inverse",
         "lam_x", "z_adjoint", "x_adjoint"]


def _key(k):
    n, p = k
    return (n or 0, ORDER.index(p) if p in ORDER else len(ORDER), p)


def print_trace(path, k2max=None, rk4=()):
    t = trace(path)
    if k2max is None:
        print("| N | pass | launches | mean us | total ms |")
        print("|---|---|---|---|---|")
    else:
        print("| N | pass | launches | mean us | total ms | algorithmic MB | GB/s | of 8 TB/s |")
        print("|---|---|---|---|---|---|---|---|")
    pb = {}
    for k in sorted(t, key=_key):
        d = t[k]
        mean = sum(d) / len(d)
        line = f"| {k[0] or '-'} | {k[1]} | {len(d)} | {mean:.2f} | {sum(d) * 1e-3:.3f} |"
        if k2max is not None:
            n = k[0]
            if n is not None and n not in pb:
                pb[n] = pass_bytes(geometry(n, k2max), 7.5 if n in rk4 else 6.0)
            b = pb.get(n, {}).get(k[1])
            line += (f" {b / 1e6:.1f} | {b / (mean * 1e-6) / 1e9:.0f} | {b / (mean * 1e-6) / 1e9 / HBM_PEAK_GBS:.3f} |"
                     if b else " | | |")
        print(line)


SQ = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_WAVE_CYCLES",
      "SQ_ACTIVE_INST_VALU", "SQ_LDS_BANK_CONFLICT")


def print_sq(path):
    vals = {c: counters(path, c)[0] for c in SQ}
    print("| N | pass | dispatches | waves | VALU / wave | LDS / wave | VMEM rd / wr per wave | VALU-active share "
          "of wave cycles | bank-conflict cycles / LDS instr |")
    print("|---|---|---|---|---|---|---|---|---|")
    for k in sorted(vals["SQ_WAVES"], key=_key):
        if k[0] is None:
            continue
        m = {c: sum(vals[c][k]) / len(vals[c][k]) for c in SQ if vals[c].get(k)}
        w = m.get("SQ_WAVES", 0.0)
        if w <= 0 or len(m) < len(SQ):
            continue
        print(f"| {k[0]} | {k[1]} | {len(vals['SQ_WAVES'][k])} | {w:.0f} | {m['SQ_INSTS_VALU'] / w:.0f} | "
              f"{m['SQ_INSTS_LDS'] / w:.0f} | {m['SQ_INSTS_VMEM_RD'] / w:.0f} / {m['SQ_INSTS_VMEM_WR'] / w:.0f} | "
              f"{m['SQ_ACTIVE_INST_VALU'] / m['SQ_WAVE_CYCLES']:.2f} | "
              f"{m['SQ_LDS_BANK_CONFLICT'] / max(m['SQ_INSTS_LDS'], 1.0):.2f} |")


def print_traffic(fetch_dir, write_dir, workload, copy_mib=256):
    f, fc = counters(fetch_dir, "FETCH_SIZE")
    w, wc = counters(write_dir, "WRITE_SIZE")
    if fc is None or wc is None:
        raise SystemExit("no calibration copy (torch.neg) in the counter runs: run the bench with --copy-mb")
    ff, wf = copy_mib * 1024 / fc, copy_mib * 1024 / wc
    print(f"calibration: torch.neg over {copy_mib} MiB reads FETCH_SIZE {fc:.0f} KiB, WRITE_SIZE {wc:.0f} KiB "
          f"-> factors {ff:.4f} (fetch), {wf:.4f} (write)")
    print("| N | pass | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB (scaled) | write MB | traffic MB |")
    print("|---|---|---|---|---|---|---|---|")
    per = {}
    for k in sorted(set(f) & set(w), key=_key):
        fk, wk = sum(f[k]) / len(f[k]), sum(w[k]) / len(w[k])
        rd, wr = fk * 1024 * ff, wk * 1024 * wf
        print(f"| {k[0] or '-'} | {k[1]} | {len(f[k])} | {fk:.0f} | {wk:.0f} | {rd / 1e6:.1f} | {wr / 1e6:.1f} | "
              f"{(rd + wr) / 1e6:.1f} |")
        if k[0] is not None:
            per[f"{workload}@{k[0]}:{k[1]}"] = int(round(rd + wr))
    print("```json")
    print(json.dumps({"source_hash": source_hash(), "fetch_factor": round(ff, 4), "write_factor": round(wf, 4),
                      "per_launch_bytes": per}, indent=1))
    print("```")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("trace")
    a.add_argument("dir")
    a.add_argument("--k2max", type=int)
    a.add_argument("--rk4", default="", help="comma list of grid sizes that ran RK4")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("workload")
    b.add_argument("--copy-mib", type=int, default=256)
    c = sub.add_parser("sq")
    c.add_argument("dir")
    args = ap.parse_args(argv)
    if args.cmd == "trace":
        print_trace(args.dir, args.k2max, tuple(int(x) for x in args.rk4.split(",") if x))
    elif args.cmd == "sq":
        print_sq(args.dir)
    else:
        print_traffic(args.fetch_dir, args.write_dir, args.workload, args.copy_mib)


if __name__ == "__main__":
    main()
