"""The rocprofv3 summariser (paper_2603_08892_amd/profsum.py) on small synthetic
CSV files shaped like rocprofv3's: kernel names to passes, per-pass means, the
counter calibration and the traffic record bench.py reads; and the algorithmic
byte model against a hand count on a small grid."""

import csv
import json
import re

import numpy as np
import pytest

from paper_2603_08892_amd import profsum

PLAN = "ns::LinePlan<256, 32, ns::Radices<8, 8, 4>, ns::Radices<4, 8, 8> >"
NAMES = {
    "x_inverse": f"void ns::f_xinv<{PLAN}, false>(ns::Cx<float> const*, ns::Lay, ns::Cx<float>*)",
    "y_inverse": f"void ns::f_ycurl<{PLAN} >(ns::Cx<float>*, ns::Cx<float> const*, int, ns::Geom)",
    "y_forward": f"void ns::f_ypass<{PLAN}, -1>(ns::Cx<float>*, ns::Cx<float> const*, int, ns::Geom)",
    "z_fused": f"void ns::f_zcross<{PLAN}, 8>(ns::Cx<float>*, ns::Cx<float> const*, ns::Geom)",
    "x_forward_epilogue": f"void ns::f_xfwd<{PLAN}, 3, 0, false>(ns::Cx<float>*, ns::Cx<float> const*, ns::Shift)",
    "x_forward_inverse": f"void ns::f_xfwd<{PLAN}, 2, 2, false>(ns::Cx<float>*, ns::Cx<float> const*, ns::Shift)",
}
# the same passes of a size without the vorticity formed in the y-inverse pass
OTHER = {
    "x_inverse": f"void ns::f_xinv<{PLAN}, true>(ns::Cx<float> const*, ns::Lay, ns::Cx<float>*)",
    "y_inverse": f"void ns::f_ypass<{PLAN}, 1>(ns::Cx<float>*, ns::Cx<float> const*, int, ns::Geom)",
    "x_forward_epilogue": f"void ns::f_xfwd<{PLAN}, 3, 0, true>(ns::Cx<float>*, ns::Cx<float> const*, ns::Shift)",
    "x_forward_inverse": f"void ns::f_xfwd<{PLAN}, 2, 1, true>(ns::Cx<float>*, ns::Cx<float> const*, ns::Shift)",
}


def test_classify_names():
    for want, name in list(NAMES.items()) + list(OTHER.items()):
        assert profsum.classify(name) == (256, want)
    assert profsum.classify("void ns::k_spectra<float>(ns::Cx<float> const*)") == (None, "k_spectra")
    assert profsum.classify("ns::k_budget_step(double const*, int)") == (None, "k_budget_step")
    assert profsum.classify("__amd_rocclr_copyBuffer") == (None, None)


def _write(path, fname, fields, rows):
    path.mkdir(parents=True, exist_ok=True)
    with open(path / fname, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_trace_means(tmp_path):
    rows = []
    for k, (p, us) in enumerate([("z_fused", 10.0), ("z_fused", 20.0), ("x_inverse", 7.0)]):
        rows.append({"Kernel_Name": NAMES[p], "Start_Timestamp": 1000 * k, "End_Timestamp": 1000 * k + int(us * 1e3)})
    _write(tmp_path, "run_kernel_trace.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    t = profsum.trace(str(tmp_path))
    assert t[(256, "z_fused")] == [10.0, 20.0] and t[(256, "x_inverse")] == [7.0]


def test_traffic_record(tmp_path, capsys):
    neg = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(...)>"
    f = tmp_path / "fetch"
    w = tmp_path / "write"
    fields = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    _write(f, "run_counter_collection.csv", fields,
           [{"Kernel_Name": neg, "Counter_Name": "FETCH_SIZE", "Counter_Value": 131072.0},
            {"Kernel_Name": NAMES["z_fused"], "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000.0},
            {"Kernel_Name": NAMES["z_fused"], "Counter_Name": "FETCH_SIZE", "Counter_Value": 3000.0}])
    _write(w, "run_counter_collection.csv", fields,
           [{"Kernel_Name": neg, "Counter_Name": "WRITE_SIZE", "Counter_Value": 262144.0},
            {"Kernel_Name": NAMES["z_fused"], "Counter_Name": "WRITE_SIZE", "Counter_Value": 500.0}])
    profsum.print_traffic(str(f), str(w), "wl", 256)
    out = capsys.readouterr().out
    rec = json.loads(re.search(r"```json\n(.*?)\n```", out, re.S).group(1))
    # the copy of 256 MiB reads as 131072 KiB: fetch scaled by 2, write by 1
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    assert rec["per_launch_bytes"]["wl@256:z_fused"] == (2000 * 2 + 500) * 1024
    assert rec["source_hash"] == profsum.source_hash()


def test_pass_bytes_hand_count():
    """N = 8, K2max = 4 (k^2 <= 4): count the retained modes and active lines by hand."""
    n, k2 = 8, 4
    g = profsum.geometry(n, k2)
    k = [0, 1, 2, 3, -4, -3, -2, -1]
    retained = sum(1 for a in k for b in k for c in range(3) if a * a + b * b + c * c <= k2)
    lines = sum(1 for b in k for c in range(3) if b * b + c * c <= k2)
    assert (g["retained"], g["lines"], g["kzn"]) == (retained, lines, 3)
    pb = profsum.pass_bytes(g)  # 8 is not a size with the curl in the y-inverse pass
    planes = n * n * 3
    assert pb["z_fused"] == 9 * planes * 8
    assert pb["x_forward_inverse"] == (9 * lines * n + 6 * retained) * 8
    assert profsum.pass_bytes(g, 7.5)["x_forward_inverse"] == int((9 * lines * n + 7.5 * retained) * 8)
    assert np.isclose(pb["y_inverse"], (6 * lines * n + 6 * planes) * 8)
    # five fields between the x-inverse and y-inverse passes instead of six
    yc = profsum.pass_bytes(g, yc=True)
    assert pb["x_forward_inverse"] - yc["x_forward_inverse"] == lines * n * 8
    assert pb["x_inverse"] - yc["x_inverse"] == lines * n * 8
    assert pb["y_inverse"] - yc["y_inverse"] == lines * n * 8
    assert yc["z_fused"] == pb["z_fused"] and yc["y_forward"] == pb["y_forward"]


def test_yc_sizes_match_the_kernel_configs():
    """YC_SIZES names exactly the FastCfg configurations of csrc/ns_fast.hpp with YC on."""
    text = open(f"{profsum.CSRC}/ns_fast.hpp").read()
    cfgs = re.findall(r"using Fast(\d+) = FastCfg<([^;]*)>;", text)
    assert len(cfgs) == 13
    on = {int(n) for n, args in cfgs if args.replace(" ", "").endswith(",true")}
    assert on == set(profsum.YC_SIZES)
