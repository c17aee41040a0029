"""Host-side check of every compile-time line plan of the specialised passes.

Each `LinePlan<N, TPL, Radices<inverse>, Radices<forward>>` in csrc/ns_fast.hpp is
run through a Python model of the register FFT's thread mapping (csrc/fft_reg.hpp):
a stage of radix R has N/R butterflies, thread t takes butterflies t + TPL b and
the ones past N/R are predicated off; butterfly j of a stage after NS points have
been combined twiddles its inputs by W^(k m N/(NS R)) (k = j mod NS), applies an
R-point DFT and writes point m to q NS R + k + m NS (q = j div NS); the next stage
reads its butterfly j's inputs at j + m N/R.  The model checks that the first
stage loads, every exchange and the last stage's outputs touch each of the N
positions exactly once, that every index stays in range, that the plan's register
count is what the kernels allocate, and that the result is the DFT of the input
(numpy), in both directions.  It also checks the chaining conditions the passes
rely on (the forward list is the inverse one reversed, so a transform's outputs
sit at the next one's inputs).
"""

import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2603_08892_amd", "csrc", "ns_fast.hpp")


def _plans():
    text = open(HEADER).read()
    pat = re.compile(r"using (\w+) = LinePlan<(\d+), (\d+), Radices<([\d, ]+)>, Radices<([\d, ]+)>>;")
    out = []
    for name, n, tpl, inv, fwd in pat.findall(text):
        out.append((name, int(n), int(tpl), tuple(int(r) for r in inv.split(",")),
                    tuple(int(r) for r in fwd.split(","))))
    return out


PLANS = _plans()


def _ept(n, tpl, radices):
    return max(-(-(n // r) // tpl) * r for r in radices)


def _run_plan(n, tpl, radices, sign, x):
    """The thread mapping applied to x; returns the transform (unnormalised)."""
    ept = _ept(n, tpl, radices)
    v = np.zeros((tpl, ept), complex)
    tw = np.exp(sign * 2j * np.pi * np.arange(n) / n)
    r0 = radices[0]
    seen = np.zeros(n, int)
    for t in range(tpl):
        for i in range(ept):
            b, m = divmod(i, r0)
            j = t + tpl * b
            if j < n // r0:
                pos = j + m * (n // r0)
                assert 0 <= pos < n
                v[t, i] = x[pos]
                seen[pos] += 1
    assert (seen == 1).all(), "first-stage loads"
    ns = 1
    for s, r in enumerate(radices):
        nb = -(-(n // r) // tpl)
        dft = np.exp(sign * 2j * np.pi * np.outer(np.arange(r), np.arange(r)) / r)
        for t in range(tpl):
            for b in range(nb):
                j = t + tpl * b
                if j >= n // r:
                    continue
                k = j % ns
                a = v[t, b * r:(b + 1) * r].copy()
                if ns > 1:
                    a = a * tw[(k * np.arange(r) * (n // (ns * r))) % n]
                v[t, b * r:(b + 1) * r] = dft @ a
        if s + 1 < len(radices):
            r2 = radices[s + 1]
            lds = np.zeros(n, complex)
            wr = np.zeros(n, int)
            for t in range(tpl):
                for b in range(nb):
                    j = t + tpl * b
                    if j >= n // r:
                        continue
                    k, q = j % ns, j // ns
                    for m in range(r):
                        p = q * ns * r + k + m * ns
                        assert 0 <= p < n
                        lds[p] = v[t, b * r + m]
                        wr[p] += 1
            assert (wr == 1).all(), f"stage {s} exchange writes"
            v[:] = 0
            rd = np.zeros(n, int)
            for t in range(tpl):
                for b in range(-(-(n // r2) // tpl)):
                    j = t + tpl * b
                    if j >= n // r2:
                        continue
                    for m in range(r2):
                        p = j + m * (n // r2)
                        v[t, b * r2 + m] = lds[p]
                        rd[p] += 1
            assert (rd == 1).all(), f"stage {s} exchange reads"
        ns *= r
    rl = radices[-1]
    out = np.zeros(n, complex)
    got = np.zeros(n, int)
    for t in range(tpl):
        for i in range(ept):
            b, m = divmod(i, rl)
            j = t + tpl * b
            if j < n // rl:
                p = j + m * (n // rl)
                out[p] = v[t, i]
                got[p] += 1
    assert (got == 1).all(), "last-stage outputs"
    return out


def test_header_has_plans():
    sizes = {n for _, n, _, _, _ in PLANS}
    assert {64, 128, 144, 160, 192, 216, 240, 256, 270, 324, 360, 384, 512} <= sizes


@pytest.mark.parametrize("name,n,tpl,inv,fwd", PLANS, ids=[p[0] for p in PLANS])
def test_line_plan(name, n, tpl, inv, fwd):
    assert np.prod(inv) == n and np.prod(fwd) == n
    assert fwd == tuple(reversed(inv)), "the forward radices are the inverse ones reversed"
    assert _ept(n, tpl, inv) == _ept(n, tpl, fwd) <= 16
    rng = np.random.default_rng(n * 1000 + tpl)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    inv_out = _run_plan(n, tpl, inv, +1, x)
    assert np.abs(inv_out - np.fft.ifft(x) * n).max() <= 1e-12 * np.abs(x).sum()
    fwd_out = _run_plan(n, tpl, fwd, -1, x)
    assert np.abs(fwd_out - np.fft.fft(x)).max() <= 1e-12 * np.abs(x).sum()
