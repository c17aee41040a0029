"""ns_spectra_static (the spectra without a context or any allocation, its scratch in a
static device array) against ns_spectra on the same inputs: bit for bit, two calls in a
row with the second on a smaller grid, with and without the transfer input; and the
host-side rejection of grids beyond its static size."""

import numpy as np
import pytest

from paper_2603_08892_amd import inputs

pytestmark = pytest.mark.gpu


def _pair(n, prec, seed):
    from paper_2603_08892_amd import ns
    s = ns.Solver(n, 0.01, 1.0, precision=prec)
    k2 = ns.retained_bound(n, 1.0)
    u = s.to_device(inputs.hit_initial(n, seed, k2))
    nh = s.nonlinear(u, ps_avg=True)
    return s, u, nh


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_spectra_static_equals_ns_spectra(prec):
    from paper_2603_08892_amd import ns
    for n, seed in ((128, 3), (48, 4)):              # the second call on a smaller grid
        print(f"[no-alloc] spectra_static n={n} {prec}", flush=True)
        s, u, nh = _pair(n, prec, seed)
        for t in (None, nh):
            want = s.spectra(u, t)
            got = ns.spectra_static(u, n, 0.01, t)
            for k in want:
                assert np.array_equal(got[k], want[k]), (n, k)


def test_spectra_static_rejects_large_grids():
    import ctypes
    from paper_2603_08892_amd import ns
    out = ns.NSSpectraOut()
    L = ns.lib()
    big = ns.lib().ns_spectra_static(768, ns.NS_FP32, 0.01, ctypes.c_void_p(256), None, None, ctypes.byref(out))
    assert big == ns.NS_ERR_SIZE and b"512" in L.ns_last_error(None)
    assert L.ns_spectra_static(7, ns.NS_FP32, 0.01, ctypes.c_void_p(256), None, None, ctypes.byref(out)) == ns.NS_ERR_ARG
