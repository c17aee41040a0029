"""The package's spectral error index against the oracle's (CPU)."""

import numpy as np
import pytest

from oracle import quality as oquality
from paper_2603_08892_amd import quality


@pytest.mark.parametrize("nt,h,kmax", [(1, 10, 9), (5, 33, 31), (12, 65, 63)])
def test_error_index_matches_oracle(nt, h, kmax):
    rng = np.random.default_rng(nt * h)
    ref = rng.random((nt, 3, h)) + 0.05
    run = ref * (1 + 0.2 * rng.standard_normal((nt, 3, h)))
    got, dirs = quality.error_index(run, ref, kmax)
    want, wdirs = oquality.error_index(list(run), list(ref), kmax)
    assert abs(got - want) <= 1e-12 * want
    assert np.allclose(dirs, wdirs, rtol=1e-12)


def test_error_index_rejects_mismatched_runs():
    with pytest.raises(ValueError):
        quality.error_index(np.ones((2, 3, 8)), np.ones((3, 3, 8)), 7)


def test_kmax108_runs_retain_the_same_modes():
    """Every run of the k_max = 108 comparison keeps exactly k^2 <= 11663."""
    from paper_2603_08892_amd import ns, quality
    for name, (_, n, ct, _, mask) in quality.RUNS108.items():
        assert ns.retained_bound(n, ct, mask) == 11663, name
    assert quality.KMAX108 ** 2 <= 11663 < (quality.KMAX108 + 1) ** 2
