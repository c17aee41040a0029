"""The accuracy-against-cost pipeline on the GPU, on a short window of the
Taylor-Green run: the reference has zero error against itself, every run has
one sample per requested time and a finite index.  (Early in the run the far
tail of the 1D spectra is below the FP32 round-off of the fields, so the index
of this window is not an accuracy figure; the documented comparison uses the
transition window t in [7, 12].)"""

import numpy as np
import pytest

from paper_2603_08892_amd import quality

pytestmark = pytest.mark.gpu


def test_quality_pipeline_short_window():
    rows = quality.compare(2.0, 2.2, 0.1, runs=["ps_random_128", "rk4_128_aliased"])
    assert rows[quality.REFERENCE]["error_pct"] == 0.0
    for name, r in rows.items():
        assert np.isfinite(r["error_pct"]) and r["wall_s"] > 0, name
    times, spec, _ = quality.run_taylor_green("random", 128, 1.0, 0.1, 0.3, 0.1)
    assert np.allclose(times, [0.1, 0.2, 0.3]) and spec.shape == (3, 3, quality.KMAX + 1)
