"""Error index of a run against a reference run (oracle; test infrastructure only).

Sec. "Performance and accuracy for a decaying flow", Eq. quality and its
discrete form in the appendix (Eq. quality-i-disc): for each direction i, the
time average over the N_t samples between t_start and t_end of the
1/k-weighted mean over the 1D wavenumbers k_n = n of 100 |E_ref - E| / E_ref,
normalised by N_t sum_n 1/k_n; the index is the mean over the three
directions.  The printed sum starts at n = 0, where 1/k_n is undefined; the sum
here starts at n = 1 (k_n = n, spectral step 1).  Written with explicit loops,
for small inputs.
"""


def error_index(e1d, e1d_ref, kmax):
    """e1d, e1d_ref: sequences over time samples of [3][>= kmax + 1] 1D spectra
    (E_x(k_x), E_y(k_y), E_z(k_z)); kmax: largest wavenumber n included."""
    nt = len(e1d)
    if nt == 0 or nt != len(e1d_ref):
        raise ValueError("need the same, non-zero number of samples in both runs")
    norm = nt * sum(1.0 / n for n in range(1, kmax + 1))
    per_dir = []
    for i in range(3):
        acc = 0.0
        for j in range(nt):
            for n in range(1, kmax + 1):
                ref = float(e1d_ref[j][i][n])
                acc += (1.0 / n) * 100.0 * abs(ref - float(e1d[j][i][n])) / ref
        per_dir.append(acc / norm)
    return sum(per_dir) / 3.0, per_dir
