"""Plain, slow, FP64 CPU oracle for the dealiased nonlinear term of 3D periodic
incompressible Navier-Stokes and for the Runge-Kutta schemes that call it.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
anything in this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path: every formula here is written out from the paper (arXiv 2603.08892,
"Aliasing and phase shifting in pseudo-spectral simulations of the
incompressible Navier-Stokes equations") in NumPy/SciPy, in float64.

Modules
-------
grid       wavenumbers, truncation thresholds and masks, Hermitian weights, shells
transforms forward (1/N per axis) and inverse (unnormalised) real FFTs
nonlinear  phase shift, curl, projection, u x omega, shift averages, padded product,
           and the transpose of the linearised nonlinear term (for the adjoint)
schemes    integrating-factor Euler, midpoint RK2, Lawson RK4 (optional forcing),
           phase-shifted RK2 (exact / approx / random, optional split forcing) and the
           step adjoint
spectra    shell, 1D, dissipation and transfer spectra; totals; the time-integrated
           energy budget E - E0 + int eps dt - int P dt
forcing    SplitMix64 counter-based draws, forcing amplitudes, injection scaling and
           the energy injected per step
quality    error index of a run's 1D spectra against a reference run
nl1d       the 1D quadratic model dS/dt = -S^2

Parity status: every function is pinned by at least one test in
``tests/test_oracle_pins.py``: the forcing inside the schemes by the closed-form
forced solution of a linear model and by self-convergence orders, the transfer
spectrum by T(u, u) = 2 E(k) and the shell energy balance, the budget by the
exact-decay closed form and its convergence orders.  The forcing draw itself is
parity unpinned against the paper, which gives no forcing formula: its shape is
a reading, and only its injection rate is pinned.
"""

from . import grid, transforms, nonlinear, schemes, spectra, forcing, nl1d  # noqa: F401
