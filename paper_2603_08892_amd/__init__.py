"""MI355X-native dealiased nonlinear term and phase-shift Runge-Kutta schemes for
3D periodic incompressible Navier-Stokes (arXiv 2603.08892).

The compute path is a C-ABI shared library of hand-written HIP kernels for gfx950
(``libns.so``, declared in ``include/ns.h``); ``paper_2603_08892_amd.ns`` is the
thin Python binding over it.  ``inputs`` holds seeded synthetic workloads.
"""
