// ns_aux_types.hpp -- FP64 records the auxiliary kernels keep in the workspace.
#pragma once

namespace ns {

// FP64 record of the last forcing draw (ForceState, in the workspace): the
// projected shape g of the 48 independent modes, the amplitude a, B = <u0, g>,
// G = <g, g>, r = sqrt(B^2 + 2 dt G inj) and the energy the step injects,
// dt (a B + a^2 dt/2 G) (= E(u0 + dt O) - E(u0)); `dot` is scratch of the forced
// step adjoint.
struct ForceState {
  double g[48][3][2];
  double amp, B, G, r, injected, dot;
};

// Budget record (FP64, in the workspace), updated after every step while the
// budget is on: t, E, eps, E0, int eps dt (trapezoid rule step by step),
// int P dt (the energy each forced step injects), P of the last step, and the
// residual E - E0 + int eps dt - int P dt.
struct Budget {
  double t, E, eps, E0, int_eps, int_p, p_last, residual;
};

}  // namespace ns
