"""FP64 CPU oracle of the flux-reconstruction residual, RK4 update and probe statistics.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
executes this package; only ``tests/``, the smoke check and the bench's CPU
baseline leg use it.  It shares no code with the HIP path: it builds its own
operators, metrics and connectivity from the mesh description, in plain
PyTorch float64 CPU ops (so that reverse-mode autograd of it gives the oracle
gradient) with numpy / scipy only for the integer face matching.

What it computes and where the paper fixes it:
* conservation law, inviscid and viscous fluxes, ideal gas, stress tensor and
  heat flux: Eqs. (1)-(7) of the governing-equations subsection;
* FR spatial discretisation (Huynh's scheme, cited in the flow-solver
  subsection; the paper defers details to earlier work), read as: Gauss-Legendre
  solution and flux points, the g_DG correction function, Rusanov inviscid and
  LDG viscous common fluxes, adiabatic no-slip walls, Riemann-invariant far field;
* drag coefficient Eq. (8); OASPL, RMS and cumulative mean, Eqs. (9)-(12); the spanwise
  observer average and the Welch spectra of the case sections (``spectra.py``);
* a solution degree per element (the airfoil case's P0-P4 sponge, ``vardeg.py``), with
  mixed-degree faces read as mortars on the higher side's flux points;
* classical RK4 time stepping with a given dt (the paper's own integrator is a
  second-order optimal scheme whose coefficients it does not print).

Parity status per function is listed in ``oracle/PINS.md``.
"""
from .basis import (  # noqa: F401
    gauss_legendre, lagrange_eval, lagrange_deriv, correction_deriv, gll_nodes, TensorOps,
)
from .fr import OracleSystem, airfoil_objective, cumulative_prms, force_coefficients, oaspl_from_series  # noqa: F401
from .spectra import observer_oaspl, welch_psd  # noqa: F401
from .vardeg import VarDegreeOracle  # noqa: F401
