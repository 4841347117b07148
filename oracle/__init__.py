"""FP64 CPU oracle for the stochastic-heating emissivity solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (``paper_1311_4627_amd``); the two meet only in the seeded inputs of the
``synth`` package.

It is a plain, slow, obviously correct implementation of what the method
computes for one (radiation field, grain size) pair, written from
Porter & Vladimirov (arXiv:1311.4627), Sec. 2 (the matrix formalism of
Guhathakurta & Draine and Draine & Li in the "thermal continuous"
approximation):

* enthalpy grid, Debye heat capacity and bin temperatures (Sec. 2.1);
* heating rates from the field by log-log interpolation (Sec. 2.2,
  eq:heating and eq:interpolation), plus the continuous intrabin term of
  Draine & Li (2001) that the paper's text omits (reading R6);
* cooling to the adjacent lower bin (Sec. 2.2, eq:cooling);
* the cumulative matrix B (eq:bmatrix, built by the recurrence of
  eq:brecurrence in the appendix on pruning and recurrence), the recursion
  for X (eq:xf) with power-of-two rescaling (the appendix on precision
  control), and the renormalisation (eq:renormalization);
* the grain emission spectrum (Sec. 2.3, eq:emission and eq:emission-lambda);
* a dense solve of the steady-state master equation (eq:steady-state with
  eq:level-sum) as an independent check at small bin counts;
* energy-balance diagnostics;
* ``oracle.mlp``: the FP64 reference of the learned surrogate (features,
  targets, the MLP's forward and backward passes, Adam, the band-error
  metric), against which the GPU trainer's gradients and the inference
  kernel's outputs are checked.

Every floating-point step is IEEE double precision.  Each reading of a
garbled or ambiguous passage carries a label (R1..R12) and is stated at the
function that uses it.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, special cases, brute force or invariants; none is
"parity unpinned".
"""

from .physics import (  # noqa: F401
    H, C, K, EV, AMU,
    planck_lambda,
    debye_energy,
    temperature_of_energy,
    cross_section,
)
from .model import (  # noqa: F401
    GrainSetup,
    grain_setup,
    heating_matrix,
    b_matrix_recurrence,
    b_matrix_triple_sum,
    recursion,
    emission,
    diagnostics,
    solve_pair,
    equilibrium_temperature,
    size_convolution,
)
from .dense import dense_steady_state  # noqa: F401
