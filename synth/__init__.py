"""Seeded synthetic inputs for the stochastic-heating emissivity solve.

This package is the only code shared by the FP64 oracle (``oracle/``) and the
HIP path (``paper_1311_4627_amd``).  It builds *inputs* only: wavelength grids,
grain descriptions (size, density, atom mass, Debye temperature, enthalpy-grid
end points, bin count, absorption cross-section table) and radiation fields
(sums of diluted blackbodies, optionally attenuated).  It holds none of the
method's arithmetic: no heating or cooling rates, no heat-capacity inversion,
no recursion, no emission.

The paper (Porter & Vladimirov, Sec. 2 and Sec. 3.2) runs on Draine's optical
tables, WD01 size distributions and the Mathis et al. ISRF; none of those are
available here, so the workloads below stand in for them with analytic
absorption efficiencies and diluted-blackbody fields whose total energy density
matches the ISRF normalisation the paper quotes (0.46 eV cm^-3, Sec. 2.3.1).
"""

from .configs import (  # noqa: F401
    CONSTANTS,
    Grain,
    Workload,
    wavelength_grid_cm,
    make_grain,
    bins_for_radius,
    workload,
    WORKLOAD_NAMES,
    radii_cm,
    size_weights,
)
from .fields import make_fields, FieldRecipe  # noqa: F401
