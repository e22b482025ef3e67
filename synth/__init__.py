"""Seeded synthetic inputs for the transport-matrix time step.

The paper's experiments use twelve explicit and twelve implicit monthly
transport matrices derived from an ocean circulation model on a 2.8125 degree
grid with 15 layers (52749 points per tracer; section 7).  Those matrices are
not available here, so this package draws inputs with the same shapes and
structure:

* ``grid``      -- lat-lon grid, seeded land mask and bathymetry, row ordering.
* ``transport`` -- monthly explicit (horizontal) and implicit (vertical)
                   matrices in CSR form.
* ``params``    -- biogeochemical parameter vectors, bounds, Latin-hypercube
                   ensembles, spin-up lengths and observation noise.
* ``workloads`` -- the named workloads (tiny 16x8x4, global 128x64x15,
                   ensemble 256x128x23, one degree 360x180x23).

Nothing here evaluates the time step, the biogeochemical model or any
derivative of them: both the reference implementation and the GPU library
take these arrays as plain inputs.
"""

from .grid import Grid, make_grid  # noqa: F401
from .transport import Transport, make_transport  # noqa: F401
from .params import (  # noqa: F401
    MODEL_N, MODEL_NDOP, MODEL_NDOPPHY, NTRACER, NPARAM, PARAM_NAMES,
    nominal, bounds, latin_hypercube, spinup_lengths, hidden_params, obs_noise,
)
from .workloads import Inputs, tiny, small_ndop, global_2p8, ensemble_1p4, one_degree, custom, by_name  # noqa: F401
