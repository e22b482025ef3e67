"""Named synthetic workloads.

* ``tiny``         16x8x4 grid, 90 wet columns, 300 points, one-tracer N model,
                   one euphotic layer.
* ``global_2p8``   128x64x15 grid (2.8125 degrees, as in section 7 of the paper),
                   exactly 4448 wet columns and 52749 points, N-DOP model, two
                   euphotic layers.
* ``ensemble_1p4`` 256x128x23 grid (1.40625 degrees), 22000 wet columns and
                   500000 points, N-DOP model, two euphotic layers.

All use twelve monthly matrices of each kind and 2880 steps per model year.
"""

from dataclasses import dataclass

import numpy as np

from .grid import Grid, make_grid
from .params import MODEL_N, MODEL_NDOP, MODEL_NDOPPHY, NTRACER, NPARAM
from .transport import Transport, make_transport


@dataclass
class Inputs:
    name: str
    grid: Grid
    tm: Transport
    model: int
    neuphotic: int
    y_init: tuple          # constant initial value per tracer
    nbgc: int = 1          # internal BGC steps per ocean step (section 7)

    @property
    def n(self):
        return self.grid.n

    @property
    def ntracer(self):
        return NTRACER[self.model]

    @property
    def nparam(self):
        return NPARAM[self.model]

    @property
    def nstep(self):
        return self.tm.nstep

    @property
    def nmat(self):
        return self.tm.nmat

    def initial_state(self, nbatch: int = 1) -> np.ndarray:
        """Row-major ``n x (nbatch*ntracer)`` constant initial field."""
        row = np.tile(np.asarray(self.y_init, dtype=np.float64), nbatch)
        return np.broadcast_to(row, (self.n, row.size)).copy()

    def desc_arrays(self) -> dict:
        """Flat arrays in the order of the transport-matrix descriptor."""
        g, t = self.grid, self.tm
        return dict(
            n=g.n, ncol=g.ncol, nlayer=g.nlayer,
            col_start=np.ascontiguousarray(g.col_start, dtype=np.int32),
            lat=np.ascontiguousarray(g.lat, dtype=np.float64),
            lon=np.ascontiguousarray(g.lon_c[g.col_i], dtype=np.float64),
            area=np.ascontiguousarray(g.area, dtype=np.float64),
            dz=np.ascontiguousarray(g.dz, dtype=np.float64),
            nmat=t.nmat, nstep=t.nstep, model=self.model, neuphotic=self.neuphotic, nbgc=self.nbgc,
            ae_rowptr=t.ae_rowptr, ae_colidx=t.ae_colidx, ae_val=np.ascontiguousarray(t.ae_val),
            ai_rowptr=t.ai_rowptr, ai_colidx=t.ai_colidx, ai_val=np.ascontiguousarray(t.ai_val),
        )


def _build(name, nlon, nlat, nlayer, ncol, n, model, neu, y_init, seed, nmat=12, nstep=2880):
    grid = make_grid(nlon, nlat, nlayer, ncol, n, seed)
    tm = make_transport(grid, seed + 1, nmat=nmat, nstep=nstep)
    return Inputs(name=name, grid=grid, tm=tm, model=model, neuphotic=neu, y_init=y_init)


# constant initial field per tracer: PO4, DOP, PHY (mmol P / m^3)
Y_INIT = {MODEL_N: (2.17,), MODEL_NDOP: (2.17, 1e-4), MODEL_NDOPPHY: (2.17, 1e-4, 1e-2)}


def tiny(seed: int = 7, model: int = MODEL_N, nstep: int = 2880) -> Inputs:
    neu = 1 if model == MODEL_N else 2
    return _build("tiny_16x8x4", 16, 8, 4, 90, 300, model, neu, Y_INIT[model], seed, nstep=nstep)


def global_2p8(seed: int = 11, nstep: int = 2880, model: int = MODEL_NDOP) -> Inputs:
    return _build("global_128x64x15", 128, 64, 15, 4448, 52749, model, 2, Y_INIT[model], seed, nstep=nstep)


def ensemble_1p4(seed: int = 13, nstep: int = 2880) -> Inputs:
    return _build("ensemble_256x128x23", 256, 128, 23, 22000, 500000, MODEL_NDOP, 2, (2.17, 1e-4), seed,
                  nstep=nstep)


def one_degree(seed: int = 17, nstep: int = 2880, model: int = MODEL_NDOP) -> Inputs:
    """A 1.0-degree stand-in (360x180x23, 42000 wet columns, 760000 points), N-DOP by default.

    The paper runs its speedup tests at 2.8125 and 1.0 degrees (section 8) but gives
    no sizes for the latter; these are this implementation's choice (about 65 % ocean,
    18 wet layers per column on average)."""
    return _build("one_degree_360x180x23", 360, 180, 23, 42000, 760000, model, 2, Y_INIT[model], seed,
                  nstep=nstep)


def small_ndop(seed: int = 5, nstep: int = 2880, model: int = MODEL_NDOP) -> Inputs:
    """A 32x16x8 grid (about 2.7k points, N-DOP by default): several tiles and a ragged tail."""
    return _build("small_32x16x8", 32, 16, 8, 400, 2700, model, 2, Y_INIT[model], seed, nstep=nstep)


def custom(nlon: int, nlat: int, nlayer: int, ncol: int, n: int, model: int = MODEL_NDOP, neuphotic: int = 2,
           seed: int = 3, nmat: int = 12, nstep: int = 2880, nbgc: int = 1) -> Inputs:
    """Any grid shape built like the named workloads (for edge cases: single points, shallow or
    deep columns, short years, one matrix)."""
    inp = _build(f"custom_{nlon}x{nlat}x{nlayer}", nlon, nlat, nlayer, ncol, n, model, neuphotic, Y_INIT[model],
                 seed, nmat=nmat, nstep=nstep)
    inp.nbgc = nbgc
    return inp


def by_name(name: str) -> Inputs:
    """The named workloads, plus the global grid's PO4-DOP-PHY model ("global_phy") and its
    8 internal BGC steps per ocean step ("global_nbgc8")."""
    if name == "global_phy":
        return global_2p8(model=MODEL_NDOPPHY)
    if name == "global_nbgc8":
        inp = global_2p8()
        inp.nbgc = 8
        return inp
    table = {"tiny": tiny, "global": global_2p8, "ensemble": ensemble_1p4, "small": small_ndop,
             "one_degree": one_degree}
    return table[name]()
