"""Lat-lon grid with a seeded land mask and bathymetry.

Row ordering follows the biogeochemical interface's column assumption
(section 5.1): all points of one water column are contiguous, surface first.
Columns are ordered by latitude row, then longitude (longitude fastest).
"""

from dataclasses import dataclass

import numpy as np

EARTH_RADIUS = 6.371e6  # m


@dataclass
class Grid:
    nlon: int
    nlat: int
    nlayer: int
    lat_c: np.ndarray       # [nlat] cell-centre latitudes (degrees)
    lon_c: np.ndarray       # [nlon] cell-centre longitudes (degrees)
    depth: np.ndarray       # [nlat, nlon] number of wet layers (0 = land)
    dz: np.ndarray          # [nlayer] layer heights h_k (m)
    col_j: np.ndarray       # [ncol] latitude row of each wet column
    col_i: np.ndarray       # [ncol] longitude index of each wet column
    col_start: np.ndarray   # [ncol+1] first row of each column (int32)
    lat: np.ndarray         # [ncol] latitude of each column (degrees)
    area: np.ndarray        # [ncol] horizontal cell area (m^2)

    @property
    def ncol(self) -> int:
        return int(self.col_j.size)

    @property
    def n(self) -> int:
        return int(self.col_start[-1])

    def column_depths(self) -> np.ndarray:
        return np.diff(self.col_start)

    def volumes(self) -> np.ndarray:
        """Cell volume V_i = area_c * h_k for every row (m^3)."""
        nc = self.column_depths()
        k = np.concatenate([np.arange(m) for m in nc])
        return np.repeat(self.area, nc) * self.dz[k]

    def row_layer(self) -> np.ndarray:
        nc = self.column_depths()
        return np.concatenate([np.arange(m) for m in nc]).astype(np.int32)

    def row_column(self) -> np.ndarray:
        return np.repeat(np.arange(self.ncol, dtype=np.int32), self.column_depths())

    def index_map(self) -> np.ndarray:
        """[nlayer, nlat, nlon] row index of each wet cell, -1 on land."""
        idx = np.full((self.nlayer, self.nlat, self.nlon), -1, dtype=np.int64)
        for c in range(self.ncol):
            j, i = self.col_j[c], self.col_i[c]
            s, e = self.col_start[c], self.col_start[c + 1]
            idx[: e - s, j, i] = np.arange(s, e)
        return idx


def layer_heights(nlayer: int, top: float = 50.0, bottom: float = 700.0) -> np.ndarray:
    """Layer heights growing linearly from ``top`` to ``bottom`` metres."""
    if nlayer == 1:
        return np.array([top])
    return top + (bottom - top) * np.arange(nlayer) / (nlayer - 1)


def _smooth_field(nlat: int, nlon: int, rng: np.random.Generator, nmodes: int = 24) -> np.ndarray:
    """Smooth periodic-in-longitude random field used to place land and sea."""
    lat = (np.arange(nlat) + 0.5) / nlat * np.pi          # 0..pi
    lon = (np.arange(nlon) + 0.5) / nlon * 2.0 * np.pi    # 0..2pi
    f = np.zeros((nlat, nlon))
    for _ in range(nmodes):
        kx = rng.integers(1, 5)
        ky = rng.integers(1, 4)
        a = rng.normal() / np.sqrt(kx * kx + ky * ky)
        px, py = rng.uniform(0, 2 * np.pi, 2)
        f += a * np.cos(kx * lon[None, :] + px) * np.cos(ky * lat[:, None] + py)
    return f


def _assign_depths(score: np.ndarray, ncol: int, n: int, nlayer: int) -> np.ndarray:
    """Depths (1..nlayer) for ``ncol`` columns ordered by ``score`` summing to ``n``."""
    if not (ncol <= n <= ncol * nlayer):
        raise ValueError("n must lie in [ncol, ncol*nlayer]")
    order = np.argsort(-score, kind="stable")            # deepest first
    s = 1.0 - (np.arange(ncol) + 0.5) / ncol              # 1 .. 0 rank fraction

    def depths(gamma):
        return np.clip(np.ceil(nlayer * s ** gamma), 1, nlayer).astype(np.int64)

    lo, hi = 1e-3, 1e3                                    # total decreases with gamma
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        if depths(mid).sum() > n:
            lo = mid
        else:
            hi = mid
    d = depths(hi)
    diff = n - int(d.sum())
    # greedy exact adjustment: deepen the deepest-ranked columns, or shallow the shallowest
    while diff != 0:
        changed = False
        seq = range(ncol) if diff > 0 else range(ncol - 1, -1, -1)
        for r in seq:
            if diff > 0 and d[r] < nlayer:
                d[r] += 1
                diff -= 1
                changed = True
            elif diff < 0 and d[r] > 1:
                d[r] -= 1
                diff += 1
                changed = True
            if diff == 0:
                break
        if not changed:
            raise RuntimeError("cannot reach the requested number of points")
    out = np.empty(ncol, dtype=np.int64)
    out[order] = d
    return out


def make_grid(nlon: int, nlat: int, nlayer: int, ncol: int, n: int, seed: int) -> Grid:
    """Seeded grid with exactly ``ncol`` wet columns and ``n`` wet points."""
    rng = np.random.default_rng(seed)
    field = _smooth_field(nlat, nlon, rng)
    flat = field.ravel()
    wet_cells = np.argsort(-flat, kind="stable")[:ncol]
    wet_cells.sort()                                      # lat-row major, lon fastest
    score = flat[wet_cells]
    d = _assign_depths(score, ncol, n, nlayer)
    depth = np.zeros(nlat * nlon, dtype=np.int64)
    depth[wet_cells] = d
    depth = depth.reshape(nlat, nlon)

    col_j = (wet_cells // nlon).astype(np.int32)
    col_i = (wet_cells % nlon).astype(np.int32)
    col_start = np.zeros(ncol + 1, dtype=np.int32)
    col_start[1:] = np.cumsum(d)

    dlat = 180.0 / nlat
    lat_c = -90.0 + (np.arange(nlat) + 0.5) * dlat
    lon_c = (np.arange(nlon) + 0.5) * 360.0 / nlon
    lat_s = np.radians(-90.0 + np.arange(nlat) * dlat)
    lat_n = np.radians(-90.0 + (np.arange(nlat) + 1) * dlat)
    row_area = EARTH_RADIUS ** 2 * (2.0 * np.pi / nlon) * (np.sin(lat_n) - np.sin(lat_s))

    return Grid(
        nlon=nlon, nlat=nlat, nlayer=nlayer,
        lat_c=lat_c, lon_c=lon_c, depth=depth, dz=layer_heights(nlayer),
        col_j=col_j, col_i=col_i, col_start=col_start,
        lat=lat_c[col_j].astype(np.float64), area=row_area[col_j].astype(np.float64),
    )
