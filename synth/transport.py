"""Monthly explicit and implicit transport matrices (synthetic stand-ins).

Section 3 of the paper: the discretised transport is linear and extremely
sparse; operator splitting gives an explicit matrix for the horizontal
directions and an implicit one for the vertical; twelve monthly matrices of
each kind are stored and interpolated linearly in time.

The paper's matrices come from an ocean model and are not available, so this
module draws matrices with the same structure:

* ``Ae_m = I + s*L_h``: a 5-point horizontal operator per layer combining a
  symmetric diffusion (conductance ``U(0,1)*min(V_a,V_b)`` per wet face) and
  first-order upwind advection by a divergence-free flow given by a stream
  function on cell corners (zero on every corner that touches land).  Rows sum
  to one and ``V^T Ae = V^T`` (mass conservation).  ``s`` is chosen so that
  the smallest diagonal entry is exactly 0.5, which keeps ``Ae`` non-negative.
* ``Ai_m = (I - dt_s*K_v)^{-1}`` per water column, with ``K_v`` a tridiagonal
  vertical diffusion (``kappa ~ U(1e-5, 1e-3)`` m^2/s per interface).  The
  inverse is stored as a dense ``n_c x n_c`` block per column; it is
  non-negative, row-stochastic and volume-conserving.

Both families share one sparsity pattern across the twelve months and are
returned in CSR form (int32 indices, float64 values ``[nmat, nnz]``).
"""

from dataclasses import dataclass

import numpy as np

from .grid import Grid

SECONDS_PER_YEAR = 360.0 * 86400.0  # 360-day year (section 5.1)


@dataclass
class Transport:
    nmat: int
    nstep: int
    ae_rowptr: np.ndarray   # [n+1] int32
    ae_colidx: np.ndarray   # [nnz_e] int32
    ae_val: np.ndarray      # [nmat, nnz_e] float64
    ai_rowptr: np.ndarray
    ai_colidx: np.ndarray
    ai_val: np.ndarray      # [nmat, nnz_i] float64

    @property
    def ae_nnz(self) -> int:
        return int(self.ae_colidx.size)

    @property
    def ai_nnz(self) -> int:
        return int(self.ai_colidx.size)


def _faces(grid: Grid):
    """Wet horizontal faces (a, b, layer, kind); kind 0 = east, 1 = north."""
    idx = grid.index_map()
    fa, fb, fk, kind, fj, fi = [], [], [], [], [], []
    K, J, I = idx.shape
    jj, ii = np.meshgrid(np.arange(J), np.arange(I), indexing="ij")
    for k in range(K):
        a = idx[k]
        # east neighbour (periodic in longitude)
        b = np.roll(a, -1, axis=1)
        m = (a >= 0) & (b >= 0)
        if I == 1:
            m[:] = False
        fa.append(a[m]); fb.append(b[m]); fk.append(np.full(m.sum(), k))
        kind.append(np.zeros(m.sum(), dtype=np.int8)); fj.append(jj[m]); fi.append(ii[m])
        # north neighbour (no crossing of the poles)
        b = np.full_like(a, -1)
        b[:-1] = a[1:]
        m = (a >= 0) & (b >= 0)
        fa.append(a[m]); fb.append(b[m]); fk.append(np.full(m.sum(), k))
        kind.append(np.ones(m.sum(), dtype=np.int8)); fj.append(jj[m]); fi.append(ii[m])
    cat = np.concatenate
    return cat(fa), cat(fb), cat(fk), cat(kind), cat(fj), cat(fi), idx


def _stream_function(idx: np.ndarray, rng: np.random.Generator, vol_scale: np.ndarray):
    """Corner stream function [K, J+1, I], zero on corners adjacent to land or poles.

    Values are multiples of a power of two no larger than 2^21 units, so the
    face fluxes (corner differences) and their sums are exact in float64 and
    the discrete flow is exactly divergence-free.
    """
    K, J, I = idx.shape
    wet = idx >= 0
    psi = np.zeros((K, J + 1, I))
    for k in range(K):
        unit = 2.0 ** np.floor(np.log2(max(vol_scale[k], 1e-300))) / 2.0 ** 20
        vals = np.round(rng.uniform(0.0, 1.0, size=(J + 1, I)) * 2.0 ** 20) * unit
        ok = np.zeros((J + 1, I), dtype=bool)
        ok[1:J] = True
        w = wet[k]
        wl = np.roll(w, 1, axis=1)   # cell (j, ic-1)
        # corner (jc, ic) touches cells (jc-1, ic-1), (jc-1, ic), (jc, ic-1), (jc, ic)
        ok[1:J] &= w[:-1] & wl[:-1] & w[1:] & wl[1:]
        psi[k] = np.where(ok, vals, 0.0)
    return psi


def _explicit_month(grid, faces, vol, rng, scale_to=0.5):
    fa, fb, fk, kind, fj, fi, idx = faces
    K, J, I = idx.shape
    n = grid.n
    g = rng.uniform(0.0, 1.0, size=fa.size) * np.minimum(vol[fa], vol[fb])
    layer_vol = np.array([np.median(vol[idx[k][idx[k] >= 0]]) if (idx[k] >= 0).any() else 1.0
                          for k in range(K)])
    psi = _stream_function(idx, rng, 0.5 * layer_vol)
    ip1 = (fi + 1) % I
    # flux from a to b across the face (positive = a -> b)
    f_east = psi[fk, fj + 1, ip1] - psi[fk, fj, ip1]
    f_north = psi[fk, fj + 1, fi] - psi[fk, fj + 1, ip1]
    F = np.where(kind == 0, f_east, f_north)
    inflow_a = np.maximum(-F, 0.0)     # from b into a
    inflow_b = np.maximum(F, 0.0)      # from a into b
    off_ab = (g + inflow_a) / vol[fa]  # L[a, b]
    off_ba = (g + inflow_b) / vol[fb]  # L[b, a]
    rowsum = np.bincount(fa, weights=off_ab, minlength=n) + np.bincount(fb, weights=off_ba, minlength=n)
    s = scale_to / rowsum.max() if rowsum.max() > 0 else 0.0
    off_ab = s * off_ab
    off_ba = s * off_ba
    diag = 1.0 - (np.bincount(fa, weights=off_ab, minlength=n) + np.bincount(fb, weights=off_ba, minlength=n))
    return np.concatenate([diag, off_ab, off_ba])


def _implicit_month(grid, rng, dt_s, kappa_lo=1e-5, kappa_hi=1e-3):
    nc = grid.column_depths()
    dz = grid.dz
    blk_off = np.zeros(grid.ncol + 1, dtype=np.int64)
    blk_off[1:] = np.cumsum(nc.astype(np.int64) ** 2)
    val = np.empty(int(blk_off[-1]))
    kappa = rng.uniform(kappa_lo, kappa_hi, size=(grid.ncol, grid.nlayer))
    for m in np.unique(nc):
        cols = np.nonzero(nc == m)[0]
        M = np.broadcast_to(np.eye(m), (cols.size, m, m)).copy()
        for k in range(m - 1):
            gk = kappa[cols, k] / (0.5 * (dz[k] + dz[k + 1]))   # per unit area
            M[:, k, k] += dt_s * gk / dz[k]
            M[:, k, k + 1] -= dt_s * gk / dz[k]
            M[:, k + 1, k + 1] += dt_s * gk / dz[k + 1]
            M[:, k + 1, k] -= dt_s * gk / dz[k + 1]
        Ai = np.linalg.inv(M)
        pos = blk_off[cols][:, None] + np.arange(m * m)[None, :]
        val[pos.ravel()] = Ai.reshape(cols.size, m * m).ravel()
    return val


def implicit_pattern(grid: Grid):
    nc = grid.column_depths().astype(np.int64)
    rowptr = np.zeros(grid.n + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(np.repeat(nc, nc))
    cs = grid.col_start.astype(np.int64)
    colidx = np.concatenate([np.tile(np.arange(cs[c], cs[c + 1]), nc[c]) for c in range(grid.ncol)]) \
        if grid.ncol else np.zeros(0, dtype=np.int64)
    return rowptr.astype(np.int32), colidx.astype(np.int32)


def make_transport(grid: Grid, seed: int, nmat: int = 12, nstep: int = 2880) -> Transport:
    """Seeded monthly matrices; independent draws per month."""
    n = grid.n
    vol = grid.volumes()
    faces = _faces(grid)
    fa, fb = faces[0], faces[1]
    rows = np.concatenate([np.arange(n), fa, fb])
    cols = np.concatenate([np.arange(n), fb, fa])
    perm = np.lexsort((cols, rows))
    counts = np.bincount(rows, minlength=n)
    ae_rowptr = np.zeros(n + 1, dtype=np.int64)
    ae_rowptr[1:] = np.cumsum(counts)
    ae_colidx = cols[perm].astype(np.int32)

    ai_rowptr, ai_colidx = implicit_pattern(grid)
    dt_s = SECONDS_PER_YEAR / nstep

    ae_val = np.empty((nmat, ae_colidx.size))
    ai_val = np.empty((nmat, ai_colidx.size))
    ss = np.random.SeedSequence(seed)
    for m, child in enumerate(ss.spawn(nmat)):
        rng = np.random.default_rng(child)
        ae_val[m] = _explicit_month(grid, faces, vol, rng)[perm]
        ai_val[m] = _implicit_month(grid, rng, dt_s)
    return Transport(nmat=nmat, nstep=nstep,
                     ae_rowptr=ae_rowptr.astype(np.int32), ae_colidx=ae_colidx, ae_val=ae_val,
                     ai_rowptr=ai_rowptr, ai_colidx=ai_colidx, ai_val=ai_val)
