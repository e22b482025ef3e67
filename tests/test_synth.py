"""Construction invariants of the synthetic inputs (no method arithmetic)."""

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from synth.transport import SECONDS_PER_YEAR


def _csr(rowptr, colidx, val, n):
    return sp.csr_matrix((val, colidx, rowptr), shape=(n, n))


@pytest.mark.parametrize("name", ["tiny", "small"])
def test_matrices_stochastic_and_conservative(name):
    inp = synth.by_name(name)
    g, tm = inp.grid, inp.tm
    V = g.volumes()
    one = np.ones(g.n)
    for m in range(tm.nmat):
        Ae = _csr(tm.ae_rowptr, tm.ae_colidx, tm.ae_val[m], g.n)
        Ai = _csr(tm.ai_rowptr, tm.ai_colidx, tm.ai_val[m], g.n)
        for A in (Ae, Ai):
            assert np.abs(A @ one - 1.0).max() < 1e-14          # row-stochastic
            assert np.abs(A.T @ V - V).max() < 1e-14 * V.max()  # volume-conserving
            assert A.data.min() >= 0.0
        assert Ae.diagonal().min() == pytest.approx(0.5, abs=1e-15)


def test_implicit_is_inverse_of_vertical_diffusion(tiny_n):
    """Ai (I - dt_s K_v) = I per column, with K_v rebuilt from the block's own inverse."""
    g, tm = tiny_n.grid, tiny_n.tm
    nc = g.column_depths()
    off = np.concatenate([[0], np.cumsum(nc.astype(np.int64) ** 2)])
    for m in (0, 5):
        for c in range(g.ncol):
            k = nc[c]
            A = tm.ai_val[m, off[c]:off[c + 1]].reshape(k, k)
            M = np.linalg.inv(A)
            # I - dt K_v is tridiagonal with unit row sums and non-positive off-diagonals
            assert np.abs(np.triu(M, 2)).max(initial=0) < 1e-12
            assert np.abs(M.sum(1) - 1).max() < 1e-13
            assert (M - np.diag(np.diag(M)) <= 1e-15).all()
            assert np.abs(A @ M - np.eye(k)).max() < 1e-14


def test_grid_counts_and_order():
    inp = synth.global_2p8()
    g = inp.grid
    assert g.n == 52749 and g.ncol == 4448
    assert g.nlayer == 15 and g.nlon == 128 and g.nlat == 64
    nc = g.column_depths()
    assert nc.min() >= 1 and nc.max() <= 15
    key = g.col_j.astype(np.int64) * g.nlon + g.col_i
    assert (np.diff(key) > 0).all()                  # latitude row, then longitude
    assert g.dz[0] == 50.0 and g.dz[-1] == 700.0
    assert g.dz.sum() == pytest.approx(5625.0)
    # every latitude row's cells tile the sphere: sum over all cells = 4 pi R^2
    lat_s = np.radians(g.lat_c - 90.0 / g.nlat)
    lat_n = np.radians(g.lat_c + 90.0 / g.nlat)
    full = (synth.grid.EARTH_RADIUS ** 2 * 2 * np.pi * (np.sin(lat_n) - np.sin(lat_s))).sum()
    assert full == pytest.approx(4 * np.pi * synth.grid.EARTH_RADIUS ** 2, rel=1e-12)
    row_area = {j: a for j, a in zip(g.col_j, g.area)}
    assert sum(row_area[j] * g.nlon for j in row_area) <= full
    assert SECONDS_PER_YEAR / inp.nstep == 10800.0


def test_same_pattern_every_month_and_seeded(tiny_n):
    again = synth.tiny()
    assert np.array_equal(again.tm.ae_val, tiny_n.tm.ae_val)
    assert np.array_equal(again.tm.ai_val, tiny_n.tm.ai_val)
    assert not np.array_equal(tiny_n.tm.ae_val[0], tiny_n.tm.ae_val[1])
    # explicit matrix couples only horizontal neighbours in the same layer
    g = tiny_n.grid
    layer = g.row_layer()
    rows = np.repeat(np.arange(g.n), np.diff(tiny_n.tm.ae_rowptr))
    assert (layer[rows] == layer[tiny_n.tm.ae_colidx]).all()
    # implicit matrix couples only points of one water column
    col = g.row_column()
    rows = np.repeat(np.arange(g.n), np.diff(tiny_n.tm.ai_rowptr))
    assert (col[rows] == col[tiny_n.tm.ai_colidx]).all()


def test_params_within_bounds():
    for model in (synth.MODEL_N, synth.MODEL_NDOP):
        lo, hi = synth.bounds(model)
        u = synth.latin_hypercube(model, 64, seed=3)
        assert ((u >= lo) & (u <= hi)).all()
        # one sample per stratum in every coordinate
        for p in range(lo.size):
            strata = np.floor((u[:, p] - lo[p]) / (hi[p] - lo[p]) * 64).astype(int)
            assert sorted(strata) == list(range(64))
        nom = synth.nominal(model)
        assert ((nom >= lo) & (nom <= hi)).all()
        hid = synth.hidden_params(model, seed=1)
        assert ((hid >= lo) & (hid <= hi)).all()
    L = synth.spinup_lengths(64, seed=4)
    assert L.min() >= 1 and L.max() <= 8
