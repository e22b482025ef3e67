"""How the GPU parity tests measure a difference from the oracle.

The tracers of one state differ in size by orders of magnitude (PO4 near 2,
DOP near 1e-4, section 2.2.1), and the parameter gradient's components by
four (dJ/dlambda'_2 against dJ/dK_I).  A difference divided by the largest
value of the whole array would hold the small ones to almost nothing, so:

* states (every tracer stays positive within the parameter bounds) are
  compared point by point, each difference relative to the oracle's own
  value there;
* signed fields (tangents, cotangents, finite differences) are compared per
  state column (one tracer of one member), relative to the largest magnitude
  of that column;
* parameter gradients are compared component by component, each relative to
  its own value.

Each function returns the worst ratio and prints the per-tracer (or
per-component) figures, so that a GPU log shows the margin of every check.

The bars:

* ``STEP`` (one time step, point by point) 1e-13: a few ulp of the products,
  plus the insolation near the polar-night terminator.  There the daily-mean
  formula cancels (condition number up to ~2e4 on the global grids) and the
  arc cosine is steep, so the device's and the host's libm, each within an ulp,
  give light values that differ by up to ~1e-11 relative; the light-limited
  production then moves DOP by up to ~2e-14 of its value (seen in 64-member
  steps of the 256x128x23 grid).
* ``YEAR`` 1e-12 per model year, ``TANGENT`` 1e-11, ``ADJOINT`` 1e-10 (dJ/du
  and dJ/dy0), ``MISFIT`` 1e-12 (J per member).
* ``FD`` 1e-4 between two finite-difference products: each carries rounding
  noise of about eps |phi(y)| / h with h = 1e-8 |y| / |v|, which for the DOP
  column (values 1e-4 next to PO4 near 2, one h per member) is ~1e-5 of that
  column's largest derivative.
"""

import numpy as np

STEP = 1e-13
YEAR = 1e-12
TANGENT = 1e-11
ADJOINT = 1e-10
MISFIT = 1e-12
FD = 1e-4


def _cols(a):
    a = np.asarray(a, dtype=np.float64)
    return a.reshape(-1, a.shape[-1]) if a.ndim > 1 else a.reshape(-1, 1)


def _show(label, per_col, ntr):
    if label is None:
        return
    per_col = np.asarray(per_col)
    if ntr and per_col.size % ntr == 0 and per_col.size > ntr:
        per_tr = per_col.reshape(-1, ntr).max(axis=0)
    else:
        per_tr = per_col
    print(f"[parity] {label}: " + " ".join(f"{x:.2e}" for x in np.atleast_1d(per_tr)), flush=True)


def pointwise(got, exp, ntr=None, label=None):
    """max over points of |got - exp| / |exp|, for a positive field.

    The last axis indexes state columns (member * ntr + tracer); the printed
    figures are the worst ratio of each tracer over all members."""
    g, e = _cols(got), _cols(exp)
    if g.shape != e.shape:
        raise ValueError(f"shape {g.shape} vs {e.shape}")
    if not (e > 0).all():
        raise ValueError("pointwise comparison needs a positive reference field")
    per_col = (np.abs(g - e) / e).max(axis=0)
    _show(label, per_col, ntr)
    return float(per_col.max())


def columnwise(got, exp, ntr=None, label=None):
    """max over state columns of max |got - exp| / max |exp| within the column."""
    g, e = _cols(got), _cols(exp)
    if g.shape != e.shape:
        raise ValueError(f"shape {g.shape} vs {e.shape}")
    scale = np.abs(e).max(axis=0)
    if not (scale > 0).all():
        raise ValueError("a reference column is identically zero")
    per_col = np.abs(g - e).max(axis=0) / scale
    _show(label, per_col, ntr)
    return float(per_col.max())


def componentwise(got, exp, label=None):
    """max over components of |got - exp| / |exp| (parameter gradients, misfits).

    A component the oracle gives as exactly zero (the Martin exponent b of a
    grid with no layer below the euphotic zone, for one) is measured against
    the largest component instead."""
    g = np.asarray(got, dtype=np.float64).ravel()
    e = np.asarray(exp, dtype=np.float64).ravel()
    if g.shape != e.shape:
        raise ValueError(f"shape {g.shape} vs {e.shape}")
    scale = np.abs(e).max()
    if scale == 0:
        raise ValueError("every reference component is zero")
    per = np.abs(g - e) / np.where(e != 0, np.abs(e), scale)
    _show(label, per, None)
    return float(per.max())
