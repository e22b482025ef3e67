"""Launch-configuration autotuner for libtmm.

For one handle and ensemble size it tries every execution option that may
change speed but not results beyond rounding order:

* single member: the persistent year kernel with several domain sizes
  (rows per workgroup), and the launch-per-step path with and without graph
  capture;
* ensembles: the member-parallel step kernel and the tile kernel, with and
  without graph capture.

Each candidate runs one untimed model year, then timed years (HIP events on
the handle's stream).  Its final state is checked against the default
configuration's (max relative difference <= 1e-12); a candidate that differs
more is rejected.  The winner is applied to the handle and can be written to
and read back from a JSON table keyed by the workload's shape.
"""

import json
import os

import numpy as np
import torch

from . import tmm as T

DOMAIN_ROWS = (160, 192, 224, 256, 320, 448)


def _signature(t, nbatch):
    return f"n{t.n}_c{int(t.desc.ncol)}_l{int(t.desc.nlayer)}_m{t.model}_b{nbatch}"


def _candidates(t, nbatch):
    out = []
    if nbatch == 1 and t.query(T.TMM_Q_PERSISTENT):
        for rows in DOMAIN_ROWS:
            out.append({T.TMM_OPT_PERSISTENT: 1, T.TMM_OPT_DOMAIN_ROWS: rows})
    for graph in (1, 0):
        if nbatch > 1:
            out.append({T.TMM_OPT_PERSISTENT: 0, T.TMM_OPT_MEMBER_KERNEL_MIN: 1, T.TMM_OPT_GRAPH: graph})
        out.append({T.TMM_OPT_PERSISTENT: 0, T.TMM_OPT_MEMBER_KERNEL_MIN: 0, T.TMM_OPT_GRAPH: graph})
    return out


DEFAULTS = {T.TMM_OPT_PERSISTENT: 1, T.TMM_OPT_DOMAIN_ROWS: 0, T.TMM_OPT_MEMBER_KERNEL_MIN: 16, T.TMM_OPT_GRAPH: 1}


def apply(t, options):
    for opt, val in options.items():
        t.set_option(int(opt), int(val))


def _time_years(t, y0, years):
    out = t.state()
    t.year(y0, nyears=1, out=out, residuals=False)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(t.stream)
    t.year(y0, nyears=years, out=out, residuals=False)
    e.record(t.stream)
    torch.cuda.synchronize()
    return s.elapsed_time(e) / years


def tune(t, u, y0, years=2, rtol=1e-12, log=None):
    """Times every candidate for parameters u (one row per member) from state
    y0 (host array); applies and returns the fastest validated one."""
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    t.set_params(u)
    nb = u.shape[0]
    yd = t.state(np.asarray(y0, dtype=np.float64))
    apply(t, DEFAULTS)
    ref, _ = t.year(yd, nyears=1, residuals=False)
    ref = ref.cpu().numpy()
    scale = np.abs(ref).max()
    results = []
    for cand in _candidates(t, nb):
        apply(t, DEFAULTS)
        apply(t, cand)
        got, _ = t.year(yd, nyears=1, residuals=False)
        err = float(np.abs(got.cpu().numpy() - ref).max() / scale)
        ok = err <= rtol
        ms = _time_years(t, yd, years) if ok else float("inf")
        rec = {"options": {str(k): v for k, v in cand.items()}, "ms_per_year": ms, "max_rel_diff": err, "ok": ok}
        results.append(rec)
        if log:
            log(rec)
    best = min((r for r in results if r["ok"]), key=lambda r: r["ms_per_year"])
    apply(t, DEFAULTS)
    apply(t, {int(k): v for k, v in best["options"].items()})
    return {"signature": _signature(t, nb), "best": best, "candidates": results}


def save(result, path):
    table = {}
    if os.path.exists(path):
        with open(path) as fh:
            table = json.load(fh)
    table[result["signature"]] = {"options": result["best"]["options"], "ms_per_year": result["best"]["ms_per_year"]}
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def load(t, nbatch, path):
    """Applies a saved configuration for this workload shape; returns it, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        table = json.load(fh)
    rec = table.get(_signature(t, nbatch))
    if rec is None:
        return None
    apply(t, DEFAULTS)
    apply(t, {int(k): v for k, v in rec["options"].items()})
    return rec
