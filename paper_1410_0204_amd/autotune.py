"""Launch-configuration autotuner for libtmm.

For one handle, parameter table and initial state it tries the compiled
kernel variants and launch shapes that change speed but not results beyond
rounding order:

* one member: the single-launch year kernel with several domain sizes (rows
  per workgroup; each domain is one workgroup of up to 256 or 512 rows), and
  the launch-per-step tile kernel with each tile size (32 .. 256 rows per
  workgroup);
* ensembles: the member-parallel kernel (one wavefront per water column,
  lane = member) with 2, 4 or 8 wavefronts per workgroup and its column order
  (bands of 4 .. 32 latitude rows swept by longitude, or the natural order),
  the tiled member kernel (4 or 8 neighbouring columns per workgroup, each
  state row their explicit rows read staged once per layer in LDS; bands of 2
  latitude rows), and the tile kernel with each tile size.

Each candidate runs one untimed model year, whose final state must equal the
default configuration's to 1e-12 relative at every point (a candidate that
differs more is rejected), then timed years (HIP events on the handle's
stream).  The winner is applied to the handle.  Results are kept in a JSON
table keyed by the workload's shape; ``apply_tuned`` loads the table shipped
with the package (``tuned.json``, measured on an MI355X) or another one and
applies the entry for a handle, which the drivers and the benchmark do by
default.

Usage on a GPU: python -m paper_1410_0204_amd.autotune global 1 [out.json]
"""

import json
import os
import sys

import numpy as np
import torch

from . import tmm as T

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED_PATH = os.path.join(HERE, "tuned.json")

DOMAIN_ROWS = (128, 160, 192, 224, 256, 320, 384, 448, 512)
TILE_ROWS = (32, 64, 128, 256)
MEMBER_WAVES = (2, 4, 8)
MEMBER_BANDS = (-1, 4, 8, 16, 32)
MEMBER_TILES = (4, 8)

# the tiled member kernel is switched off before the band order changes (it needs bands)
DEFAULTS = {T.TMM_OPT_MEMBER_TILE: 0, T.TMM_OPT_MEMBER_PACK: 1, T.TMM_OPT_PERSISTENT: 1, T.TMM_OPT_DOMAIN_ROWS: 0,
            T.TMM_OPT_MEMBER_KERNEL_MIN: -1,
            T.TMM_OPT_GRAPH: 1, T.TMM_OPT_TILE_ROWS: 0, T.TMM_OPT_MEMBER_WAVES: 0, T.TMM_OPT_MEMBER_BAND_ROWS: 0}

NAMES = {T.TMM_OPT_PERSISTENT: "persistent", T.TMM_OPT_DOMAIN_ROWS: "domain_rows",
         T.TMM_OPT_MEMBER_KERNEL_MIN: "member_kernel_min", T.TMM_OPT_GRAPH: "graph",
         T.TMM_OPT_TILE_ROWS: "tile_rows", T.TMM_OPT_MEMBER_WAVES: "member_waves",
         T.TMM_OPT_MEMBER_BAND_ROWS: "member_band_rows", T.TMM_OPT_MEMBER_TILE: "member_tile",
         T.TMM_OPT_MEMBER_PACK: "member_pack"}


def signature(t, nbatch):
    """Key of a workload shape: points, columns, layers, model, internal BGC steps, members."""
    return (f"n{t.n}_c{int(t.desc.ncol)}_l{int(t.desc.nlayer)}_m{t.model}_s{max(int(t.desc.nbgc), 1)}"
            f"_b{nbatch}")


def describe(options):
    """The options of a candidate by name (for logs and the benchmark line)."""
    return {NAMES[int(k)]: int(v) for k, v in options.items()}


def candidates(t, nbatch):
    """Option sets to try for this handle and member count (each applied on top of DEFAULTS)."""
    out = []
    if nbatch == 1 and t.query(T.TMM_Q_PERSISTENT):
        for rows in DOMAIN_ROWS:
            out.append({T.TMM_OPT_PERSISTENT: 1, T.TMM_OPT_DOMAIN_ROWS: rows})
    for rows in TILE_ROWS:
        out.append({T.TMM_OPT_PERSISTENT: 0, T.TMM_OPT_MEMBER_KERNEL_MIN: 0, T.TMM_OPT_TILE_ROWS: rows})
    # the library's default crossover to the member kernel (see TMM_OPT_MEMBER_KERNEL_MIN)
    kmin = 2 if t.ntracer == 2 and max(int(t.desc.nbgc), 1) == 1 and int(t.desc.nlayer) <= 24 else 6
    if nbatch > 1 and t.ntracer <= 2:
        for waves in MEMBER_WAVES:
            for band in MEMBER_BANDS:
                # the member kernel at this width; narrower batches (members that
                # finish early) keep the default crossover to the tile kernel
                out.append({T.TMM_OPT_PERSISTENT: 0,
                            T.TMM_OPT_MEMBER_KERNEL_MIN: min(kmin, nbatch),
                            T.TMM_OPT_MEMBER_WAVES: waves, T.TMM_OPT_MEMBER_BAND_ROWS: band})
        if t.ntracer == 2:
            for tile in MEMBER_TILES:
                out.append({T.TMM_OPT_PERSISTENT: 0,
                            T.TMM_OPT_MEMBER_KERNEL_MIN: min(kmin, nbatch),
                            T.TMM_OPT_MEMBER_BAND_ROWS: 2, T.TMM_OPT_MEMBER_TILE: tile})
    return out


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


def _time_steps(t, y0, steps, j0=1439):
    a, b = t.state(), t.state()
    t.step(j0, y0, a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(t.stream)
    for k in range(steps):
        t.step(j0 + k, a if k % 2 == 0 else b, b if k % 2 == 0 else a)
    e.record(t.stream)
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps * t.nstep


def _max_rel(got, ref):
    """max over points of |got - ref| / |ref| (states are positive)."""
    return float((np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)).max())


def tune(t, u, y0, years=2, rtol=1e-12, log=None, only=None, steps=0):
    """Times every candidate (or the list ``only``) for parameters u (one row
    per member) from state y0 (host array); applies the fastest validated one
    and returns {signature, best, candidates}.  With ``steps`` > 0 (large
    ensembles, where a model year per candidate takes too long) a candidate is
    checked on one time step (to 1e-14) and timed over that many steps,
    scaled to a model year; the single-launch year kernel is then not tried."""
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    t.set_params(u)
    nb = u.shape[0]
    yd = t.state(np.asarray(y0, dtype=np.float64))
    apply(t, DEFAULTS)

    def run(handle):
        if steps > 0:
            return handle.step(1439, yd)
        return handle.year(yd, nyears=1, residuals=False)[0]

    ref = run(t).cpu().numpy()
    tol = 1e-14 if steps > 0 else rtol
    results = []
    for cand in (only if only is not None else candidates(t, nb)):
        if steps > 0 and int(cand.get(T.TMM_OPT_PERSISTENT, 0)):
            continue
        apply(t, DEFAULTS)
        try:
            apply(t, cand)
        except T.TmmError as ex:          # a variant this handle cannot run (e.g. a tile too wide)
            rec = {"options": {str(k): int(v) for k, v in cand.items()}, "named": describe(cand),
                   "ms_per_year": float("inf"), "max_rel_diff": None, "ok": False, "refused": str(ex)}
            results.append(rec)
            if log:
                log(rec)
            continue
        err = _max_rel(run(t).cpu().numpy(), ref)
        ok = err <= tol
        if not ok:
            ms = float("inf")
        elif steps > 0:
            ms = _time_steps(t, yd, steps)
        else:
            ms = _time_years(t, yd, years)
        rec = {"options": {str(k): int(v) for k, v in cand.items()}, "named": describe(cand), "ms_per_year": ms,
               "max_rel_diff": err, "ok": ok}
        results.append(rec)
        if log:
            log(rec)
    best = min((r for r in results if r["ok"]), key=lambda r: r["ms_per_year"])
    apply(t, DEFAULTS)
    apply(t, {int(k): v for k, v in best["options"].items()})
    return {"signature": signature(t, nb), "best": best, "candidates": results}


def save(result, path=TUNED_PATH, device=None):
    table = {}
    if os.path.exists(path):
        with open(path) as fh:
            table = json.load(fh)
    table[result["signature"]] = {"options": result["best"]["options"], "named": result["best"]["named"],
                                  "ms_per_year": result["best"]["ms_per_year"],
                                  "device": device or (torch.cuda.get_device_name(0)
                                                       if torch.cuda.is_available() else "unknown"),
                                  "candidates": len(result["candidates"])}
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(t, nbatch, path=TUNED_PATH):
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        table = json.load(fh)
    return table.get(signature(t, nbatch))


def apply_tuned(t, nbatch, path=TUNED_PATH):
    """Applies the tuned options for this handle's shape and member count, if
    the table has them; returns the entry (with the options by name) or None."""
    if not hasattr(t, "set_option") or not hasattr(t, "desc"):
        return None                      # not a libtmm handle (e.g. a host-side stand-in)
    rec = lookup(t, nbatch, path)
    if rec is None:
        return None
    apply(t, DEFAULTS)
    apply(t, {int(k): v for k, v in rec["options"].items()})
    return rec


load = apply_tuned


def main(argv):
    """Tunes a named workload with nbatch members and saves the result."""
    import synth
    name, nbatch = argv[0], int(argv[1])
    path = argv[2] if len(argv) > 2 else TUNED_PATH
    inp = synth.by_name(name)
    U = synth.nominal(inp.model) if nbatch == 1 else synth.latin_hypercube(inp.model, nbatch, seed=17)
    t = T.TMM(inp.desc_arrays(), nbatch_max=nbatch)
    res = tune(t, U, inp.initial_state(nbatch), years=2, steps=20 if inp.n * nbatch > 4000000 else 0,
               log=lambda r: print(json.dumps(r), flush=True))
    save(res, path)
    print(json.dumps({"signature": res["signature"], "best": res["best"]}), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
