"""Throughput of the transport-matrix year map on one MI355X.

A "step" of this benchmark is one model year (2880 time steps) of the
global 128x64x15 workload (52749 wet points in 4448 columns, N-DOP model,
two tracers, float64), i.e. one evaluation of the year map phi that spin-up
and Newton-Krylov iterate.  Inputs are synthetic and seeded, shaped like the
paper's 2.8125-degree configuration; they are resident in HBM before timing
starts.

Printed as one JSON line: model-years/s, the effective bandwidth of the step
kernel against MI355X peak HBM bandwidth (roofline), the bytes the kernel
really moves past the L2 (from the committed counter summary), the latency
floor of a time step measured on the device (exchange round trip and
workgroup barriers), the adjoint/forward cost ratio, the batched ensemble
against one-member runs (256x128x23 grid, 64 members), Newton-Krylov to the
periodic solution, and the CPU oracle's rate on the host as a reported
baseline (single thread and all threads).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-ensemble] [--no-newton]

Further measurements, each printed as its own JSON line (not run by default):
  --mode newton       Newton-Krylov steady periodic solve on the same grid
                      (FD and tangent Jacobian-vector products), with spin-up
                      at the same cost for comparison;
  --mode ensemble     64 N-DOP parameter vectors (Latin hypercube) with spin-up
                      lengths 1..8 years on the 256x128x23 grid, batched, against
                      one-member runs;
  --mode copy         a plain 512 MiB device copy, for scaling hardware byte
                      counters;
  --mode grids        the launch-per-step path on the global, 256x128x23 and
                      1.0-degree 360x180x23 grids (bandwidth against grid size).
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_step(n, nnz_e, nnz_i, W):
    """Algorithmic bytes of one time step: both bracketing months' values (8 B
    each) and the column index (4 B) of every nonzero of Ae and Ai, the two
    CSR row-pointer arrays, and the state read and written."""
    return (nnz_e + nnz_i) * (2 * 8 + 4) + 2 * 4 * (n + 1) + 2 * 8 * n * W


def kernel_source_hash():
    from paper_1410_0204_amd.build import source_hash
    return source_hash()


def measured_traffic(kernel, workload="global_128x64x15"):
    """Bytes per launch past the L2 (FETCH_SIZE + WRITE_SIZE, calibrated on a
    plain copy) from the committed counter summary, if it was taken with the
    current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec["bytes_per_launch"]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inp, u, B):
    """The oracle (the same C source the tests check against) built for this
    host with -O3 -march=native -fopenmp, which gives the plain build's results
    bit for bit: one model year of the headline workload, median of 3 years
    after a warm-up year, on one thread and on every thread this process may
    use."""
    import shutil
    import tempfile
    import oracle
    from oracle import build as obuild
    d = tempfile.mkdtemp(prefix="tmm_oracle_timing_")
    try:
        lib = obuild.build_timing(os.path.join(d, "liboracle_timing.so"))
        o = oracle.Oracle(inp, lib_path=lib)
        y = inp.initial_state()
        allowed = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
        rows = {}
        for want in sorted({1, allowed}):
            used = oracle.threads(want, lib)
            o.year(u, y, 1)                                    # warm-up
            times = []
            for _ in range(3):
                t0 = time.perf_counter()
                o.year(u, y, 1)
                times.append(time.perf_counter() - t0)
            med = sorted(times)[1]
            rows[want] = {"threads": used, "s_per_year": med, "model_years_per_s": 1.0 / med,
                          "effective_GBps": B * inp.nstep / med / 1e9, "years_s": times}
            log(f"[bench] cpu oracle, {used} thread(s): {med:.2f} s per model year (median of 3)")
        # the oracle's own adjoint/forward ratio (full-trajectory reverse sweep), on every thread
        import synth
        n, W = inp.n, inp.ntracer
        obs = (np.broadcast_to(inp.initial_state(), (12, n, W))
               * (1 + 0.05 * synth.obs_noise((12, n, W), seed=3)))
        t0 = time.perf_counter()
        o.year_adjoint(u, y, obs)
        adj_s = time.perf_counter() - t0
        rows[allowed]["adjoint_s"] = adj_s
        rows[allowed]["adjoint_forward_ratio"] = adj_s / rows[allowed]["s_per_year"]
        log(f"[bench] cpu oracle adjoint year, {rows[allowed]['threads']} thread(s): {adj_s:.2f} s "
            f"({adj_s / rows[allowed]['s_per_year']:.2f}x its forward year)")
    finally:
        shutil.rmtree(d, ignore_errors=True)
    full = rows[allowed]
    return {"value": full["model_years_per_s"], "unit": "model-years/s", "cores": full["threads"],
            "kind": "oracle",
            "sample": (f"one model year (2880 steps) of the same global 128x64x15 N-DOP workload, median of 3 "
                       f"years after one warm-up year, C oracle built with gcc -O3 -march=native -fopenmp "
                       f"(bitwise equal to the plain build), {full['threads']} threads"),
            "single_thread": rows[1], "all_threads": full, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0))}


def latency_floor(t, us_per_step):
    """Per-step floor of the single-launch year kernel from the primitives it
    chains in every step, measured on this device: one hand-over of a value
    to another workgroup (half a store-and-poll round trip, the slower of
    same-XCD and cross-XCD pairs: every step has both) and the step's
    workgroup barriers (one with wave-aligned water columns, else three)."""
    from paper_1410_0204_amd import tmm
    p = t.probe_exchange(2000)
    nbar = 1 if t.query(tmm.TMM_Q_WAVE_LOCAL) else 3
    hop = 0.5 * max(p["round_trip_same_xcd_us"], p["round_trip_cross_xcd_us"])
    floor = hop + nbar * p["barrier_us"]
    p.update({"hop_us": hop, "barriers_per_step": nbar, "floor_us_per_step": floor,
              "floor_over_step": floor / us_per_step,
              "model": f"one hand-over of the state (half a round trip) + {nbar} workgroup barrier(s) per step"})
    log(f"[bench] exchange probe: round trip {p['round_trip_same_xcd_us']:.3f} us (same XCD), "
        f"{p['round_trip_cross_xcd_us']:.3f} us (across XCDs), barrier {p['barrier_us']:.4f} us, "
        f"agent load {p['agent_load_us']:.3f} us -> floor {floor:.3f} us per step ({floor / us_per_step:.2f} of it)")
    return p


def newton_leg(t, inp, u):
    """Newton-Krylov to ||phi(y) - y|| <= 1e-8 from the constant initial field
    (FD and tangent Jacobian-vector products, GMRES(30), Eisenstat-Walker,
    line search), and spin-up for as many model years as the FD solve used."""
    import torch
    from paper_1410_0204_amd import drivers
    y0 = inp.initial_state()
    out = {"workload": "global_128x64x15 N-DOP", "tol": 1e-8, "restart": 30}
    # one untimed Newton step with a few Krylov products first: the timed solves then do not
    # include the first use of the device vector kernels (their code objects load on first call)
    drivers.newton_krylov(t, u, y0, tol=1.0, jvp="fd", restart=30, max_newton=1, max_krylov=4)
    for jvp in ("fd", "tangent"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y, hist = drivers.newton_krylov(t, u, y0, tol=1e-8, jvp=jvp, restart=30, max_newton=30, max_krylov=300)
        dt = time.perf_counter() - t0
        out[jvp] = {"fnorm_first": hist["fnorm"][0], "fnorm_last": hist["fnorm"][-1], "year_maps": hist["years"],
                    "seconds": dt, "newton_iterations": len(hist["newton"])}
        log(f"[bench] Newton ({jvp} JVP): |F| {hist['fnorm'][0]:.3e} -> {hist['fnorm'][-1]:.3e}, "
            f"{len(hist['newton'])} Newton steps, {hist['years']} year maps, {dt:.2f} s")
    years = out["fd"]["year_maps"]
    t0 = time.perf_counter()
    _, r = drivers.spinup(t, u, y0, years=years)
    out["spinup_same_years"] = {"years": years, "residual_last": float(r[-1]), "seconds": time.perf_counter() - t0}
    log(f"[bench] spin-up for {years} years: residual {r[0]:.3e} -> {r[-1]:.3e}")
    return out


def cpu_ensemble_sample(inp, U, L, steps=2):
    """The oracle's time for the batched ensemble, extrapolated from a bounded
    sample: `steps` time steps at full width (W = 2 x members) and at one
    member (W = 2), timing build of the oracle on every thread this process
    may use, one untimed step before each; a step at W active columns is
    taken as linear in W between the two, summed over the years of the
    uneven spin-up lengths (batched) or over the member-years at W = 2
    (sequential)."""
    import shutil
    import tempfile
    import oracle
    from oracle import build as obuild
    d = tempfile.mkdtemp(prefix="tmm_oracle_timing_")
    try:
        lib = obuild.build_timing(os.path.join(d, "liboracle_timing.so"))
        o = oracle.Oracle(inp, lib_path=lib)
        used = oracle.threads(int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0))), lib)
        nm = U.shape[0]
        per = {}
        for w, uu in ((2 * nm, U), (2, U[:1])):
            y = inp.initial_state(uu.shape[0])
            y = o.step(uu, 0, y)                       # untimed
            t0 = time.perf_counter()
            for j in range(1, steps + 1):
                y = o.step(uu, j, y)
            per[w] = (time.perf_counter() - t0) / steps
            log(f"[bench] cpu oracle, ensemble grid, W = {w}: {per[w]:.3f} s per step ({used} threads)")
    finally:
        shutil.rmtree(d, ignore_errors=True)
    wide, one = per[2 * nm], per[2]

    def step_s(W):
        return one + (wide - one) * (W - 2) / (2 * nm - 2)
    batched = sum(inp.nstep * step_s(2 * int((L > yr).sum())) for yr in range(int(L.max())))
    sequential = int(L.sum()) * inp.nstep * one
    return {"threads": used, "steps_timed": steps, "s_per_step_full_width": wide, "s_per_step_one_member": one,
            "batched_s_extrapolated": batched, "sequential_s_extrapolated": sequential,
            "batched_member_years_per_s": int(L.sum()) / batched, "speedup": sequential / batched,
            "note": "extrapolated from the timed steps: a step taken as linear in the number of active columns"}


def ensemble_leg(dev, stream, steps=30, cpu=False):
    """64 N-DOP parameter vectors (Latin hypercube) with spin-up lengths of
    1..8 model years on the 256x128x23 grid (500000 points): full-width steps
    (W = 128) timed alone, then the whole batched run with compaction of
    finished members, against one member's model year times the member-years."""
    import torch
    import synth
    from paper_1410_0204_amd import tmm
    t0 = time.perf_counter()
    inp = synth.ensemble_1p4()
    gen_s = time.perf_counter() - t0
    log(f"[bench] ensemble inputs {inp.name}: n={inp.n} ({gen_s:.1f} s to generate)")
    nm = 64
    U = synth.latin_hypercube(synth.MODEL_NDOP, nm, seed=17)
    L = synth.spinup_lengths(nm, seed=18)
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=nm, device=dev, stream=stream)
    from paper_1410_0204_amd import autotune
    tuned = autotune.apply_tuned(t, nm)
    t.set_params(U)
    y0 = t.state(inp.initial_state(nm))
    s, e = _events()
    buf = [t.state(), t.state()]
    t.step(0, y0, buf[0])
    torch.cuda.synchronize()
    s.record(stream)
    for j in range(steps):
        t.step(j, buf[j % 2], buf[(j + 1) % 2])
    e.record(stream)
    torch.cuda.synchronize()
    us = s.elapsed_time(e) * 1000.0 / steps
    Bfull = bytes_per_step(inp.n, inp.tm.ae_nnz, inp.tm.ai_nnz, 2 * nm)
    s.record(stream)
    out_b, _ = t.year(y0, nyears=int(L.max()), years_per_member=L, residuals=False)
    e.record(stream)
    torch.cuda.synchronize()
    ms_b = s.elapsed_time(e)
    member_years = int(L.sum())
    # the plain method: one member at a time, in its own best configuration
    autotune.apply(t, autotune.DEFAULTS)
    tuned1 = autotune.apply_tuned(t, 1)
    t.set_params(U[0])
    y1 = t.state(inp.initial_state(1))
    t.year(y1, nyears=1, residuals=False)
    torch.cuda.synchronize()
    s.record(stream)
    t.year(y1, nyears=1, residuals=False)
    e.record(stream)
    torch.cuda.synchronize()
    ms_1 = s.elapsed_time(e)
    # what the byte counts alone predict: every year of the batch moves the
    # matrices once for all members still running
    B1 = bytes_per_step(inp.n, inp.tm.ae_nnz, inp.tm.ai_nnz, 2)
    batched_bytes = sum(bytes_per_step(inp.n, inp.tm.ae_nnz, inp.tm.ai_nnz, 2 * int((L > yr).sum()))
                        for yr in range(int(L.max())))
    res = {"workload": "ensemble_256x128x23 N-DOP", "n": inp.n, "members": nm, "member_years": member_years,
           "full_width_us_per_step": us, "full_width_bytes_per_step": Bfull,
           "full_width_GBps": Bfull / (us * 1e-6) / 1e9,
           "full_width_frac": Bfull / (us * 1e-6) / 1e9 / HBM_PEAK_GBPS,
           "batched_ms": ms_b, "batched_member_years_per_s": member_years / (ms_b / 1000.0),
           "one_member_ms_per_year": ms_1, "sequential_member_years_per_s": 1000.0 / ms_1,
           "speedup": member_years * ms_1 / ms_b,
           "speedup_from_bytes": member_years * B1 / batched_bytes,
           "tuned": tuned["named"] if tuned else "library defaults",
           "tuned_one_member": tuned1["named"] if tuned1 else "library defaults",
           "inputs_generation_s": gen_s}
    log(f"[bench] ensemble: full-width step {us:.1f} us ({res['full_width_GBps']:.0f} GB/s, "
        f"{100 * res['full_width_frac']:.1f} % of peak); {member_years} member-years in {ms_b:.0f} ms "
        f"({res['batched_member_years_per_s']:.2f}/s) vs one member {ms_1:.1f} ms/year: "
        f"{res['speedup']:.2f}x (bytes alone: {res['speedup_from_bytes']:.2f}x)")
    t.close()
    del t, y0, buf, out_b, y1
    torch.cuda.empty_cache()
    if cpu:
        res["cpu_oracle"] = cpu_ensemble_sample(inp, U, L)
        c = res["cpu_oracle"]
        log(f"[bench] cpu oracle ensemble (extrapolated): batched {c['batched_s_extrapolated']:.0f} s, "
            f"sequential {c['sequential_s_extrapolated']:.0f} s ({c['speedup']:.2f}x); the GPU batch "
            f"{c['batched_s_extrapolated'] / (ms_b / 1000.0):.0f}x faster than the oracle's")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed model years")
    ap.add_argument("--warmup", type=int, default=2, help="untimed model years")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble leg")
    ap.add_argument("--no-newton", action="store_true", help="skip the Newton-Krylov leg")
    ap.add_argument("--mode", default="forward", choices=["forward", "newton", "ensemble", "copy", "grids"])
    ap.add_argument("--log", default=None, help="JSONL progress log (newton mode)")
    ap.add_argument("--grid-steps", type=int, default=0,
                    help="grids / ensemble modes: time this many single steps instead of model years")
    ap.add_argument("--member-band", type=int, default=None,
                    help="ensemble mode: latitude rows per band of the member kernel's column order (-1: natural)")
    ap.add_argument("--member-waves", type=int, default=None,
                    help="ensemble mode: wavefronts per workgroup of the member kernel")
    ap.add_argument("--member-tile", type=int, default=None,
                    help="ensemble mode: columns per workgroup of the tiled member kernel (0: off)")
    ap.add_argument("--forward-only", action="store_true",
                    help="skip the per-step comparison and the adjoint (for hardware counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X; --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)
    if args.mode != "forward":
        {"newton": bench_newton, "ensemble": bench_ensemble, "copy": bench_copy, "grids": bench_grids}[args.mode](args)
        return

    import torch
    import synth
    from paper_1410_0204_amd import tmm

    inp = synth.global_2p8()
    n, W = inp.n, inp.ntracer
    B = bytes_per_step(n, inp.tm.ae_nnz, inp.tm.ai_nnz, W)
    log(f"[bench] {inp.name}: n={n} ncol={inp.grid.ncol} nnz_e={inp.tm.ae_nnz} nnz_i={inp.tm.ai_nnz} "
        f"bytes/step={B}")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1, adjoint_nbatch_max=1, ckpt_every=240, device=dev, stream=stream)
    from paper_1410_0204_amd import autotune
    tuned = autotune.apply_tuned(t, 1)
    log(f"[bench] launch configuration: {tuned['named'] if tuned else 'library defaults'}")
    u = synth.nominal(inp.model)
    t.set_params(u)
    y0 = t.state(inp.initial_state())
    y1 = t.state()

    # warm-up years (spin-up from the constant field)
    y, _ = t.year(y0, nyears=max(args.warmup, 1), out=y1, residuals=False)
    torch.cuda.synchronize()

    persistent = bool(t.query(tmm.TMM_Q_PERSISTENT))
    kernel = "k_year_persistent" if persistent else "k_step"
    log(f"[bench] path: {kernel}" + (f" ({t.query(tmm.TMM_Q_DOMAINS)} domains on "
                                     f"{t.query(tmm.TMM_Q_COMPUTE_UNITS)} CUs)" if persistent else ""))

    # timed years: events on the stream the library launches on
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ya = t.state()
    torch.cuda.synchronize()
    start.record(stream)
    t.year(y, nyears=args.steps, out=ya, residuals=False)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    ms_per_year = ms / args.steps
    years_per_s = 1000.0 / ms_per_year
    us_per_step = ms * 1000.0 / (args.steps * inp.nstep)
    # one launch of the dominant kernel covers a model year (persistent) or a step
    units = inp.nstep if persistent else 1
    launches = args.steps if persistent else args.steps * inp.nstep
    us_per_launch = ms * 1000.0 / launches
    achieved = B * units / (us_per_launch * 1e-6) / 1e9
    log(f"[bench] forward: {ms_per_year:.3f} ms/model-year, {years_per_s:.2f} model-years/s, "
        f"{us_per_step:.2f} us/step, {achieved:.0f} GB/s effective")
    # the same years one call each, for the median and spread of single years
    single = []
    for _ in range(max(5, min(args.steps, 20))):
        start.record(stream)
        t.year(y, nyears=1, out=ya, residuals=False)
        stop.record(stream)
        torch.cuda.synchronize()
        single.append(start.elapsed_time(stop))
    single.sort()
    year_stats = {"years": len(single), "median_ms": single[len(single) // 2], "min_ms": single[0],
                  "max_ms": single[-1]}
    log(f"[bench] single years: median {year_stats['median_ms']:.3f} ms (min {single[0]:.3f}, max {single[-1]:.3f})")
    floor = latency_floor(t, us_per_step) if persistent else None

    # the one-launch-per-step path on the same handle, for comparison
    per_step = None
    if persistent and not args.forward_only:
        t.set_option(tmm.TMM_OPT_PERSISTENT, 0)
        t.year(y, nyears=1, out=ya, residuals=False)
        torch.cuda.synchronize()
        start.record(stream)
        t.year(y, nyears=2, out=ya, residuals=False)
        stop.record(stream)
        torch.cuda.synchronize()
        t.set_option(tmm.TMM_OPT_PERSISTENT, 1)
        ms_ps = start.elapsed_time(stop) / 2
        per_step = {"ms_per_year": ms_ps, "model_years_per_s": 1000.0 / ms_ps}
        log(f"[bench] per-step kernels: {ms_ps:.3f} ms/model-year")

    # adjoint / forward cost ratio (one model year each): the whole year's
    # states stored by the forward sweep (nstep x n x W doubles, 2.4 GB), and
    # checkpoints every 240 steps with recomputation
    ratio = ratio_ckpt = None
    if not args.forward_only:
        obs = torch.as_tensor(np.broadcast_to(inp.initial_state(), (12, n, W)).copy()
                              * (1 + 0.05 * synth.obs_noise((12, n, W), seed=3))).to(dev)
        start.record(stream)
        t.year(y0, nyears=1, out=ya, residuals=False)
        stop.record(stream)
        torch.cuda.synchronize()
        ms_fwd1 = start.elapsed_time(stop)
        ta = tmm.TMM(inp.desc_arrays(), nbatch_max=1, adjoint_nbatch_max=1, ckpt_every=inp.nstep, device=dev,
                     stream=stream)
        autotune.apply_tuned(ta, 1)       # the same launch configuration as the forward years
        ta.set_params(u)
        for h, ck in ((ta, inp.nstep), (t, 240)):
            h.year_adjoint(y0, obs, want_dy0=False)   # warm-up
            torch.cuda.synchronize()
            start.record(stream)
            h.year_adjoint(y0, obs, want_dy0=True)
            stop.record(stream)
            torch.cuda.synchronize()
            ms_adj = start.elapsed_time(stop)
            log(f"[bench] adjoint year (ckpt every {ck} steps) {ms_adj:.2f} ms vs forward {ms_fwd1:.2f} ms: "
                f"ratio {ms_adj / ms_fwd1:.2f}")
            if ck == 240:
                ratio_ckpt = ms_adj / ms_fwd1
            else:
                ratio = ms_adj / ms_fwd1
        ta.close()

    # the same grid with 8 internal BGC steps per ocean step (section 7), and
    # with the three-tracer PO4-DOP-PHY model (section 2.2.2)
    substeps = phy = None
    if not args.forward_only:
        import dataclasses
        substeps = bench_variant(args, dataclasses.replace(inp, nbgc=8), dev, stream, ms_per_year,
                                 "8 internal BGC steps")
        substeps["nbgc"] = 8
        phy = bench_variant(args, synth.global_2p8(model=synth.MODEL_NDOPPHY), dev, stream, ms_per_year,
                            "PO4-DOP-PHY")

    newton = None
    if not args.no_newton and not args.forward_only:
        newton = newton_leg(t, inp, u)

    ensemble = None
    if not args.no_ensemble and not args.forward_only:
        ensemble = ensemble_leg(dev, stream, cpu=not args.no_cpu_baseline)

    cpu = None
    if not args.no_cpu_baseline and not args.forward_only:
        cpu = cpu_baseline(inp, u, B)

    traffic = measured_traffic(kernel) if persistent else None
    out = {
        "metric": "model-years/s + HBM GB/s (N-DOP, 52749 pts); adjoint/forward cost ratio",
        "value": years_per_s,
        "unit": "model-years/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_year,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded 128x64x15 grid and monthly matrices shaped like the paper's 2.8125-degree set)",
        "config": {"workload": "global_128x64x15 N-DOP forward model years", "n": n, "columns": inp.grid.ncol,
                   "layers": 15, "tracers": W, "nstep": inp.nstep, "nnz_explicit": inp.tm.ae_nnz,
                   "nnz_implicit": inp.tm.ai_nnz, "step": "one model year",
                   "path": kernel, "tuned": tuned["named"] if tuned else "library defaults"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "hbm_frac_measured": (traffic / (us_per_launch * 1e-6) / 1e9 / HBM_PEAK_GBPS
                                           if traffic else None),
                     "traffic_note": "traffic = FETCH_SIZE + WRITE_SIZE per launch (bytes past the L2, "
                                     "calibrated on a plain copy) from the committed counter summary of this "
                                     "kernel source; null if the source changed since. The year's working set "
                                     "(state ring 108 MB, 12 monthly matrix pairs) fits the 256 MB Infinity "
                                     "Cache, so these bytes need not all reach HBM: hbm_frac_measured is an "
                                     "upper bound on the HBM share",
                     "kernel": kernel, "us_per_launch": us_per_launch, "bytes_per_launch": B * units,
                     "us_per_time_step": us_per_step,
                     "binding": "latency" if persistent else "hbm",
                     "latency": floor,
                     "note": "algorithmic bytes count the interpolated month pair of Ae and Ai in every step; "
                             "the single-launch kernel keeps both in registers for the whole launch, so frac "
                             "can exceed 1 and is not a bandwidth figure; the step is bound by the chain of "
                             "exchange and barriers, whose measured floor is under latency"},
        "year_stats": year_stats,
        "per_step_path": per_step,
        "adjoint_forward_ratio": ratio,
        "adjoint_forward_ratio_ckpt240": ratio_ckpt,
        "bgc_substeps_8": substeps,
        "po4_dop_phy": phy,
        "newton": newton,
        "ensemble": ensemble,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    t.close()


def bench_variant(args, inp, dev, stream, ms_plain, label):
    """Forward model years and the adjoint of a model variant on the same grid
    (internal BGC steps, or another BGC model), against the headline forward."""
    import torch
    from paper_1410_0204_amd import tmm
    import synth
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1, adjoint_nbatch_max=1, ckpt_every=inp.nstep, device=dev,
                stream=stream)
    from paper_1410_0204_amd import autotune
    autotune.apply_tuned(t, 1)            # this shape's tuned entry, if the table has one
    t.set_params(synth.nominal(inp.model))
    y0 = t.state(inp.initial_state())
    ya = t.state()
    t.year(y0, nyears=1, out=ya, residuals=False)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    years = max(2, min(args.steps, 5))
    start.record(stream)
    t.year(y0, nyears=years, out=ya, residuals=False)
    stop.record(stream)
    torch.cuda.synchronize()
    ms_fwd = start.elapsed_time(stop) / years
    shape = (inp.nmat, inp.n, inp.ntracer)
    obs = torch.as_tensor(np.broadcast_to(inp.initial_state(), shape).copy()
                          * (1 + 0.05 * synth.obs_noise(shape, seed=3))).to(dev)
    t.year_adjoint(y0, obs, want_dy0=False)
    torch.cuda.synchronize()
    start.record(stream)
    t.year_adjoint(y0, obs, want_dy0=True)
    stop.record(stream)
    torch.cuda.synchronize()
    ms_adj = start.elapsed_time(stop)
    rec = {"ms_per_year": ms_fwd, "model_years_per_s": 1000.0 / ms_fwd,
           "cost_vs_headline": ms_fwd / ms_plain, "adjoint_ms": ms_adj, "adjoint_forward_ratio": ms_adj / ms_fwd,
           "forward_path": "k_year_persistent" if t.query(tmm.TMM_Q_PERSISTENT) else "k_step",
           "adjoint_path": "k_adjoint_persistent" if t.query(tmm.TMM_Q_PERSISTENT_ADJOINT) else "k_adjoint",
           "adjoint_ckpt_every": inp.nstep}
    log(f"[bench] {label}: {ms_fwd:.3f} ms/model-year ({ms_fwd / ms_plain:.2f}x), "
        f"adjoint {ms_adj:.2f} ms (ratio {ms_adj / ms_fwd:.2f}, {rec['adjoint_path']})")
    t.close()
    return rec


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def bench_copy(args):
    """512 MiB device-to-device copy: reads and writes 512 MiB each."""
    import torch
    n = 512 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    s, e = _events()
    torch.cuda.synchronize()
    s.record()
    for _ in range(3):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / 3
    print(json.dumps({"mode": "copy", "bytes_read": n * 8, "bytes_written": n * 8, "ms": ms,
                      "GB_per_s": 2 * n * 8 / ms / 1e6}), flush=True)


def bench_grids(args):
    """Launch-per-step model years (graph-replayed k_step, one member, N-DOP) on the
    global 128x64x15, the 256x128x23 and the 1.0-degree 360x180x23 grids: how the
    achieved bandwidth of the step kernel scales with the grid.  On the larger
    grids the month pair of matrices no longer fits the 256 MB Infinity Cache and
    every step streams it from HBM."""
    import torch
    import synth
    from paper_1410_0204_amd import tmm
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    rows = []
    for make in (synth.global_2p8, synth.ensemble_1p4, synth.one_degree):
        inp = make()
        B = bytes_per_step(inp.n, inp.tm.ae_nnz, inp.tm.ai_nnz, inp.ntracer)
        t = tmm.TMM(inp.desc_arrays(), nbatch_max=1, device=dev, stream=stream)
        t.set_option(tmm.TMM_OPT_PERSISTENT, 0)
        t.set_params(synth.nominal(inp.model))
        y0 = t.state(inp.initial_state())
        ya = t.state()
        s, e = _events()
        if args.grid_steps > 0:
            # a few single steps only (hardware-counter passes serialise every launch)
            yb = t.step(0, y0)
            torch.cuda.synchronize()
            s.record(stream)
            for j in range(args.grid_steps):
                yb = t.step(j % inp.nstep, yb)
            e.record(stream)
            torch.cuda.synchronize()
            us_step = s.elapsed_time(e) * 1000.0 / args.grid_steps
            ms = us_step * inp.nstep / 1000.0
            tiles = {"default": (ms, us_step)}
        else:
            # the default tiling (by state width), then every tile size of the kernel
            tiles = {}
            for rows_opt in (0, 32, 64, 128, 256):
                t.set_option(tmm.TMM_OPT_TILE_ROWS, rows_opt)
                t.year(y0, nyears=1, out=ya, residuals=False)
                torch.cuda.synchronize()
                years = 2
                s.record(stream)
                t.year(y0, nyears=years, out=ya, residuals=False)
                e.record(stream)
                torch.cuda.synchronize()
                ms_t = s.elapsed_time(e) / years
                tiles["default" if rows_opt == 0 else f"tile_rows_{rows_opt}"] = (ms_t, ms_t * 1000.0 / inp.nstep)
            ms, us_step = tiles["default"]
        best = min(tiles, key=lambda k: tiles[k][0])
        ms_b, us_b = tiles[best]
        rec = {"workload": inp.name, "n": inp.n, "nnz_explicit": inp.tm.ae_nnz, "nnz_implicit": inp.tm.ai_nnz,
               "bytes_per_step": B, "ms_per_year": ms, "model_years_per_s": 1000.0 / ms, "us_per_step": us_step,
               "GB_per_s": B / (us_step * 1e-6) / 1e9, "frac_of_peak": B / (us_step * 1e-6) / 1e9 / HBM_PEAK_GBPS,
               "best_tiling": best, "best_ms_per_year": ms_b, "best_us_per_step": us_b,
               "best_GB_per_s": B / (us_b * 1e-6) / 1e9, "best_frac_of_peak": B / (us_b * 1e-6) / 1e9 / HBM_PEAK_GBPS,
               "ms_per_year_by_tiling": {k: v[0] for k, v in tiles.items()}}
        log(f"[bench] {inp.name}: {ms:.2f} ms/model-year, {us_step:.1f} us/step, {rec['GB_per_s']:.0f} GB/s "
            f"(default tiling); best {best}: {ms_b:.2f} ms/model-year, {us_b:.1f} us/step, "
            f"{rec['best_GB_per_s']:.0f} GB/s ({100 * rec['best_frac_of_peak']:.0f} % of peak)")
        rows.append(rec)
        t.close()
        del t
        torch.cuda.empty_cache()
    print(json.dumps({"mode": "grids", "kernel": "k_step (graph-replayed, one launch per step)", "rows": rows}),
          flush=True)


def bench_newton(args):
    """Steady periodic solution of the global grid by Newton-Krylov (FD and
    tangent JVPs with the line search, tangent with the trust region, tangent
    with the transport preconditioner), and spin-up for the same number of
    model years."""
    import torch
    import synth
    from paper_1410_0204_amd import drivers, tmm

    inp = synth.global_2p8()
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1)
    u = synth.nominal(inp.model)
    y0 = inp.initial_state()
    out = {"mode": "newton", "workload": "global_128x64x15 N-DOP", "tol": 1e-8, "restart": 30}
    for jvp, glob, pre in (("fd", "line_search", None), ("tangent", "line_search", None),
                           ("tangent", "trust_region", None), ("tangent", "line_search", "transport")):
        key = jvp if glob == "line_search" else f"{jvp}_trust_region"
        key = key if pre is None else f"{key}_preconditioned"
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y, hist = drivers.newton_krylov(t, u, y0, tol=1e-8, jvp=jvp, restart=30, max_newton=args.steps,
                                        max_krylov=300, log_path=args.log, globalization=glob,
                                        preconditioner=pre)
        dt = time.perf_counter() - t0
        out[key] = {"fnorm": hist["fnorm"], "year_maps": hist["years"], "seconds": dt,
                    "newton_iterations": len(hist["newton"]),
                    "krylov_per_newton": [r["krylov"] for r in hist["newton"]]}
        log(f"[newton/{key}] |F| {hist['fnorm'][0]:.3e} -> {hist['fnorm'][-1]:.3e} in {len(hist['newton'])} "
            f"Newton steps, {hist['years']} year maps, {dt:.1f} s")
    years = out["fd"]["year_maps"]
    t0 = time.perf_counter()
    _, r = drivers.spinup(t, u, y0, years=years, log_path=args.log)
    out["spinup"] = {"years": years, "residual_first": float(r[0]), "residual_last": float(r[-1]),
                     "seconds": time.perf_counter() - t0}
    log(f"[spin-up] {years} years: residual {r[0]:.3e} -> {r[-1]:.3e}")
    print(json.dumps(out), flush=True)


def bench_ensemble(args):
    """64 members with uneven spin-up lengths in one batched state (W = 128)
    against one-member runs of the same grid."""
    import torch
    import synth
    from paper_1410_0204_amd import tmm

    t0 = time.perf_counter()
    inp = synth.ensemble_1p4()
    log(f"[ensemble] inputs {inp.name}: n={inp.n} ncol={inp.grid.ncol} nnz_e={inp.tm.ae_nnz} "
        f"nnz_i={inp.tm.ai_nnz} ({time.perf_counter() - t0:.1f} s to generate)")
    nm = 64
    U = synth.latin_hypercube(synth.MODEL_NDOP, nm, seed=17)
    L = synth.spinup_lengths(nm, seed=18)
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=nm)
    from paper_1410_0204_amd import autotune
    tuned = autotune.apply_tuned(t, nm)     # the options below override it
    log(f"[ensemble] launch configuration: {tuned['named'] if tuned else 'library defaults'}")
    if args.member_band is not None:
        t.set_option(tmm.TMM_OPT_MEMBER_BAND_ROWS, args.member_band)
    if args.member_waves is not None:
        t.set_option(tmm.TMM_OPT_MEMBER_WAVES, args.member_waves)
    if args.member_tile is not None:
        t.set_option(tmm.TMM_OPT_MEMBER_TILE, args.member_tile)
    s, e = _events()
    t.set_params(U)
    y0 = t.state(inp.initial_state(nm))
    # warm-up: one step at full width
    t.step(0, y0)
    torch.cuda.synchronize()
    W = 2 * nm
    B = bytes_per_step(inp.n, inp.tm.ae_nnz, inp.tm.ai_nnz, W)
    if args.grid_steps > 0:
        # full-width steps only (for hardware-counter passes, which serialise every launch)
        yb = y0
        s.record()
        for j in range(args.grid_steps):
            yb = t.step(j % inp.nstep, yb)
        e.record()
        torch.cuda.synchronize()
        us = s.elapsed_time(e) * 1000.0 / args.grid_steps
        log(f"[ensemble] {args.grid_steps} full-width steps: {us:.1f} us/step, {B / (us * 1e-6) / 1e9:.0f} GB/s")
        print(json.dumps({"mode": "ensemble_steps", "us_per_step": us, "bytes_per_step": B,
                          "GB_per_s": B / (us * 1e-6) / 1e9}), flush=True)
        return
    s.record()
    out_b, _ = t.year(y0, nyears=int(L.max()), years_per_member=L, residuals=False)
    e.record()
    torch.cuda.synchronize()
    ms_b = s.elapsed_time(e)
    member_years = int(L.sum())
    # one-member runs: time one model year of member 0 in its own tuned
    # configuration, extrapolate to all member-years
    autotune.apply(t, autotune.DEFAULTS)
    autotune.apply_tuned(t, 1)
    t.set_params(U[0])
    y1 = t.state(inp.initial_state(1))
    t.year(y1, nyears=1, residuals=False)
    torch.cuda.synchronize()
    s.record()
    t.year(y1, nyears=1, residuals=False)
    e.record()
    torch.cuda.synchronize()
    ms_1 = s.elapsed_time(e)
    res = {"mode": "ensemble", "workload": "ensemble_256x128x23 N-DOP", "n": inp.n, "members": nm,
           "member_years": member_years, "batched_ms": ms_b,
           "batched_member_years_per_s": member_years / (ms_b / 1000.0),
           "one_member_ms_per_year": ms_1,
           "sequential_member_years_per_s_extrapolated": 1000.0 / ms_1,
           "speedup": (member_years * ms_1) / ms_b,
           "full_width_bytes_per_step": B}
    log(f"[ensemble] batched: {member_years} member-years in {ms_b:.0f} ms "
        f"({res['batched_member_years_per_s']:.2f}/s); one member {ms_1:.1f} ms/year; "
        f"speedup {res['speedup']:.1f}x")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
