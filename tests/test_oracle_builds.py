"""The other builds of the reference implementation (CPU only).

* The CPU-baseline timing build (-O3 -march=native -fopenmp) must give the
  plain build's results bit for bit, at any thread count: its parallel loops
  leave every element's summation order alone.
* The sanitizer build (AddressSanitizer + UndefinedBehaviorSanitizer, a
  stand-alone program) runs every entry point on the tiny grids without a
  report, and its results equal the plain build's.
"""

import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from oracle import build as obuild


@pytest.fixture(scope="module")
def timing_lib(tmp_path_factory):
    return obuild.build_timing(str(tmp_path_factory.mktemp("omp") / "liboracle_timing.so"))


@pytest.mark.parametrize("nthreads", [1, 3, 8])
def test_timing_build_is_bitwise_the_plain_build(timing_lib, small_ndop, tiny_ndop, nthreads):
    assert oracle.threads(nthreads, timing_lib) == nthreads
    assert oracle.threads(0) == 1                     # the plain build has no threads
    U = synth.latin_hypercube(synth.MODEL_NDOP, 3, seed=4)
    rng = np.random.default_rng(nthreads)
    y = small_ndop.initial_state(3) * rng.uniform(0.7, 1.3, size=(small_ndop.n, 6))
    plain, fast = oracle.Oracle(small_ndop), oracle.Oracle(small_ndop, lib_path=timing_lib)
    for j in (0, 119, 1439, 2879):
        assert np.array_equal(plain.step(U, j, y), fast.step(U, j, y)), j
    u = synth.nominal(synth.MODEL_NDOP)
    y0 = tiny_ndop.initial_state()
    a, ra = oracle.Oracle(tiny_ndop).year(u, y0)
    b, rb = oracle.Oracle(tiny_ndop, lib_path=timing_lib).year(u, y0)
    assert np.array_equal(a, b) and np.array_equal(ra, rb)


def _write_inputs(path, inp, U, y0, v, wbar, obs):
    a = inp.desc_arrays()
    U = np.atleast_2d(U)
    hdr = np.array([a["n"], a["ncol"], a["nlayer"], a["nmat"], a["nstep"], a["model"], a["neuphotic"],
                    a.get("nbgc", 1), a["ae_colidx"].size, a["ai_colidx"].size, U.shape[0]], dtype=np.int32)
    with open(path, "wb") as f:
        for x in (hdr, a["col_start"].astype(np.int32), a["lat"], a["area"], a["dz"],
                  a["ae_rowptr"].astype(np.int32), a["ae_colidx"].astype(np.int32), a["ae_val"],
                  a["ai_rowptr"].astype(np.int32), a["ai_colidx"].astype(np.int32), a["ai_val"],
                  U, y0, v, wbar, obs):
            f.write(np.ascontiguousarray(x).tobytes())


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    return obuild.build_sanitized(str(tmp_path_factory.mktemp("san") / "oracle_sanitized"))


@pytest.mark.parametrize("case", ["n", "ndop_batch", "phy", "ndop_nbgc8"])
def test_sanitizer_build_runs_clean(sanitized, tmp_path, case):
    model = {"n": synth.MODEL_N, "phy": synth.MODEL_NDOPPHY}.get(case, synth.MODEL_NDOP)
    inp = synth.tiny(model=model)
    if case == "ndop_nbgc8":
        inp.nbgc = 8
    nb = 2 if case == "ndop_batch" else 1
    U = synth.nominal(model)[None, :] if nb == 1 else synth.latin_hypercube(model, nb, seed=8)
    rng = np.random.default_rng(3)
    y0 = inp.initial_state(nb) * rng.uniform(0.8, 1.2, size=(inp.n, inp.ntracer * nb))
    v = rng.standard_normal(y0.shape) * y0
    wbar = rng.standard_normal(y0.shape)
    o = oracle.Oracle(inp)
    snaps = o.snapshots(U, y0)
    obs = snaps * (1 + 0.05 * synth.obs_noise(snaps.shape, seed=5))
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write_inputs(fin, inp, U, y0, v, wbar, obs)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([sanitized, fin, fout], env=env, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "ERROR" not in res.stderr and "runtime error" not in res.stderr, res.stderr[-4000:]
    got = np.fromfile(fout, dtype=np.float64)
    nbp = nb * inp.nparam
    expect = [o.step(U, 0, y0), o.step(U, inp.nstep // 2, y0)]
    yr, r = o.year(U, y0)
    expect += [yr, r[0]]
    expect += list(o.year_tangent(U, y0, v)) + list(o.year_jvp_fd(U, y0, v))
    expect.append(o.year_misfit(U, y0, obs))
    J, G, dY = o.year_adjoint(U, y0, obs)
    expect += [J, G, dY]
    expect += list(o.year_vjp(U, y0, wbar))
    flat = np.concatenate([np.ravel(x) for x in expect])
    assert got.size == flat.size == 9 * y0.size + 3 * nb + 2 * nbp
    assert np.array_equal(got, flat)
