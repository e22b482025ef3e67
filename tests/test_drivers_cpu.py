"""Host-driver logic on the CPU: GMRES, Eisenstat-Walker Newton, spin-up.

The drivers only call the handle's year / year_jvp / state methods, so here
they run against a stand-in handle whose model years come from the oracle.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1410_0204_amd import drivers
from paper_1410_0204_amd import tmm as T


class OracleHandle:
    """Minimal stand-in with the TMM methods the drivers use."""

    def __init__(self, inp):
        self.o = oracle.Oracle(inp)
        self.n, self.nstep, self.nmat, self.model = inp.n, inp.nstep, inp.nmat, inp.model
        self.ntracer = inp.ntracer
        self.nbatch = 0
        self._keep = {k: v for k, v in inp.desc_arrays().items() if isinstance(v, np.ndarray)}
        self.years = 0

    @property
    def W(self):
        return self.nbatch * self.ntracer

    def set_params(self, u):
        self.u = np.atleast_2d(u)
        self.nbatch = self.u.shape[0]

    def state(self, host=None):
        return torch.as_tensor(np.array(host, dtype=np.float64)) if host is not None else \
            torch.zeros((self.n, self.W), dtype=torch.float64)

    def year(self, y, nyears=1, years_per_member=None, out=None, residuals=True):
        self.years += nyears
        y1, r = self.o.year(self.u, y.numpy(), nyears)
        out = self.state() if out is None else out
        out.copy_(torch.as_tensor(y1))
        return out, (r if residuals else None)

    def year_jvp(self, y, v, mode=T.TMM_JVP_TANGENT, want_phi=True, phi=None):
        if mode == T.TMM_JVP_TANGENT:
            p, jv = self.o.year_tangent(self.u, y.numpy(), v.numpy())
            return torch.as_tensor(p), torch.as_tensor(jv)
        p, jv = self.o.year_jvp_fd(self.u, y.numpy(), v.numpy())
        return torch.as_tensor(p), torch.as_tensor(jv)


def test_gmres_nonsymmetric_and_restarted():
    rng = np.random.default_rng(0)
    n = 120
    A = np.eye(n) + 0.5 * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    for restart in (5, 30):
        x, r, its = drivers.gmres(lambda v: A @ v, b, 1e-10, restart=restart, maxiter=2000)
        assert np.linalg.norm(A @ x - b) <= 1.01e-10 * np.linalg.norm(b)
        assert np.allclose(r, b - A @ x)


def test_gmres_singular_consistent_system():
    """I - P with P column-stochastic-like (mass conserving): consistent rhs is solvable."""
    rng = np.random.default_rng(1)
    n = 60
    P = rng.uniform(size=(n, n))
    P /= P.sum(1, keepdims=True)              # row-stochastic: (I - P) 1 = 0
    A = np.eye(n) - P
    x0 = rng.standard_normal(n)
    b = A @ x0                                 # in the range
    x, r, _ = drivers.gmres(lambda v: A @ v, b, 1e-10, restart=30, maxiter=500)
    assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)


@pytest.mark.parametrize("jvp", ["tangent", "fd"])
def test_newton_krylov_reaches_fixed_point(tiny_ndop, jvp):
    h = OracleHandle(tiny_ndop)
    u = synth.nominal(synth.MODEL_NDOP)
    y0 = tiny_ndop.initial_state()
    y, hist = drivers.newton_krylov(h, u, y0, tol=1e-8, jvp=jvp, restart=30, max_newton=12, max_krylov=200)
    h.set_params(u)
    phi, _ = h.o.year(u, y)
    assert np.linalg.norm(y - phi) <= 1e-8
    V = tiny_ndop.grid.volumes()
    # phi conserves mass, so exact Newton updates keep the mass of y0; finite-
    # difference products (~1e-6 relative error) let a little leak into the update
    assert (V @ y.sum(1)) == pytest.approx(V @ y0.sum(1), rel=1e-10 if jvp == "tangent" else 1e-6)
    assert hist["fnorm"][-1] <= 1e-8 and hist["years"] > 0


class AtanHandle:
    """Toy year map phi(y) = y - atan(y - c) on one 'point', so F(y) = atan(y - c): full Newton
    steps diverge from |y - c| >= 1.39 (the textbook example), a globalised Newton converges."""

    n, nstep, nmat, model, ntracer = 3, 1, 1, 1, 1

    def __init__(self, c):
        self.c = np.asarray(c, dtype=np.float64).reshape(3, 1)
        self.nbatch = 1

    @property
    def W(self):
        return 1

    def set_params(self, u):
        pass

    def state(self, host=None):
        return torch.as_tensor(np.array(host, dtype=np.float64)) if host is not None else \
            torch.zeros((3, 1), dtype=torch.float64)

    def year(self, y, nyears=1, years_per_member=None, out=None, residuals=True):
        yy = y.numpy()
        out.copy_(torch.as_tensor(yy - np.arctan(yy - self.c)))
        return out, None

    def year_jvp(self, y, v, mode=T.TMM_JVP_TANGENT, want_phi=True, phi=None):
        yy, vv = y.numpy(), v.numpy()
        return None, torch.as_tensor(vv - vv / (1.0 + (yy - self.c) ** 2))


def test_trust_region_converges_where_full_newton_steps_diverge():
    c = [0.5, -1.0, 2.0]
    y0 = np.array(c).reshape(3, 1) + 3.0
    h = AtanHandle(c)
    y, hist = drivers.newton_krylov(h, [0.0], y0, tol=1e-12, jvp="tangent", max_newton=40,
                                    globalization="trust_region", delta0=0.5)
    assert np.abs(y.ravel() - np.array(c)).max() <= 1e-12
    assert any(rec["tau"] < 1.0 for rec in hist["newton"])          # the radius was active
    _, full = drivers.newton_krylov(h, [0.0], y0, tol=1e-12, jvp="tangent", max_newton=3, line_search=False)
    assert full["fnorm"][-1] > full["fnorm"][0]                     # undamped Newton moves away


@pytest.mark.parametrize("delta0", [0.2, 1e-4])
def test_trust_region_newton_reaches_the_same_fixed_point(tiny_ndop, delta0):
    h = OracleHandle(tiny_ndop)
    u = synth.nominal(synth.MODEL_NDOP)
    y0 = tiny_ndop.initial_state()
    y, hist = drivers.newton_krylov(h, u, y0, tol=1e-8, jvp="tangent", max_newton=30, max_krylov=200,
                                    globalization="trust_region", delta0=delta0)
    assert hist["fnorm"][-1] <= 1e-8
    y_ls, _ = drivers.newton_krylov(h, u, y0, tol=1e-8, jvp="tangent", max_newton=12, max_krylov=200)
    assert np.abs(y - y_ls).max() <= 1e-7 * np.abs(y_ls).max()
    if delta0 < 1e-3:
        assert hist["newton"][0]["tau"] < 1.0


def test_transport_preconditioner_reaches_the_same_fixed_point_with_fewer_krylov_iterations(tiny_ndop):
    h = OracleHandle(tiny_ndop)
    u = synth.nominal(synth.MODEL_NDOP)
    y0 = tiny_ndop.initial_state()
    y, hist = drivers.newton_krylov(h, u, y0, tol=1e-8, jvp="tangent", max_newton=20, max_krylov=200,
                                    preconditioner="transport")
    y_plain, plain = drivers.newton_krylov(h, u, y0, tol=1e-8, jvp="tangent", max_newton=20, max_krylov=200)
    assert hist["fnorm"][-1] <= 1e-8
    assert np.abs(y - y_plain).max() <= 1e-7 * np.abs(y_plain).max()
    krylov = sum(r["krylov"] for r in hist["newton"])
    assert krylov < sum(r["krylov"] for r in plain["newton"])
    assert hist["years"] < plain["years"]


def test_transport_preconditioner_inverts_pure_vertical_mixing():
    """With no horizontal exchange (Ae = I) a water column's year map of a passive tracer is
    exp(T L) restricted to the column; for the slowest nonzero mode the preconditioned operator
    (1 - e^x)(-1/x + 1/2) stays within [1/2, 1]."""
    import copy
    inp = copy.deepcopy(synth.tiny(model=synth.MODEL_N))
    tm = inp.tm
    rows = np.repeat(np.arange(inp.n), np.diff(tm.ae_rowptr))
    tm.ae_val = np.broadcast_to(np.where(rows == tm.ae_colidx, 1.0, 0.0), tm.ae_val.shape).copy()
    h = OracleHandle(inp)
    u = synth.nominal(synth.MODEL_N)
    u[0] = 0.0                                   # passive tracer
    h.set_params(u)
    apply = drivers.transport_preconditioner(h, u)
    rng = np.random.default_rng(3)
    for _ in range(3):
        v = rng.standard_normal((inp.n, 1))
        v -= v.mean()
        jv = v - h.o.year_tangent(u, np.ones((inp.n, 1)), v)[1]      # (I - phi') v
        pv = apply(jv.ravel()).reshape(inp.n, 1)
        ratio = float(np.dot(pv.ravel(), v.ravel()) / np.dot(v.ravel(), v.ravel()))
        assert 0.3 < ratio < 1.2, ratio


def test_spinup_residual_decreases_and_resumes(tiny_ndop, tmp_path):
    h = OracleHandle(tiny_ndop)
    u = synth.nominal(synth.MODEL_NDOP)
    y0 = tiny_ndop.initial_state()
    path = str(tmp_path / "state.npz")
    log = str(tmp_path / "log.jsonl")
    y3, r3 = drivers.spinup(h, u, y0, years=3, log_path=log, state_path=path, state_every=1)
    assert r3[2] < r3[0]
    y5a, r5a = drivers.spinup(h, u, y0, years=5, state_path=path, state_every=1, resume=True)
    y5b, r5b = drivers.spinup(h, u, y0, years=5)
    assert np.array_equal(y5a, y5b)            # resume from year 3 reproduces bitwise
    assert np.array_equal(r5a, r5b)
    assert len(open(log).read().splitlines()) == 3


def test_spinup_logs_mass_and_its_drift(tiny_ndop, tmp_path):
    """Each spin-up year logs every tracer's volume-weighted mass and the drift of the total: the
    transport conserves mass and the model only moves phosphorus between tracers (section 2.2.1)."""
    import json
    h = OracleHandle(tiny_ndop)
    u = synth.nominal(synth.MODEL_NDOP)
    y0 = tiny_ndop.initial_state()
    log = str(tmp_path / "log.jsonl")
    y, r, mass = drivers.spinup(h, u, y0, years=3, log_path=log, return_mass=True)
    V = tiny_ndop.grid.volumes()
    assert mass.shape == (4, 1, 2)
    assert np.allclose(mass[0, 0], V @ y0, rtol=1e-15, atol=0)
    assert np.allclose(mass[-1, 0], V @ y, rtol=1e-15, atol=0)
    assert mass[-1, 0, 1] > mass[0, 0, 1]          # DOP is produced from PO4 ...
    recs = [json.loads(x) for x in open(log).read().splitlines()]
    assert [rec["year"] for rec in recs] == [1, 2, 3]
    for rec in recs:
        assert abs(rec["mass_drift"][0]) <= 1e-13   # ... and the total is kept
        assert np.allclose(np.sum(rec["mass"]), V @ y0.sum(1), rtol=1e-13)


def test_newton_fixed_point_is_the_spinup_limit(tiny_ndop):
    """The periodic solution (section 4) found by Newton-Krylov (section 6) is where spin-up goes.

    Fixed points form a family indexed by total mass, and both methods keep the
    mass of y0, so they must meet.  Spin-up contracts slowly (about 4 % a year
    on this grid), so 120 years are not enough to get there; instead the error
    e_k = y_k - y* against the Newton solution y* must (i) fall by orders of
    magnitude and (ii) end within the contraction bound |e_K| <= r_K / (1 - rho)
    set by the spin-up's own last residual r_K and rate rho: a limit other than
    y* would leave e_k at a nonzero constant."""
    h = OracleHandle(tiny_ndop)
    u = synth.nominal(synth.MODEL_NDOP)
    y0 = tiny_ndop.initial_state()
    ystar, hist = drivers.newton_krylov(h, u, y0, tol=1e-10, jvp="tangent", max_newton=15, max_krylov=300)
    assert hist["fnorm"][-1] <= 1e-10
    V = tiny_ndop.grid.volumes()
    # GMRES leaves rounding (about 1e-12 relative) in the mass of each Newton update
    assert V @ ystar.sum(1) == pytest.approx(V @ y0.sum(1), rel=1e-11)
    K = 120
    h.set_params(u)
    errs, y = [], y0.copy()
    resid = []
    for k in range(K):
        y, r = h.o.year(u, y)
        resid.append(r[0, 0])
        errs.append(np.linalg.norm(y - ystar))
    rho = (resid[-1] / resid[-21]) ** (1 / 20)
    assert 0.5 < rho < 1.0
    bound = resid[-1] * rho / (1.0 - rho)            # |y_K - y*| for a linear contraction, |phi(y_K) - y_K| = r_K
    assert errs[-1] <= 0.02 * errs[K // 4]
    assert errs[-1] <= 1.5 * bound + 1e-9
    assert V @ y.sum(1) == pytest.approx(V @ ystar.sum(1), rel=1e-11)
