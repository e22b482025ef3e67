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
