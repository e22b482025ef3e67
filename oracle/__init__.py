"""ctypes front end of the reference CPU implementation (``tmm_oracle.c``).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
CPU-baseline leg of the benchmark to check the GPU library.  The GPU library
never imports it.
"""

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TMM_ORACLE_LIB", os.path.join(HERE, "liboracle.so"))

MODEL_N = 1
MODEL_NDOP = 2
MODEL_NDOPPHY = 3
_NTRACER = {MODEL_N: 1, MODEL_NDOP: 2, MODEL_NDOPPHY: 3}
_NPARAM = {MODEL_N: 5, MODEL_NDOP: 7, MODEL_NDOPPHY: 11}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _Desc(C.Structure):
    _fields_ = [
        ("n", C.c_int), ("ncol", C.c_int), ("nlayer", C.c_int),
        ("col_start", _ip), ("lat", _dp), ("area", _dp), ("dz", _dp),
        ("nmat", C.c_int), ("nstep", C.c_int), ("model", C.c_int), ("neuphotic", C.c_int),
        ("ae_nnz", C.c_int), ("ae_rowptr", _ip), ("ae_colidx", _ip), ("ae_val", _dp),
        ("ai_nnz", C.c_int), ("ai_rowptr", _ip), ("ai_colidx", _ip), ("ai_val", _dp),
        ("nbgc", C.c_int),
    ]


_libs = {}


def load(path=None):
    """The oracle library at ``path`` (default: the plain build, built on first use)."""
    path = LIB_PATH if path is None else path
    if path not in _libs:
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        lib = C.CDLL(path)
        sig = {
            "oracle_threads": (C.c_int, [C.c_int]),
            "oracle_ntracer": (C.c_int, [C.c_int]),
            "oracle_nparam": (C.c_int, [C.c_int]),
            "oracle_phase": (None, [C.c_int, C.c_int, C.c_int, _ip, _ip, _dp]),
            "oracle_insolation": (C.c_double, [C.c_double, C.c_double]),
            "oracle_spmm_interp": (None, [C.c_int, _ip, _ip, _dp, _dp, C.c_double, C.c_int, _dp, _dp]),
            "oracle_bgc_column": (C.c_int, [C.c_int, C.c_double, C.c_int, _dp, _dp, _dp, _dp, C.c_int]),
            "oracle_bgc_source": (C.c_int, [C.c_int, C.c_double, C.c_int, _dp, _dp, _dp, _dp, C.c_int,
                                            C.c_double, C.c_int]),
            "oracle_step": (C.c_int, [C.POINTER(_Desc), C.c_int, _dp, C.c_int, _dp, _dp]),
            "oracle_year": (C.c_int, [C.POINTER(_Desc), C.c_int, _dp, C.c_int, _dp, _dp, _dp]),
            "oracle_year_tangent": (C.c_int, [C.POINTER(_Desc), C.c_int, _dp, _dp, _dp, _dp, _dp]),
            "oracle_year_jvp_fd": (C.c_int, [C.POINTER(_Desc), C.c_int, _dp, _dp, _dp, _dp, _dp]),
            "oracle_year_misfit": (C.c_int, [C.POINTER(_Desc), C.c_int, _dp, _dp, _dp, _dp]),
            "oracle_year_adjoint": (C.c_int, [C.POINTER(_Desc), C.c_int, _dp, _dp, _dp, _dp, _dp, _dp]),
            "oracle_year_vjp": (C.c_int, [C.POINTER(_Desc), C.c_int, _dp, _dp, _dp, _dp, _dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _libs[path] = lib
    return _libs[path]


def threads(n=0, lib_path=None):
    """Sets (n >= 1) and returns the thread count of a library's step loops."""
    return int(load(lib_path).oracle_threads(int(n)))


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def phase(j, nstep=2880, nmat=12):
    k0, k1, w = C.c_int(), C.c_int(), C.c_double()
    load().oracle_phase(j, nstep, nmat, C.byref(k0), C.byref(k1), C.byref(w))
    return k0.value, k1.value, w.value


def insolation(lat_deg, t):
    return load().oracle_insolation(float(lat_deg), float(t))


def spmm_interp(rowptr, colidx, v0, v1, w, x):
    x = _f64(x)
    n = rowptr.size - 1
    W = x.shape[1]
    y = np.zeros((n, W))
    load().oracle_spmm_interp(n, _i(np.ascontiguousarray(rowptr, dtype=np.int32)),
                              _i(np.ascontiguousarray(colidx, dtype=np.int32)),
                              _d(_f64(v0)), _d(_f64(v1)), float(w), W, _d(x), _d(y))
    return y


def bgc_column(model, insol, h, y, u, neuphotic):
    """q for one column; y is [ntracer, nlayer] (tracer-major)."""
    y = _f64(y)
    q = np.zeros_like(y)
    h = _f64(h)
    rc = load().oracle_bgc_column(model, float(insol), y.shape[1], _d(h), _d(y), _d(q), _d(_f64(u)),
                                  neuphotic)
    if rc:
        raise ValueError("oracle_bgc_column failed")
    return q


def bgc_source(model, insol, h, y, u, neuphotic, dt, nsub):
    """Source of one ocean step for one column with nsub internal BGC steps; y is [ntracer, nlayer]."""
    y = _f64(y)
    inc = np.zeros_like(y)
    rc = load().oracle_bgc_source(model, float(insol), y.shape[1], _d(_f64(h)), _d(y), _d(inc), _d(_f64(u)),
                                  neuphotic, float(dt), int(nsub))
    if rc:
        raise ValueError("oracle_bgc_source failed")
    return inc


class Oracle:
    """Reference implementation bound to one set of inputs (a ``synth.Inputs``)."""

    def __init__(self, inputs, nstep=None, model=None, neuphotic=None, nbgc=None, lib_path=None):
        a = inputs.desc_arrays()
        self._keep = {k: v for k, v in a.items() if isinstance(v, np.ndarray)}
        self.n = a["n"]
        self.model = model if model is not None else a["model"]
        self.ntracer = _NTRACER[self.model]
        self.nparam = _NPARAM[self.model]
        self.nstep = nstep if nstep is not None else a["nstep"]
        self.nmat = a["nmat"]
        k = self._keep
        self.desc = _Desc(
            a["n"], a["ncol"], a["nlayer"], _i(k["col_start"]), _d(k["lat"]), _d(k["area"]), _d(k["dz"]),
            a["nmat"], self.nstep, self.model, neuphotic if neuphotic is not None else a["neuphotic"],
            k["ae_colidx"].size, _i(k["ae_rowptr"]), _i(k["ae_colidx"]), _d(k["ae_val"]),
            k["ai_colidx"].size, _i(k["ai_rowptr"]), _i(k["ai_colidx"]), _d(k["ai_val"]),
            int(nbgc if nbgc is not None else a.get("nbgc", 1)),
        )
        self.nbgc = int(self.desc.nbgc)
        self.lib = load(lib_path)

    def _u(self, u):
        u = np.atleast_2d(_f64(u))
        if u.shape[1] != self.nparam:
            raise ValueError("parameter vector length")
        return np.ascontiguousarray(u), u.shape[0]

    def _check(self, rc, what):
        if rc:
            raise RuntimeError(f"{what} failed with {rc}")

    def step(self, u, j, y):
        u, nb = self._u(u)
        y = _f64(y)
        out = np.empty_like(y)
        self._check(self.lib.oracle_step(C.byref(self.desc), nb, _d(u), j, _d(y), _d(out)), "step")
        return out

    def year(self, u, y, nyears=1):
        u, nb = self._u(u)
        y = _f64(y)
        out = np.empty_like(y)
        resid = np.empty((nyears, nb))
        self._check(self.lib.oracle_year(C.byref(self.desc), nb, _d(u), nyears, _d(y), _d(out), _d(resid)),
                    "year")
        return out, resid

    def year_tangent(self, u, y, v):
        u, nb = self._u(u)
        y, v = _f64(y), _f64(v)
        phi, jv = np.empty_like(y), np.empty_like(y)
        self._check(self.lib.oracle_year_tangent(C.byref(self.desc), nb, _d(u), _d(y), _d(v), _d(phi), _d(jv)),
                    "tangent")
        return phi, jv

    def year_jvp_fd(self, u, y, v):
        u, nb = self._u(u)
        y, v = _f64(y), _f64(v)
        phi, jv = np.empty_like(y), np.empty_like(y)
        self._check(self.lib.oracle_year_jvp_fd(C.byref(self.desc), nb, _d(u), _d(y), _d(v), _d(phi), _d(jv)),
                    "jvp_fd")
        return phi, jv

    def year_misfit(self, u, y0, obs):
        u, nb = self._u(u)
        J = np.empty(nb)
        self._check(self.lib.oracle_year_misfit(C.byref(self.desc), nb, _d(u), _d(_f64(y0)), _d(_f64(obs)),
                                                _d(J)), "misfit")
        return J

    def year_adjoint(self, u, y0, obs):
        u, nb = self._u(u)
        y0 = _f64(y0)
        J = np.empty(nb)
        dJdu = np.empty((nb, self.nparam))
        dJdy0 = np.empty_like(y0)
        self._check(self.lib.oracle_year_adjoint(C.byref(self.desc), nb, _d(u), _d(y0), _d(_f64(obs)),
                                                 _d(J), _d(dJdu), _d(dJdy0)), "adjoint")
        return J, dJdu, dJdy0

    def year_vjp(self, u, y0, wbar):
        u, nb = self._u(u)
        y0 = _f64(y0)
        ybar = np.empty_like(y0)
        ubar = np.empty((nb, self.nparam))
        self._check(self.lib.oracle_year_vjp(C.byref(self.desc), nb, _d(u), _d(y0), _d(_f64(wbar)),
                                             _d(ybar), _d(ubar)), "vjp")
        return ybar, ubar

    def snapshots(self, u, y0):
        """States after each month-end step (m+1)*nstep/nmat: [nmat, n, W]."""
        u2, _ = self._u(u)
        y = _f64(y0)
        spm = self.nstep // self.nmat
        out = []
        for j in range(self.nstep):
            y = self.step(u2, j, y)
            if (j + 1) % spm == 0:
                out.append(y.copy())
        return np.stack(out)
