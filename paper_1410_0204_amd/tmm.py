"""Python binding of libtmm (include/tmm.h): argument marshalling only.

Every computation runs in the HIP library; PyTorch provides the device memory
(the workspace and the state tensors) and the stream.  The functions named
like the C entry points (``tmm_create``, ``tmm_step``, ...) are thin ctypes
wrappers; :class:`TMM` bundles a handle with its workspace.
"""

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtmm.so")

TMM_OK = 0
TMM_EINVAL = -1
TMM_ENOMEM = -2
TMM_EDEVICE = -3
TMM_ESTATE = -4
TMM_ENONFINITE = -5
TMM_EUNSUPPORTED = -6
TMM_ETOOBIG = -7
TMM_MODEL_N = 1
TMM_MODEL_NDOP = 2
TMM_MODEL_NDOPPHY = 3
_NTRACER = {TMM_MODEL_N: 1, TMM_MODEL_NDOP: 2, TMM_MODEL_NDOPPHY: 3}
_NPARAM = {TMM_MODEL_N: 5, TMM_MODEL_NDOP: 7, TMM_MODEL_NDOPPHY: 11}
TMM_JVP_FD = 0
TMM_JVP_TANGENT = 1
TMM_JVP_FD_GIVEN_PHI = 2
TMM_OPT_PERSISTENT = 1
TMM_OPT_DOMAIN_ROWS = 2
TMM_OPT_MEMBER_KERNEL_MIN = 3
TMM_OPT_GRAPH = 4
TMM_OPT_SPIN_LIMIT = 5
TMM_OPT_CHECK_FINITE = 6
TMM_OPT_MEMBER_WAVES = 7
TMM_OPT_MEMBER_BAND_ROWS = 8
TMM_OPT_TILE_ROWS = 9
TMM_OPT_WAVE_LOCAL = 10
TMM_OPT_MEMBER_TILE = 11
TMM_OPT_MEMBER_PACK = 12
TMM_Q_PERSISTENT = 1
TMM_Q_DOMAINS = 2
TMM_Q_WORKSPACE = 3
TMM_Q_COMPUTE_UNITS = 4
TMM_Q_PERSISTENT_ADJOINT = 5
TMM_Q_INSOLATION_LDS = 6
TMM_Q_WAVE_LOCAL = 7

EXPORTED = (
    "tmm_workspace_bytes", "tmm_create", "tmm_destroy", "tmm_set_params", "tmm_step", "tmm_year",
    "tmm_year_jvp", "tmm_year_adjoint", "tmm_set_option", "tmm_query", "tmm_strerror", "tmm_probe_exchange",
    "tmm_year_noalloc",
)

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class TmmDesc(C.Structure):
    """Mirror of ``tmm_desc``."""

    _fields_ = [
        ("n", C.c_int), ("ncol", C.c_int), ("nlayer", C.c_int),
        ("col_start", _ip), ("lat", _dp), ("area", _dp), ("dz", _dp),
        ("nmat", C.c_int), ("nstep", C.c_int), ("model", C.c_int), ("neuphotic", C.c_int), ("nbgc", C.c_int),
        ("nbatch_max", C.c_int), ("adjoint_nbatch_max", C.c_int), ("ckpt_every", C.c_int),
        ("ae_nnz", C.c_int), ("ae_rowptr", _ip), ("ae_colidx", _ip), ("ae_val", _dp),
        ("ai_nnz", C.c_int), ("ai_rowptr", _ip), ("ai_colidx", _ip), ("ai_val", _dp),
        ("lon", _dp),
    ]


class TmmError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {tmm_strerror(status)} ({status})")
        self.status = status


_lib = None


def load():
    """Loads libtmm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libtmm.so not built at {LIB_PATH}; run __graft_entry__.build()")
        lib = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        sig = {
            "tmm_workspace_bytes": (C.c_int, [C.POINTER(TmmDesc), C.POINTER(C.c_size_t)]),
            "tmm_create": (C.c_int, [C.POINTER(TmmDesc), vp, C.c_size_t, vp, C.POINTER(vp)]),
            "tmm_destroy": (C.c_int, [vp]),
            "tmm_set_params": (C.c_int, [vp, C.c_int, _dp]),
            "tmm_step": (C.c_int, [vp, C.c_int, vp, vp]),
            "tmm_year": (C.c_int, [vp, C.c_int, _ip, vp, vp, _dp]),
            "tmm_year_jvp": (C.c_int, [vp, C.c_int, vp, vp, vp, vp]),
            "tmm_year_adjoint": (C.c_int, [vp, vp, vp, C.c_int, _dp, _dp, vp]),
            "tmm_set_option": (C.c_int, [vp, C.c_int, C.c_int]),
            "tmm_query": (C.c_int, [vp, C.c_int, C.POINTER(C.c_longlong)]),
            "tmm_strerror": (C.c_char_p, [C.c_int]),
            "tmm_probe_exchange": (C.c_int, [vp, C.c_int, _dp]),
            "tmm_year_noalloc": (C.c_int, [vp, C.c_int, vp, vp, _dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(rc, what):
    if rc != TMM_OK:
        raise TmmError(rc, what)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _host_d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


# --- thin wrappers, one per C entry point ------------------------------------

def tmm_strerror(status):
    return load().tmm_strerror(int(status)).decode()


def tmm_workspace_bytes(desc):
    n = C.c_size_t()
    _check(load().tmm_workspace_bytes(C.byref(desc), C.byref(n)), "tmm_workspace_bytes")
    return n.value


def tmm_create(desc, workspace, stream):
    h = C.c_void_p()
    _check(load().tmm_create(C.byref(desc), _ptr(workspace), workspace.numel(), C.c_void_p(stream), C.byref(h)),
           "tmm_create")
    return h


def tmm_destroy(h):
    _check(load().tmm_destroy(h), "tmm_destroy")


def tmm_set_params(h, u):
    u = np.ascontiguousarray(np.atleast_2d(u), dtype=np.float64)
    _check(load().tmm_set_params(h, u.shape[0], _host_d(u)), "tmm_set_params")


def tmm_step(h, j, y_in, y_out):
    _check(load().tmm_step(h, int(j), _ptr(y_in), _ptr(y_out)), "tmm_step")


def tmm_year(h, nyears, years_per_member, y0, y1, resid_host):
    ypm = None
    if years_per_member is not None:
        ypm = np.ascontiguousarray(years_per_member, dtype=np.int32)
    _check(load().tmm_year(h, int(nyears), ypm.ctypes.data_as(_ip) if ypm is not None else None,
                           _ptr(y0), _ptr(y1), _host_d(resid_host)), "tmm_year")


def tmm_year_noalloc(h, nyears, y0, y1, resid_host):
    _check(load().tmm_year_noalloc(h, int(nyears), _ptr(y0), _ptr(y1), _host_d(resid_host)), "tmm_year_noalloc")


def tmm_year_jvp(h, mode, y, v, phi_y, jv):
    _check(load().tmm_year_jvp(h, int(mode), _ptr(y), _ptr(v), _ptr(phi_y), _ptr(jv)), "tmm_year_jvp")


def tmm_year_adjoint(h, y0, obs, ckpt_every, J_host, dJdu_host, dJdy0):
    _check(load().tmm_year_adjoint(h, _ptr(y0), _ptr(obs), int(ckpt_every), _host_d(J_host), _host_d(dJdu_host),
                                   _ptr(dJdy0)), "tmm_year_adjoint")


def tmm_set_option(h, option, value):
    _check(load().tmm_set_option(h, int(option), int(value)), "tmm_set_option")


def tmm_probe_exchange(h, rounds):
    out = np.zeros(8)
    _check(load().tmm_probe_exchange(h, int(rounds), _host_d(out)), "tmm_probe_exchange")
    return out


def tmm_query(h, what):
    v = C.c_longlong()
    _check(load().tmm_query(h, int(what), C.byref(v)), "tmm_query")
    return v.value


# --- handle with its workspace ----------------------------------------------

def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class TMM:
    """A libtmm handle with its device workspace (a torch uint8 tensor).

    ``arrays`` holds the descriptor fields (``synth.Inputs.desc_arrays()`` has
    the right keys).  States are float64 CUDA tensors of shape (n, W),
    W = nbatch * ntracer.
    """

    def __init__(self, arrays, nbatch_max=1, adjoint_nbatch_max=0, ckpt_every=240, device="cuda", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("libtmm needs a HIP device")
        load()
        self.device = torch.device(device)
        k = {name: (_i32(v) if np.asarray(v).dtype.kind in "iu" else _f64(v))
             for name, v in arrays.items() if isinstance(v, np.ndarray)}
        self._keep = k
        a = arrays
        self.n = int(a["n"])
        self.model = int(a["model"])
        self.ntracer = _NTRACER[self.model]
        self.nparam = _NPARAM[self.model]
        self.nstep = int(a["nstep"])
        self.nmat = int(a["nmat"])
        self.ckpt_every = int(ckpt_every)
        ip = lambda x: x.ctypes.data_as(_ip)  # noqa: E731
        dp = lambda x: x.ctypes.data_as(_dp)  # noqa: E731
        self.desc = TmmDesc(
            self.n, int(a["ncol"]), int(a["nlayer"]), ip(k["col_start"]), dp(k["lat"]), dp(k["area"]), dp(k["dz"]),
            self.nmat, self.nstep, self.model, int(a["neuphotic"]), int(a.get("nbgc", 1)),
            int(nbatch_max), int(adjoint_nbatch_max), int(ckpt_every),
            k["ae_colidx"].size, ip(k["ae_rowptr"]), ip(k["ae_colidx"]), dp(k["ae_val"]),
            k["ai_colidx"].size, ip(k["ai_rowptr"]), ip(k["ai_colidx"]), dp(k["ai_val"]),
            dp(k["lon"]) if "lon" in k else None,
        )
        self.workspace_bytes = tmm_workspace_bytes(self.desc)
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.handle = tmm_create(self.desc, self.workspace, self.stream.cuda_stream)
        self.nbatch = 0

    def close(self):
        if getattr(self, "handle", None) is not None:
            tmm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, option, value):
        tmm_set_option(self.handle, option, value)

    def query(self, what):
        return tmm_query(self.handle, what)

    def probe_exchange(self, rounds=2000):
        """Latencies (us) of the exchange primitives on this device: round trip within an XCD and
        across XCDs, workgroup barrier, dependent agent-scope load; then the XCDs of the pairs."""
        o = tmm_probe_exchange(self.handle, rounds)
        return {"round_trip_same_xcd_us": o[0], "round_trip_cross_xcd_us": o[1], "barrier_us": o[2],
                "agent_load_us": o[3], "xcds": [int(x) for x in o[4:]]}

    @property
    def W(self):
        return self.nbatch * self.ntracer

    def state(self, host=None):
        """A device state tensor (n, W), optionally filled from a host array."""
        if host is not None:
            return torch.as_tensor(np.ascontiguousarray(host, dtype=np.float64)).to(self.device)
        return torch.empty((self.n, self.W), dtype=torch.float64, device=self.device)

    def _state_arg(self, t):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == (self.n, self.W)):
            raise ValueError(f"state must be a contiguous float64 CUDA tensor of shape {(self.n, self.W)}")
        return t

    def set_params(self, u):
        u = np.atleast_2d(np.asarray(u, dtype=np.float64))
        tmm_set_params(self.handle, u)
        self.nbatch = u.shape[0]

    def step(self, j, y_in, y_out=None):
        y_out = self.state() if y_out is None else y_out
        tmm_step(self.handle, j, self._state_arg(y_in), self._state_arg(y_out))
        return y_out

    def year(self, y0, nyears=1, years_per_member=None, out=None, residuals=True):
        out = self.state() if out is None else out
        resid = np.zeros((nyears, self.nbatch)) if residuals else None
        tmm_year(self.handle, nyears, years_per_member, self._state_arg(y0), self._state_arg(out), resid)
        return out, resid

    def year_noalloc(self, y0, out, nyears=1, residuals=True):
        """Model years through tmm_year_noalloc: out (allocated by the caller) receives the state."""
        resid = np.zeros((nyears, self.nbatch)) if residuals else None
        tmm_year_noalloc(self.handle, nyears, self._state_arg(y0), self._state_arg(out), resid)
        return out, resid

    def year_jvp(self, y, v, mode=TMM_JVP_TANGENT, want_phi=True, phi=None):
        """jv = phi'(y) v.  With mode TMM_JVP_FD_GIVEN_PHI pass phi = phi(y)."""
        jv = self.state()
        if mode == TMM_JVP_FD_GIVEN_PHI:
            if phi is None:
                raise ValueError("TMM_JVP_FD_GIVEN_PHI needs phi")
            tmm_year_jvp(self.handle, mode, self._state_arg(y), self._state_arg(v), self._state_arg(phi), jv)
            return phi, jv
        phi = self.state() if want_phi else None
        tmm_year_jvp(self.handle, mode, self._state_arg(y), self._state_arg(v), phi, jv)
        return phi, jv

    def year_adjoint(self, y0, obs, want_dy0=True):
        if not (obs.is_cuda and obs.dtype == torch.float64 and obs.is_contiguous()
                and tuple(obs.shape) == (self.nmat, self.n, self.W)):
            raise ValueError("obs must be a contiguous float64 CUDA tensor (nmat, n, W)")
        J = np.zeros(self.nbatch)
        G = np.zeros((self.nbatch, self.nparam))
        dy0 = self.state() if want_dy0 else None
        tmm_year_adjoint(self.handle, self._state_arg(y0), obs, self.ckpt_every, J, G, dy0)
        return J, G, dy0
