"""Host drivers over the libtmm ABI: spin-up, Newton-Krylov, ensembles.

These follow sections 4, 6 and 7 of the paper.  A periodic solution is a
fixed point of the year map phi (section 4).  Spin-up finds it by the plain
iteration y <- phi(y) and logs ||y - phi(y)||_2 each year (section 7).  The
Newton solver works on F(y) = y - phi(y), globalised either by a backtracking
line search with cubic interpolation or by a trust region (the two basic
techniques of section 6, after Dennis and Schnabel).  Its linear systems are solved matrix-free by restarted
GMRES with modified Gram-Schmidt and inexact-Newton forcing terms after
Eisenstat and Walker (section 6.2).  Jacobian-vector products come from
libtmm, either as finite differences or as the exact tangent (section 6.1).

The Krylov vectors are host float64 arrays: one state holds 0.84 MB on the
global grid, small next to a model year, so each product copies one vector to
the device and one back.  Every model year runs in libtmm.
"""

import hashlib
import json
import math
import os
import time

import numpy as np
import torch

from . import autotune as _autotune
from . import tmm as _tmm


def _log(path, rec):
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps(rec) + "\n")


def _config_hash(t, u):
    h = hashlib.sha256()
    h.update(np.asarray([t.n, t.nstep, t.nmat, t.model], dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(u, dtype=np.float64).tobytes())
    for k in ("col_start", "ae_rowptr", "ae_colidx", "ae_val", "ai_val"):
        h.update(t._keep[k].tobytes())
    return h.hexdigest()[:16]


# ---------------------------------------------------------------------------
# Spin-up (pseudo-time fixed-point iteration)
# ---------------------------------------------------------------------------

def cell_volumes(t):
    """V_i = area_c h_k for every grid point of the handle's grid (m^3)."""
    k = t._keep
    depth = np.diff(np.asarray(k["col_start"], dtype=np.int64))
    layer = np.concatenate([np.arange(d) for d in depth])
    return np.repeat(np.asarray(k["area"], dtype=np.float64), depth) * np.asarray(k["dz"], dtype=np.float64)[layer]


def tracer_mass(t, y_host, V=None):
    """Volume-weighted total of every tracer of every member: [members, ntracer]."""
    V = cell_volumes(t) if V is None else V
    y = np.asarray(y_host, dtype=np.float64)
    return (V @ y).reshape(-1, t.ntracer)


def spinup(t, u, y0, years, tol=0.0, log_path=None, state_path=None, state_every=0, resume=False,
           return_mass=False, tuned=True):
    """Iterates y <- phi(y) for up to ``years`` model years.

    Returns (y, residuals), where residuals[k] = ||y_k - phi(y_k)||_2 of the
    year that started from y_k (the residual of section 7).  Stops early when
    a residual falls to ``tol`` or below.  Each year's log record also holds
    the volume-weighted mass of every tracer and the relative drift of the
    total (phosphorus) mass since the start of the call: the transport conserves
    mass and the models only move phosphorus between tracers, so the drift is
    rounding.  ``return_mass`` adds the masses ([years + 1, members, ntracer],
    the start state first) as a third result.  With ``state_path`` the state
    is saved every ``state_every`` years as .npz (y, year, u, config hash), and
    ``resume`` continues from such a file when it matches the configuration.
    With ``tuned`` the launch configuration measured best for this grid shape
    (the autotuner's table shipped with the package) is applied first.
    """
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    if tuned:
        _autotune.apply_tuned(t, u.shape[0])
    t.set_params(u)
    cfg = _config_hash(t, u)
    y = t.state(np.asarray(y0, dtype=np.float64))
    start_year = 0
    resid = []
    if resume and state_path and os.path.exists(state_path):
        with np.load(state_path, allow_pickle=False) as z:
            if str(z["config"]) == cfg:
                y = t.state(z["y"])
                start_year = int(z["year"])
                resid = list(z["resid"])
    V = cell_volumes(t)
    masses = [tracer_mass(t, y.cpu().numpy(), V)]
    total0 = masses[0].sum(axis=1)
    nxt = t.state()
    for yr in range(start_year, years):
        t0 = time.perf_counter()
        _, r = t.year(y, nyears=1, out=nxt)
        y, nxt = nxt, y
        resid.append(float(np.linalg.norm(r[0])))
        masses.append(tracer_mass(t, y.cpu().numpy(), V))
        drift = (masses[-1].sum(axis=1) - total0) / total0
        _log(log_path, {"kind": "spinup", "year": yr + 1, "residual": resid[-1],
                        "mass": masses[-1].tolist(), "mass_drift": drift.tolist(),
                        "seconds": time.perf_counter() - t0})
        if state_path and state_every and (yr + 1) % state_every == 0:
            tmp = state_path + ".tmp.npz"
            np.savez(tmp, y=y.cpu().numpy(), year=yr + 1, u=u, config=cfg, resid=np.asarray(resid))
            os.replace(tmp, state_path)
        if resid[-1] <= tol:
            break
    if return_mass:
        return y.cpu().numpy(), np.asarray(resid), np.asarray(masses)
    return y.cpu().numpy(), np.asarray(resid)


# ---------------------------------------------------------------------------
# GMRES(m) with modified Gram-Schmidt, x0 = 0
# ---------------------------------------------------------------------------

def _norm(a):
    return float(torch.linalg.vector_norm(a)) if torch.is_tensor(a) else float(np.linalg.norm(a))


def _dot(a, b):
    return float(torch.dot(a, b)) if torch.is_tensor(a) else float(np.dot(a, b))


def gmres(matvec, b, rtol, restart=30, maxiter=300, log=None):
    """Solves A x = b to ||b - A x|| <= rtol ||b||.

    b and the vectors matvec takes and returns are NumPy arrays or torch
    tensors (on the device that holds the states: the Krylov basis then stays
    there, and only the scalars of the Gram-Schmidt and Givens steps come to
    the host).  Returns (x, r, matvecs) with r = b - A x the true residual at
    exit."""
    bnorm = _norm(b)
    x = torch.zeros_like(b) if torch.is_tensor(b) else np.zeros_like(b)
    if bnorm == 0.0:
        return x, (b.clone() if torch.is_tensor(b) else b.copy()), 0
    target = rtol * bnorm
    r = b.clone() if torch.is_tensor(b) else b.copy()
    beta = bnorm
    its = 0
    while its < maxiter and beta > target:
        V = [r / beta]
        H = np.zeros((restart + 1, restart))
        g = np.zeros(restart + 1)
        g[0] = beta
        cs, sn = np.zeros(restart), np.zeros(restart)
        k_done = 0
        for k in range(restart):
            w = matvec(V[k])
            its += 1
            for i in range(k + 1):                 # modified Gram-Schmidt
                H[i, k] = _dot(w, V[i])
                w = w - float(H[i, k]) * V[i]
            hk1 = _norm(w)
            H[k + 1, k] = hk1
            for i in range(k):                     # earlier Givens rotations
                tmp = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = tmp
            den = math.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = (1.0, 0.0) if den == 0.0 else (H[k, k] / den, H[k + 1, k] / den)
            H[k, k] = cs[k] * H[k, k] + sn[k] * H[k + 1, k]
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            k_done = k + 1
            if log:
                log(its, abs(g[k + 1]))
            if abs(g[k + 1]) <= target or its >= maxiter or hk1 == 0.0:
                break
            V.append(w / hk1)
        coef = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        for i in range(k_done):
            x = x + float(coef[i]) * V[i]
        r = b - matvec(x)
        its += 1
        beta = _norm(r)
    return x, r, its


# ---------------------------------------------------------------------------
# Preconditioner for the Newton systems
# ---------------------------------------------------------------------------

def transport_preconditioner(t, u, eps=1e-6):
    """Right preconditioner for (I - phi'(y)) d = -F built from the transport
    matrices (the direction the paper names in section 9, after Khatiwala 2008).

    One step moves a tracer by A_m = Ai_m Ae_m ~ I + dt L_m, so a year of a
    linear tracer is ~exp(T L) with T L = nstep * mean_m [(Ae_m - I) + (I - Ai_m^-1)]
    (the annual-mean generator; the implicit blocks are inverted exactly).
    For a mode with T L = x the Newton operator is 1 - e^x, and
    1/(1 - e^x) = -1/x + 1/2 + O(x): the preconditioner applies
    z -> (-T L + (eps + T lambda_tr) I)^-1 z + z/2 per tracer, one sparse LU
    factorisation per distinct linear decay rate lambda_tr of the tracer
    (DOP: lambda'_2; PHY: lambda'_3).  This keeps the slow modes of the
    transport, which make the Newton system hard (section 6), within a factor
    of two, and maps the fast ones near 1/2.  The biogeochemical coupling is
    left out.

    Transport conserves volume-weighted mass, so -T L is singular along a
    constant field and its regularised inverse inflates any mass in z by
    1/eps.  The year map conserves total phosphorus, so the Newton updates of
    the unpreconditioned solver carry none; here each member's result is
    projected back to zero total phosphorus (a constant PO4 correction),
    which keeps Newton on the initial mass and its periodic solution.
    Returns apply(z) for flat vectors of the (n, W) state.
    """
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    k = t._keep
    n, nmat, nstep, ntr = t.n, t.nmat, t.nstep, t.ntracer
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))[0]
    col_start = np.asarray(k["col_start"], dtype=np.int64)
    ae_ptr, ae_col = np.asarray(k["ae_rowptr"], dtype=np.int64), np.asarray(k["ae_colidx"], dtype=np.int64)
    ai_ptr, ai_col = np.asarray(k["ai_rowptr"], dtype=np.int64), np.asarray(k["ai_colidx"], dtype=np.int64)
    ae_val = np.asarray(k["ae_val"], dtype=np.float64).reshape(nmat, -1)
    ai_val = np.asarray(k["ai_val"], dtype=np.float64).reshape(nmat, -1)
    eye = sp.identity(n, format="csr")
    # sum over months of (I - Ae_m)
    G = nmat * eye - sp.csr_matrix((ae_val.sum(axis=0), ae_col, ae_ptr), shape=(n, n))
    # sum over months of (Ai_m^-1 - I): each water column's block, inverted, grouped by depth
    depth = np.diff(col_start)
    rows, cols, vals = [], [], []
    for nc in np.unique(depth):
        cs = np.nonzero(depth == nc)[0]
        starts = col_start[cs]
        first = ai_ptr[starts]
        blocks = np.zeros((len(cs), nc, nc))
        for m in range(nmat):
            # rows of a column's block are consecutive and hold its nc x nc entries
            idx = first[:, None] + np.arange(nc * nc)[None, :]
            if not np.array_equal(ai_col[idx].reshape(len(cs), nc, nc),
                                  np.broadcast_to(starts[:, None, None] + np.arange(nc)[None, None, :],
                                                  (len(cs), nc, nc))):
                raise ValueError("implicit matrices must store each column block densely, row by row")
            blocks += np.linalg.inv(ai_val[m][idx].reshape(len(cs), nc, nc)) - np.eye(nc)
        r = starts[:, None, None] + np.arange(nc)[None, :, None]
        c = starts[:, None, None] + np.arange(nc)[None, None, :]
        rows.append(np.broadcast_to(r, blocks.shape).ravel())
        cols.append(np.broadcast_to(c, blocks.shape).ravel())
        vals.append(blocks.ravel())
    G = G + sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    G.eliminate_zeros()
    TL = (-nstep / nmat) * G                       # T times the annual-mean generator
    days = 360.0
    if t.model == _tmm.TMM_MODEL_NDOP:
        decay = [0.0, u[4] * days]
    elif t.model == _tmm.TMM_MODEL_NDOPPHY:
        decay = [0.0, u[4] * days, u[8] * days]
    else:
        decay = [0.0]
    lus = {}
    for lam in set(decay):
        lus[lam] = spla.splu((-TL + (eps + lam) * eye).tocsc())
    layer = np.concatenate([np.arange(d) for d in depth])
    vol = np.repeat(np.asarray(k["area"], dtype=np.float64), depth) * np.asarray(k["dz"], dtype=np.float64)[layer]
    vtot = float(vol.sum())

    def apply(z):
        zz = z.reshape(n, -1)
        out = np.empty_like(zz)
        for w in range(zz.shape[1]):
            col = np.ascontiguousarray(zz[:, w])
            out[:, w] = lus[decay[w % ntr]].solve(col) + 0.5 * col
        for b in range(zz.shape[1] // ntr):
            mass = float(vol @ out[:, b * ntr:(b + 1) * ntr].sum(axis=1))
            out[:, b * ntr] -= mass / vtot
        return out.ravel()

    return apply


# ---------------------------------------------------------------------------
# Inexact Newton-Krylov for y = phi(y)
# ---------------------------------------------------------------------------

def newton_krylov(t, u, y0, tol=1e-8, jvp="fd", restart=30, max_newton=30, max_krylov=300,
                  eta0=0.5, eta_max=0.9, gamma=0.9, ew_alpha=2.0, line_search=True, log_path=None,
                  globalization="line_search", delta0=0.2, delta_max=1e10, preconditioner=None, tuned=True):
    """Solves F(y) = y - phi(y) = 0 from y0 until ||F|| <= tol.

    Linear systems (I - phi'(y)) d = -F by GMRES(restart) with forcing terms
    eta_k = gamma (|F_k|/|F_{k-1}|)^ew_alpha (Eisenstat-Walker choice 2,
    safeguarded, capped at eta_max).  ``jvp`` is "fd" (finite differences
    reusing phi(y): one model year per product) or "tangent" (exact).

    ``globalization`` = "line_search": backtracking on |F|^2 with
    quadratic/cubic interpolation (Dennis and Schnabel); ``line_search=False``
    takes full steps.  "trust_region": the step is the inexact Newton step d
    cut back to the radius Delta (s = min(1, Delta/|d|) d); with r the GMRES
    residual (J d = -F - r) the linear model predicts |F + J s|^2 =
    |(1 - tau) F - tau r|^2 without another product; the step is accepted
    when the actual reduction of |F|^2 is at least 1e-4 of the predicted one,
    and Delta shrinks to |s|/4 when their ratio is below 1/4 and doubles
    (up to ``delta_max``) when it exceeds 3/4 on the boundary.  The first
    radius is ``delta0`` * max(|y0|, 1).

    ``preconditioner`` = "transport" solves the linear systems with the
    right preconditioner of ``transport_preconditioner`` (GMRES still
    minimises the true residual).

    With ``tuned`` the autotuner's launch configuration for this grid shape
    is applied first.

    Returns (y, history); history counts year maps (tangent years count 1
    each).
    """
    if globalization not in ("line_search", "trust_region"):
        raise ValueError("globalization must be 'line_search' or 'trust_region'")
    if preconditioner not in (None, "transport"):
        raise ValueError("preconditioner must be None or 'transport'")
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    if tuned:
        _autotune.apply_tuned(t, u.shape[0])
    t.set_params(u)
    shape = (t.n, t.W)
    pre = transport_preconditioner(t, u) if preconditioner == "transport" else None
    y = np.asarray(y0, dtype=np.float64).copy()
    yd = t.state(y)
    phi, phi_try = t.state(), t.state()
    years = 0

    def F_of(y_host, y_dev, out):
        nonlocal years
        t.year(y_dev, nyears=1, out=out, residuals=False)
        years += 1
        return (y_host - out.cpu().numpy()).ravel()

    F = F_of(y, yd, phi)
    fnorm = float(np.linalg.norm(F))
    hist = {"newton": [], "years": 0, "fnorm": [fnorm]}
    _log(log_path, {"kind": "newton", "it": 0, "fnorm": fnorm, "years": years})
    eta_prev, fnorm_prev = eta0, None
    delta = delta0 * max(float(np.linalg.norm(y)), 1.0)
    for it in range(1, max_newton + 1):
        if fnorm <= tol:
            break
        if fnorm_prev is None:
            eta = eta0
        else:
            eta = gamma * (fnorm / fnorm_prev) ** ew_alpha
            safe = gamma * eta_prev ** ew_alpha
            if safe > 0.1:
                eta = max(eta, safe)
            eta = min(eta, eta_max)
        # keep the linear solve from asking for more than the outer tolerance needs
        eta = max(eta, 0.5 * tol / fnorm)
        phi_y = phi

        def matvec(v):
            nonlocal years
            vd = t.state(v.reshape(shape))
            if jvp == "tangent":
                _, jv = t.year_jvp(yd, vd, mode=_tmm.TMM_JVP_TANGENT, want_phi=False)
            else:
                _, jv = t.year_jvp(yd, vd, mode=_tmm.TMM_JVP_FD_GIVEN_PHI, phi=phi_y)
            years += 1
            return v - jv.cpu().numpy().ravel()

        def matvec_dev(v):
            # the same product on vectors that stay where the states are
            nonlocal years
            vd = v.reshape(shape)
            if jvp == "tangent":
                _, jv = t.year_jvp(yd, vd, mode=_tmm.TMM_JVP_TANGENT, want_phi=False)
            else:
                _, jv = t.year_jvp(yd, vd, mode=_tmm.TMM_JVP_FD_GIVEN_PHI, phi=phi_y)
            years += 1
            return v - jv.reshape(-1)

        if pre is None and torch.is_tensor(phi_y):
            bF = torch.as_tensor(-F).to(phi_y.device)
            d, rlin, mv = gmres(matvec_dev, bF, eta, restart=restart, maxiter=max_krylov)
            d, rlin = d.cpu().numpy(), rlin.cpu().numpy()
        elif pre is None:
            d, rlin, mv = gmres(matvec, -F, eta, restart=restart, maxiter=max_krylov)
        else:
            # right preconditioning: rlin = -F - J P z is the true residual of d = P z
            z, rlin, mv = gmres(lambda v: matvec(pre(v)), -F, eta, restart=restart, maxiter=max_krylov)
            d = pre(z)
        lres = float(np.linalg.norm(rlin))
        if globalization == "trust_region":
            dnorm = float(np.linalg.norm(d))
            rejected = 0
            while True:
                tau = min(1.0, delta / dnorm) if dnorm > 0.0 else 1.0
                y_try = y + tau * d.reshape(shape)
                yt = t.state(y_try)
                F_try = F_of(y_try, yt, phi_try)
                model = (1.0 - tau) * F - tau * rlin          # F + J s of the linear model
                pred = fnorm ** 2 - float(np.dot(model, model))
                ared = fnorm ** 2 - float(np.dot(F_try, F_try))
                ratio = ared / pred if pred > 0.0 else -1.0
                snorm = tau * dnorm
                if ratio < 0.25:
                    delta = 0.25 * snorm
                elif ratio > 0.75 and tau < 1.0:
                    delta = min(2.0 * delta, delta_max)
                if ratio >= 1e-4 or snorm < 1e-12 * max(float(np.linalg.norm(y)), 1.0):
                    break
                rejected += 1
            y, yd, F = y_try, yt, F_try
            phi, phi_try = phi_try, phi
            fnorm_prev, eta_prev = fnorm, eta
            fnorm = float(np.linalg.norm(F))
            rec = {"kind": "newton", "it": it, "fnorm": fnorm, "eta": eta, "krylov": mv, "tau": tau,
                   "delta": delta, "rho": ratio, "rejected": rejected, "linear_residual": lres, "years": years}
            hist["newton"].append(rec)
            hist["fnorm"].append(fnorm)
            _log(log_path, rec)
            continue
        # line search on f = |F|^2 / 2; J d = -F - r, so the slope is F.(J d) = -|F|^2 - F.r
        lam, f0 = 1.0, 0.5 * fnorm ** 2
        slope = -fnorm ** 2 - float(np.dot(F, rlin))
        lam_prev, fl_prev = None, None
        while True:
            y_try = y + lam * d.reshape(shape)
            yt = t.state(y_try)
            F_try = F_of(y_try, yt, phi_try)
            f_try = 0.5 * float(np.dot(F_try, F_try))
            if not line_search or f_try <= f0 + 1e-4 * lam * slope or lam < 1e-4:
                break
            if lam_prev is None:                        # quadratic model
                lam_new = -slope / (2.0 * (f_try - f0 - slope))
            else:                                       # cubic model through two trial points
                a_ = np.array([[1 / lam ** 2, -1 / lam_prev ** 2], [-lam_prev / lam ** 2, lam / lam_prev ** 2]])
                rhs = np.array([f_try - f0 - lam * slope, fl_prev - f0 - lam_prev * slope]) / (lam - lam_prev)
                ca, cb = a_ @ rhs
                if ca == 0:
                    lam_new = -slope / (2 * cb)
                else:
                    disc = max(cb * cb - 3 * ca * slope, 0.0)
                    lam_new = (-cb + math.sqrt(disc)) / (3 * ca)
            lam_prev, fl_prev = lam, f_try
            lam = float(min(max(lam_new, 0.1 * lam), 0.5 * lam))
        y, yd, F = y_try, yt, F_try
        phi, phi_try = phi_try, phi
        fnorm_prev, eta_prev = fnorm, eta
        fnorm = float(np.linalg.norm(F))
        rec = {"kind": "newton", "it": it, "fnorm": fnorm, "eta": eta, "krylov": mv, "lambda": lam,
               "linear_residual": lres, "years": years}
        hist["newton"].append(rec)
        hist["fnorm"].append(fnorm)
        _log(log_path, rec)
    hist["years"] = years
    return y, hist


# ---------------------------------------------------------------------------
# Ensembles with uneven spin-up lengths
# ---------------------------------------------------------------------------

def ensemble(t, U, lengths, y0, tuned=True):
    """Runs member b of parameter table U for lengths[b] model years, all in
    one batched state (members leave the batch when their years are done).
    With ``tuned`` the autotuner's launch configuration for this grid shape and
    member count is applied first."""
    U = np.atleast_2d(np.asarray(U, dtype=np.float64))
    if tuned:
        _autotune.apply_tuned(t, U.shape[0])
    lengths = np.asarray(lengths, dtype=np.int32)
    t.set_params(U)
    y = t.state(np.asarray(y0, dtype=np.float64))
    out, resid = t.year(y, nyears=int(lengths.max()), years_per_member=lengths)
    return out.cpu().numpy(), resid

