"""Biogeochemical parameter vectors and other seeded draws.

Parameter order follows the paper's table for the PO4-DOP model
(section 2.2.1): alpha, K_H2O, K_1, K_I, lambda'_2, sigma_2, b.  The one-tracer
nutrient model ("N") drops the DOP tracer and its two parameters:
alpha, K_H2O, K_N, K_I, b.

The PO4-DOP-PHY model (section 2.2.2) has three tracers (PO4, DOP, PHY) and
eleven parameters, in the order of its table: mu_1, K_H2O, K_1, K_I,
lambda'_2, sigma_2, lambda_3, kappa_3, lambda'_3, sigma_3, b.

The paper lists names and units but no values or bounds; the nominal values
and bounds below are this implementation's choice.  They keep
``dt_d * alpha_max / K_1,min = 0.5`` no larger than the smallest diagonal
entry of the explicit matrices, so one step cannot drive a concentration
negative.  For PO4-DOP-PHY the growth term is proportional to PHY; the rates
are chosen so that dt_d times any linear rate stays below 0.5.
"""

import numpy as np

MODEL_N = 1
MODEL_NDOP = 2
MODEL_NDOPPHY = 3
NTRACER = {MODEL_N: 1, MODEL_NDOP: 2, MODEL_NDOPPHY: 3}
NPARAM = {MODEL_N: 5, MODEL_NDOP: 7, MODEL_NDOPPHY: 11}
PARAM_NAMES = {
    MODEL_NDOP: ("alpha", "K_H2O", "K_1", "K_I", "lambda2", "sigma2", "b"),
    MODEL_N: ("alpha", "K_H2O", "K_N", "K_I", "b"),
    MODEL_NDOPPHY: ("mu1", "K_H2O", "K_1", "K_I", "lambda2", "sigma2", "lambda3", "kappa3", "lambda3p",
                    "sigma3", "b"),
}

_NOMINAL_NDOP = np.array([0.5, 0.02, 0.5, 30.0, 0.5 / 360.0, 0.67, 0.858])
_LO_NDOP = np.array([0.25, 0.01, 0.25, 15.0, 0.25 / 360.0, 0.05, 0.7])
_HI_NDOP = np.array([1.0, 0.05, 1.0, 60.0, 1.0 / 360.0, 0.95, 1.5])
_N_SEL = [0, 1, 2, 3, 6]
_NOMINAL_PHY = np.array([2.0, 0.02, 0.5, 30.0, 0.5 / 360.0, 0.67, 0.03, 1.0, 0.01, 0.5, 0.858])
_LO_PHY = np.array([1.0, 0.01, 0.25, 15.0, 0.25 / 360.0, 0.05, 0.01, 0.5, 0.005, 0.1, 0.7])
_HI_PHY = np.array([3.0, 0.05, 1.0, 60.0, 1.0 / 360.0, 0.95, 0.05, 2.0, 0.05, 0.9, 1.5])


def nominal(model: int) -> np.ndarray:
    if model == MODEL_NDOPPHY:
        return _NOMINAL_PHY.copy()
    return _NOMINAL_NDOP.copy() if model == MODEL_NDOP else _NOMINAL_NDOP[_N_SEL].copy()


def bounds(model: int):
    if model == MODEL_NDOPPHY:
        return _LO_PHY.copy(), _HI_PHY.copy()
    if model == MODEL_NDOP:
        return _LO_NDOP.copy(), _HI_NDOP.copy()
    return _LO_NDOP[_N_SEL].copy(), _HI_NDOP[_N_SEL].copy()


def latin_hypercube(model: int, nsamples: int, seed: int) -> np.ndarray:
    """Latin-hypercube sample of parameter vectors within the bounds."""
    lo, hi = bounds(model)
    rng = np.random.default_rng(seed)
    d = lo.size
    u = np.empty((nsamples, d))
    for p in range(d):
        strata = (rng.permutation(nsamples) + rng.uniform(size=nsamples)) / nsamples
        u[:, p] = lo[p] + strata * (hi[p] - lo[p])
    return u


def spinup_lengths(nmembers: int, seed: int, lo: int = 1, hi: int = 8) -> np.ndarray:
    """Per-member spin-up lengths in model years, uniform integers in [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=nmembers).astype(np.int32)


def hidden_params(model: int, seed: int, spread: float = 0.2) -> np.ndarray:
    """'True' parameters for synthetic observations: nominal*(1+spread*U(-1,1)), clipped."""
    lo, hi = bounds(model)
    rng = np.random.default_rng(seed)
    u = nominal(model) * (1.0 + spread * rng.uniform(-1.0, 1.0, size=lo.size))
    return np.clip(u, lo, hi)


def obs_noise(shape, seed: int) -> np.ndarray:
    """Standard-normal draws for multiplicative observation noise."""
    return np.random.default_rng(seed).standard_normal(shape)
