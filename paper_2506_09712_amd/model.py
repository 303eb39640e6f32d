"""Modelling and parameterisation of simulated charge clouds (arXiv:2506.09712,
Sec. 3): the drift-time approximation (Eq. 9), maximum-likelihood fits of the
generalized Gaussian (Eq. 8) to the collected holes, and the fits of
alpha(t), beta(t) (Eqs. 10, 11) that `ct_generate` takes.

Host-side analysis of simulation results: the simulations themselves run in
the library's kernels (`parameterise`), the fits here in numpy/scipy.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np
from scipy import optimize, special


def hole_mobility(sensor) -> tuple:
    """(mu0 [um^2/(V ns)], E_c [V/um]) of holes: Jacoboni-Canali at T unless
    the sensor overrides them."""
    T = sensor.temperature_k
    ec = 1.24 * T**1.68 * 1e-4
    mu0 = 1.62e8 * T**-0.52 * 1e-5 / ec
    if not math.isnan(sensor.mu0_override):
        mu0 = sensor.mu0_override
    if not math.isnan(sensor.ec_override):
        ec = sensor.ec_override
    return mu0, ec


def drift_time(sensor, h):
    """Eq. 9 for holes absorbed at depth h (um from the entrance side): the
    field of Eq. 6 rises linearly from (Vb - Vd)/H at the entrance to
    (Vb + Vd)/H at the pixels with slope k = 2 Vd / H^2, and
    t = [ln(E(H)/E(h)) / k + (H - h)/E_c] / mu0."""
    mu0, ec = hole_mobility(sensor)
    H, vb, vd = sensor.thickness_um, sensor.v_bias, sensor.v_dep
    h = np.asarray(h, dtype=np.float64)
    e_h = (vb - vd) / H + 2.0 * vd * h / (H * H)
    if vd == 0.0:
        return (H - h) * (1.0 / e_h + 1.0 / ec) / mu0
    k = 2.0 * vd / (H * H)
    return (np.log(((vb + vd) / H) / e_h) / k + (H - h) / ec) / mu0


def ggd_mle(x) -> tuple:
    """Maximum-likelihood (alpha, beta) of a zero-centred generalized Gaussian
    for samples x.  For a given beta the likelihood peaks at
    alpha = (beta / n * sum |x|^beta)^(1/beta); the profile likelihood in beta
    is maximised over beta in [0.2, 20]."""
    ax = np.abs(np.asarray(x, dtype=np.float64))
    ax = ax[ax > 0]
    n = ax.size
    lx = np.log(ax)
    m = lx.max()

    def alpha_of(b):
        # log of (beta/n sum |x|^beta)^(1/beta), with the largest term factored out
        s = np.sum(np.exp(b * (lx - m)))
        return math.exp(m + (math.log(b / n) + math.log(s)) / b)

    def neg_profile(lb):
        b = math.exp(lb)
        a = alpha_of(b)
        return -(n * (math.log(b) - math.log(2.0 * a) - special.gammaln(1.0 / b)) - n / b)

    r = optimize.minimize_scalar(neg_profile, bounds=(math.log(0.2), math.log(20.0)),
                                 method="bounded", options={"xatol": 1e-10})
    b = math.exp(r.x)
    return alpha_of(b), b


def alpha_model(t, p):
    t = np.asarray(t, dtype=np.float64)
    return p[0] + p[1] * np.sqrt(t) + p[2] * t + p[3] * t * t


def beta_model(t, p):
    t = np.asarray(t, dtype=np.float64)
    return 2.0 + p[0] * (t - p[1]) ** p[2] + p[3] * np.exp(p[4] * t)


def fit_alpha(t, alpha, sigma: Optional[Sequence[float]] = None) -> np.ndarray:
    """Eq. 10 by weighted linear least squares."""
    t = np.asarray(t, dtype=np.float64)
    w = np.ones_like(t) if sigma is None else 1.0 / np.asarray(sigma, dtype=np.float64)
    A = np.column_stack([np.ones_like(t), np.sqrt(t), t, t * t]) * w[:, None]
    return np.linalg.lstsq(A, np.asarray(alpha) * w, rcond=None)[0]


def fit_beta(t, beta, p0, sigma: Optional[Sequence[float]] = None) -> np.ndarray:
    """Eq. 11 by weighted nonlinear least squares with p_beta1 < 0, so that
    the power term is defined at every drift time t >= 0."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(beta, dtype=np.float64)
    w = np.ones_like(t) if sigma is None else 1.0 / np.asarray(sigma, dtype=np.float64)
    lo = [-np.inf, -np.inf, -np.inf, -np.inf, -np.inf]
    hi = [np.inf, -1e-9, np.inf, np.inf, np.inf]
    p0 = np.clip(np.asarray(p0, dtype=np.float64), np.array(lo) + 1e-12, np.array(hi) - 1e-12)
    r = optimize.least_squares(lambda p: (beta_model(t, p) - y) * w, p0, bounds=(lo, hi),
                               xtol=1e-14, ftol=1e-14, gtol=1e-14, max_nfev=20000)
    return r.x


def parameterise(sensor, energy_kev: float, depths: Sequence[float], repeats: int = 10,
                 precision: int = 1, sigma_um: float = -1.0, beta_p0=(0.5, -0.5, -0.8, -0.5, -1.0),
                 device: int = 0) -> dict:
    """Simulate `repeats` events of energy_kev at each absorption depth (um
    from the entrance side) with the library (holes, or holes and electrons
    when the sensor simulates both), fit the GGD to the collected holes' x
    and y (pooled, relative to the absorption point) at each depth,
    then Eqs. 10 and 11 over the drift times of Eq. 9 (with at least five
    depths; else p_alpha and p_beta are None).  The initial cloud width is
    Eq. 2 unless sigma_um >= 0."""
    from . import binding
    from workloads import Batch

    depths = np.asarray(depths, dtype=np.float64)
    H = sensor.thickness_um
    B = len(depths) * repeats
    z0 = np.repeat(H - depths, repeats)  # the library's z axis: distance from the pixel plane
    deposits = np.column_stack([np.zeros(B), np.zeros(B), z0])
    batch = Batch(energy_kev=np.full(B, energy_kev), n_carriers=np.zeros(B, dtype=np.int32),
                  sigma_um=np.full(B, sigma_um), n_deposits=np.ones(B, dtype=np.int32),
                  deposits=deposits, name="parameterise")
    with binding.Simulator(sensor, precision, device=device) as sim:
        r = sim.run(batch)
    off = r["offsets"]
    # each event's rows hold its holes, then (two species) as many electrons
    n_holes = (off[1:] - off[:-1]) // (2 if sensor.electrons else 1)
    alpha, beta = np.zeros(len(depths)), np.zeros(len(depths))
    for i in range(len(depths)):
        rows = [r["xyz"][off[e]:off[e] + n_holes[e], :2]
                for e in range(i * repeats, (i + 1) * repeats)]
        xy = np.concatenate(rows).reshape(-1)
        alpha[i], beta[i] = ggd_mle(xy)
    t = drift_time(sensor, depths)
    # Eq. 11 has five parameters: fit the parameterisation from five depths up
    pa = fit_alpha(t, alpha) if len(depths) >= 5 else None
    pb = fit_beta(t, beta, beta_p0) if len(depths) >= 5 else None
    return {"depth": depths, "t": t, "alpha": alpha, "beta": beta, "p_alpha": pa, "p_beta": pb,
            "steps": r["steps"]}
