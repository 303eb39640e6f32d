"""FP64 oracle of the paper's modelling, parameterisation and fast event
generation (arXiv:2506.09712, Sec. 3 and Sec. 4.2).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline leg of the benchmark use it; the library never does.  Plain numpy
and scipy written from the paper's description; the random draws come from
the oracle's Philox (ct_oracle.c), keyed as the library keys them.

Readings (the paper is silent or garbled on these):
  - Eq. 8 is read as the symmetric generalized Gaussian density on the whole
    line, f(x) = beta / (2 alpha Gamma(1/beta)) exp(-|x/alpha|^beta), x
    measured from the absorption point; its CDF is
    F(x) = 1/2 + sign(x) P(1/beta, |x/alpha|^beta) / 2, with P the
    regularized lower incomplete gamma function.
  - Eq. 9 with the paper's depth axis (z from the entrance side, field of
    Eq. 6 rising towards the pixels): t = [ln(E(H)/E(h))/k + (H - h)/E_c]/mu0,
    k = 2 V_dep / H^2; with V_dep = 0 the limit (H - h)(1/E + 1/E_c)/mu0.
    mu0 and E_c are the Jacoboni-Canali hole values of the sensor.
  - Eq. 11's power term needs t - p_beta1 > 0 for every drift time t >= 0,
    so p_beta1 < 0 is required.
  - Generation (Sec. 4.2), per event with id e, draws keyed (counter, e, 5):
      block (0, 0, e, 5): u_h, u_x, u_y from words 0, 1, 2;
      depth h = -lambda ln(1 - u_h (1 - exp(-H/lambda))) (absorption
      depth, exponential, conditioned on absorption inside the sensor);
      normals (1, 0, e, 5), first one, g: carrier count
      N = max(0, floor(E/w + sqrt(F E/w) g + 1/2)) (Fano factor F);
      sub-pixel shift x0 = (u_x - 1/2) pitch, y0 = (u_y - 1/2) pitch;
      carrier j: block (j div 2, 1, e, 5), words (0, 1) for even j and
      (2, 3) for odd j give (u, v); its column is the pixel whose edges
      bracket the point of the x distribution with CDF u (so
      F(edge_i - x0) <= u < F(edge_{i+1} - x0), a carrier on an edge going
      to the higher pixel), its row likewise from v; outside the grid in
      either direction: the overflow bin;
      pixel p's energy: count_p w + sigma_noise n_p, n_p the (p mod 3)-th
      normal of normals (p div 3, 2, e, 5).
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np
from scipy import optimize, special

from . import mobility_params, normals_many, philox_many

DOMAIN = 5


def _unit(w: np.ndarray) -> np.ndarray:
    return (w.astype(np.float64) + 0.5) * (1.0 / 4294967296.0)


# ------------------------------------------------------------------ Eq. 9

def drift_field_paper(sensor, zp):
    """Eq. 6 on the paper's axis (zp from the entrance side), V/um."""
    H = sensor.thickness_um
    return (sensor.v_bias - sensor.v_dep) / H + 2.0 * sensor.v_dep * np.asarray(zp) / H**2


def drift_time(sensor, h):
    """Eq. 9: approximate drift time (ns) of a hole absorbed at depth h (um
    from the entrance side) to the pixel plane."""
    mu0, ec, _ = mobility_params(sensor)
    H = sensor.thickness_um
    h = np.asarray(h, dtype=np.float64)
    k = 2.0 * sensor.v_dep / H**2
    if k == 0.0:
        E = drift_field_paper(sensor, h)
        return (H - h) * (1.0 / E + 1.0 / ec) / mu0
    return (np.log(drift_field_paper(sensor, H) / drift_field_paper(sensor, h)) / k
            + (H - h) / ec) / mu0


# ------------------------------------------------------------------ Eq. 8

def ggd_pdf(x, alpha, beta):
    x = np.asarray(x, dtype=np.float64)
    return beta / (2.0 * alpha * special.gamma(1.0 / beta)) * np.exp(-np.abs(x / alpha) ** beta)


def ggd_cdf(x, alpha, beta):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 + 0.5 * np.sign(x) * special.gammainc(1.0 / beta, np.abs(x / alpha) ** beta)


def ggd_fit(x) -> tuple:
    """Maximum-likelihood (alpha, beta) of samples of a GGD centred at 0."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size

    def nll(q):
        a, b = np.exp(q)
        return -(n * (np.log(b) - np.log(2.0 * a) - special.gammaln(1.0 / b))
                 - np.sum(np.abs(x / a) ** b))

    a0 = math.sqrt(2.0 * np.mean(x * x))  # Gaussian start: alpha = sqrt(2) sigma
    r = optimize.minimize(nll, [math.log(a0), math.log(2.0)], method="Nelder-Mead",
                          options={"xatol": 1e-10, "fatol": 1e-10, "maxiter": 4000})
    a, b = np.exp(r.x)
    return float(a), float(b)


# ------------------------------------------------------------ Eqs. 10, 11

def alpha_model(t, p):
    t = np.asarray(t, dtype=np.float64)
    return p[0] + p[1] * np.sqrt(t) + p[2] * t + p[3] * t * t


def beta_model(t, p):
    t = np.asarray(t, dtype=np.float64)
    return 2.0 + p[0] * (t - p[1]) ** p[2] + p[3] * np.exp(p[4] * t)


def fit_alpha(t, alpha, sigma: Optional[Sequence[float]] = None):
    """Eq. 10 parameters by (weighted) least squares."""
    p, _ = optimize.curve_fit(lambda tt, a, b, c, d: alpha_model(tt, (a, b, c, d)), t, alpha,
                              p0=[float(np.min(alpha)), 0.0, 0.0, 0.0], sigma=sigma)
    return p


def fit_beta(t, beta, p0, sigma: Optional[Sequence[float]] = None):
    """Eq. 11 parameters by (weighted) nonlinear least squares, p_beta1 < min t."""
    lo = [-np.inf, -np.inf, -np.inf, -np.inf, -np.inf]
    hi = [np.inf, float(np.min(t)) - 1e-9, np.inf, np.inf, np.inf]
    p, _ = optimize.curve_fit(lambda tt, a, b, c, d, e: beta_model(tt, (a, b, c, d, e)), t, beta,
                              p0=p0, sigma=sigma, bounds=(lo, hi), maxfev=20000)
    return p


# ------------------------------------------------------------ generation

def generate(sensor, gen, n_events: int, first_event_id: int = 0) -> dict:
    """Parameterised events (Sec. 4.2) as read above.  gen: energy_kev, fano,
    noise_kev, atten_um, p_alpha[4], p_beta[5].  Returns per event the depth,
    drift time, carrier count, shift, pixel counts [G^2 + 1] and energies
    [G^2] (keV)."""
    H, pitch, G = sensor.thickness_um, sensor.pitch_um, sensor.grid_n
    w_kev = sensor.pair_energy_ev / 1000.0
    mean_n = gen.energy_kev / w_kev
    lam = gen.atten_um
    edges = (np.arange(G + 1) - G / 2.0) * pitch
    out = {k: [] for k in ("h", "t", "n", "x0", "y0", "counts", "energy")}
    for b in range(n_events):
        e = (first_event_id + b) & 0xFFFFFFFF
        w = philox_many(sensor.seed, np.array([[0, 0, e, DOMAIN]]))[0]
        u_h, u_x, u_y = _unit(w[:3])
        h = -lam * math.log(1.0 - u_h * (1.0 - math.exp(-H / lam)))
        t = float(drift_time(sensor, h))
        alpha = float(alpha_model(t, gen.p_alpha))
        beta = float(beta_model(t, gen.p_beta))
        g = normals_many(sensor.seed, np.array([[1, 0, e, DOMAIN]]))[0, 0]
        n = max(0, int(math.floor(mean_n + math.sqrt(gen.fano * mean_n) * g + 0.5)))
        x0, y0 = (u_x - 0.5) * pitch, (u_y - 0.5) * pitch
        cx = ggd_cdf(edges - x0, alpha, beta)
        cy = ggd_cdf(edges - y0, alpha, beta)
        counts = np.zeros(G * G + 1, dtype=np.int64)
        if n > 0:
            j = np.arange((n + 1) // 2, dtype=np.uint32)
            ctr = np.column_stack([j, np.ones_like(j), np.full_like(j, e), np.full_like(j, DOMAIN)])
            words = philox_many(sensor.seed, ctr)
            uv = _unit(words).reshape(-1, 2)[:n]  # carrier 2j: words 0, 1; 2j + 1: words 2, 3
            col = np.searchsorted(cx, uv[:, 0], side="right") - 1
            row = np.searchsorted(cy, uv[:, 1], side="right") - 1
            inside = (col >= 0) & (col < G) & (row >= 0) & (row < G)
            pix = np.where(inside, row * G + col, G * G)
            counts = np.bincount(pix, minlength=G * G + 1)
        nb = (G * G + 2) // 3
        pc = np.arange(nb, dtype=np.uint32)
        noise = normals_many(sensor.seed, np.column_stack(
            [pc, np.full_like(pc, 2), np.full_like(pc, e), np.full_like(pc, DOMAIN)])).reshape(-1)
        energy = counts[:G * G] * w_kev + gen.noise_kev * noise[:G * G]
        for k, v in (("h", h), ("t", t), ("n", n), ("x0", x0), ("y0", y0), ("counts", counts),
                     ("energy", energy)):
            out[k].append(v)
    return {k: np.array(v) for k, v in out.items()}
