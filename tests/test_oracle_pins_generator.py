"""Pins of the oracle's modelling, parameterisation and event generation
(Sec. 3, Eqs. 8-11; Sec. 4.2).

Each test checks the oracle against something other than itself: the
simulator's own collection times and a numerical integral (Eq. 9), scipy's
generalized normal law and its maximum-likelihood fit (Eq. 8), recovery of
known parameters (Eqs. 10, 11), and the distributions the generator must
produce (Fano variance, truncated-exponential depths, uniform shifts,
multinomial pixel counts, noise), including an exact point-like limit.
"""
import math
from dataclasses import dataclass

import numpy as np
import pytest
from scipy import integrate, stats

from workloads import Sensor, explicit_batch


@pytest.fixture(scope="module")
def gen():
    import oracle
    oracle.build(force=False)
    import oracle.generator as g
    return g


@dataclass
class Gen:
    energy_kev: float = 2.0
    fano: float = 0.13
    noise_kev: float = 0.13
    atten_um: float = 400.0
    p_alpha: tuple = (5.0, 0.0, 0.0, 0.0)
    p_beta: tuple = (0.0, -1.0, -1.0, 0.5, 0.0)  # beta(t) = 2.5 for every t


def test_drift_time_matches_the_simulator_and_the_integral(oracle_lib, gen):
    """With a beta = 1 mobility, Eq. 9 is the exact drift time of a hole from
    depth h: it equals the integral of 1/v over the path and the collection
    time of the simulator (within two steps, converging at first order)."""
    mu0, ec = 48.0, 1.7
    for vd in (60.0, 0.0):
        s = Sensor(v_dep=vd, repulsion=False, diffusion=False, beta_override=1.0,
                   mu0_override=mu0, ec_override=ec)
        H = s.thickness_um
        h = np.array([1.0, 70.0, 170.0, 250.0, 310.0])  # from the entrance side
        t9 = gen.drift_time(s, h)
        for hi, ti in zip(h, t9):
            E = lambda zp: float(gen.drift_field_paper(s, zp))
            ref = integrate.quad(lambda zp: (1.0 + E(zp) / ec) / (mu0 * E(zp)), hi, H,
                                 epsabs=0, epsrel=1e-12)[0]
            assert ti == pytest.approx(ref, rel=1e-10)
        assert gen.drift_time(s, H) == 0.0
        errs = []
        for dt in (0.05, 0.0125):
            r = oracle_lib.run(s.replace(dt_ns=dt),
                               explicit_batch([np.column_stack([np.zeros(5), np.zeros(5), H - h])]))
            err = np.abs(r["cstep"] * dt - t9)
            assert np.all(err < 2 * dt), (vd, dt, err)
            errs.append(err.max())
        assert errs[1] < 0.5 * errs[0]


def test_ggd_density_and_cdf(gen):
    """Eq. 8 as a density on the line: unit mass, beta = 2 is the normal law
    with sigma = alpha / sqrt 2, beta = 1 the Laplace law with scale alpha,
    and the CDF is scipy's generalized normal CDF."""
    for a, b in ((1.3, 2.0), (4.0, 2.6), (2.0, 1.0), (0.7, 4.0)):
        assert integrate.quad(lambda x: gen.ggd_pdf(x, a, b), -np.inf, np.inf)[0] == pytest.approx(1, abs=1e-10)
        x = np.linspace(-4 * a, 4 * a, 41)
        np.testing.assert_allclose(gen.ggd_cdf(x, a, b), stats.gennorm.cdf(x, b, scale=a), rtol=0, atol=1e-14)
        np.testing.assert_allclose(gen.ggd_pdf(x, a, b), stats.gennorm.pdf(x, b, scale=a), rtol=1e-13)
    x = np.linspace(-5, 5, 11)
    np.testing.assert_allclose(gen.ggd_pdf(x, 1.4, 2.0), stats.norm.pdf(x, scale=1.4 / math.sqrt(2)), rtol=1e-13)
    np.testing.assert_allclose(gen.ggd_pdf(x, 1.4, 1.0), stats.laplace.pdf(x, scale=1.4), rtol=1e-13)
    assert gen.ggd_cdf(0.0, 3.0, 2.5) == 0.5


def test_ggd_fit_recovers_and_matches_scipy(gen):
    rng = np.random.default_rng(4)
    for a, b in ((3.0, 2.0), (5.0, 2.63), (2.0, 3.5)):
        x = stats.gennorm.rvs(b, scale=a, size=40_000, random_state=rng)
        fa, fb = gen.ggd_fit(x)
        assert fa == pytest.approx(a, rel=0.02) and fb == pytest.approx(b, rel=0.04)
        sb, _, sa = stats.gennorm.fit(x, floc=0)
        assert fa == pytest.approx(sa, rel=1e-4) and fb == pytest.approx(sb, rel=1e-4)


def test_parameterisation_fits_recover_known_parameters(gen):
    """Eqs. 10 and 11 fitted to exact model values give back the parameters;
    Eq. 11 starts at 2 when p3 = -p0 (-p1)^p2 and tends to 2."""
    t = np.linspace(0.05, 6.0, 60)
    pa = (1.2, 3.1, -0.4, 0.02)
    np.testing.assert_allclose(gen.fit_alpha(t, gen.alpha_model(t, pa)), pa, rtol=1e-8, atol=1e-10)
    q0, q1, q2, q4 = 0.9, -0.4, -1.3, -0.8
    pb = (q0, q1, q2, -q0 * (-q1) ** q2, q4)
    assert gen.beta_model(0.0, pb) == pytest.approx(2.0, abs=1e-12)
    assert gen.beta_model(1e4, pb) == pytest.approx(2.0, abs=1e-3)
    fit = gen.fit_beta(t, gen.beta_model(t, pb), p0=(1.0, -0.5, -1.0, -2.0, -1.0))
    np.testing.assert_allclose(gen.beta_model(t, fit), gen.beta_model(t, pb), rtol=0, atol=1e-7)


def test_generator_distributions(gen):
    """Carrier counts: mean E/w, variance F E/w (Fano); depths: the exponential
    law truncated to the sensor; shifts uniform over the pixel; every carrier
    in a pixel or the overflow bin; noise: normal with sigma_noise."""
    s = Sensor(seed=11)
    g = Gen()
    r = gen.generate(s, g, 3000, first_event_id=500)
    mean_n = g.energy_kev / (s.pair_energy_ev / 1000.0)
    assert r["n"].mean() == pytest.approx(mean_n, abs=4 * math.sqrt(g.fano * mean_n / 3000))
    assert r["n"].var() == pytest.approx(g.fano * mean_n, rel=0.1)
    np.testing.assert_array_equal(r["counts"].sum(axis=1), r["n"])
    H, lam = s.thickness_um, g.atten_um
    cdf = lambda h: (1 - np.exp(-h / lam)) / (1 - math.exp(-H / lam))
    assert stats.kstest(r["h"], cdf).pvalue > 1e-3
    assert stats.kstest(r["x0"] / s.pitch_um + 0.5, "uniform").pvalue > 1e-3
    resid = r["energy"] - r["counts"][:, :25] * (s.pair_energy_ev / 1000.0)
    assert resid.std() == pytest.approx(g.noise_kev, rel=0.03)
    assert abs(resid.mean()) < 0.01
    np.testing.assert_allclose(r["t"], gen.drift_time(s, r["h"]), rtol=1e-14)


def test_generator_pixel_counts_are_multinomial(gen):
    """One 200 keV event with fixed alpha and beta: the pixel counts follow
    the multinomial law with the GGD's pixel probabilities (chi-square)."""
    s = Sensor(seed=3, pitch_um=10.0)
    g = Gen(energy_kev=200.0, p_alpha=(8.0, 0, 0, 0), p_beta=(0.0, -1.0, -1.0, 0.8, 0.0))
    pv = []
    for e in range(6):
        r = gen.generate(s, g, 1, first_event_id=e)
        edges = (np.arange(6) - 2.5) * s.pitch_um
        px = np.diff(np.concatenate([[0.0], gen.ggd_cdf(edges - r["x0"][0], 8.0, 2.8), [1.0]]))
        py = np.diff(np.concatenate([[0.0], gen.ggd_cdf(edges - r["y0"][0], 8.0, 2.8), [1.0]]))
        p = np.outer(py[1:-1], px[1:-1]).reshape(-1)
        p = np.append(p, 1.0 - p.sum())
        n = r["n"][0]
        pv.append(stats.chisquare(r["counts"][0], n * p).pvalue)
    assert min(pv) > 1e-4 and np.median(pv) > 0.02


def test_generator_point_like_limit_is_exact(gen):
    """alpha -> 0: every carrier lands in the pixel holding the shift point,
    which lies in the central pixel."""
    s = Sensor(seed=9)
    g = Gen(p_alpha=(1e-9, 0, 0, 0), noise_kev=0.0)
    r = gen.generate(s, g, 50)
    assert np.all(r["counts"][:, 12] == r["n"])
    np.testing.assert_allclose(r["energy"][:, 12], r["n"] * s.pair_energy_ev / 1000.0, rtol=1e-15)
