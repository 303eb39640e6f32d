"""Host-side modelling code of the library (paper_2506_09712_amd.model)
against the oracle's independent implementation: the drift time of Eq. 9,
maximum-likelihood GGD fits (Eq. 8) and the fits of Eqs. 10 and 11."""
import numpy as np
import pytest
from scipy import stats

from paper_2506_09712_amd import model
from workloads import Sensor


@pytest.fixture(scope="module")
def og():
    import oracle
    oracle.build(force=False)
    import oracle.generator as g
    return g


def test_drift_time_matches_oracle(og):
    h = np.linspace(0.0, 319.9, 41)
    for s in (Sensor(v_dep=29.6, temperature_k=307.85), Sensor(v_dep=0.0), Sensor(thickness_um=650, v_dep=34.7)):
        np.testing.assert_allclose(model.drift_time(s, h), og.drift_time(s, np.minimum(h, s.thickness_um)),
                                   rtol=1e-13, atol=1e-15)


def test_ggd_mle_matches_oracle_fit(og):
    rng = np.random.default_rng(8)
    for a, b in ((4.0, 2.0), (6.0, 2.6), (2.5, 3.4)):
        x = stats.gennorm.rvs(b, scale=a, size=30_000, random_state=rng)
        ma, mb = model.ggd_mle(x)
        oa, ob = og.ggd_fit(x)
        assert ma == pytest.approx(oa, rel=2e-5) and mb == pytest.approx(ob, rel=2e-5)


def test_parameterisation_fits_match_oracle(og):
    rng = np.random.default_rng(2)
    t = np.linspace(0.1, 15.0, 40)
    pa = (2.0, 2.5, 0.1, -0.002)
    a = model.alpha_model(t, pa) * (1 + 0.01 * rng.standard_normal(t.size))
    # the oracle iterates (curve_fit) to about 1e-7; the library solves the linear problem exactly
    np.testing.assert_allclose(model.fit_alpha(t, a), og.fit_alpha(t, a), rtol=1e-5, atol=1e-8)
    pb = (0.8, -0.5, -0.7, -0.8 * 0.5**-0.7, -3.0)
    b = model.beta_model(t, pb) + 0.002 * rng.standard_normal(t.size)
    mb = model.fit_beta(t, b, p0=(0.5, -0.4, -0.6, -1.0, -2.0))
    ob = og.fit_beta(t, b, p0=(0.5, -0.4, -0.6, -1.0, -2.0))
    np.testing.assert_allclose(model.beta_model(t, mb), og.beta_model(t, ob), rtol=0, atol=2e-6)
