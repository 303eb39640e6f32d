"""Parity of the GPU event generator (ct_generate, Sec. 4.2) with the oracle's
generator, through the C ABI.

Integers exact: carrier counts and pixel counts of every event (both sides
decide a carrier's pixel by comparing the same FP64 uniform with FP64 edge
CDFs, which differ only by the rounding of the incomplete gamma function);
depth, drift time and shift within 1e-12 relative; energies within 1e-9 keV.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import oracle.generator  # noqa: F401  (oracle.generator.generate)
from workloads import GenParams, Sensor

pytestmark = pytest.mark.gpu

PA = (2.0, 2.5, 0.1, 0.0)
PB = (0.8, -0.5, -0.7, -0.8 * 0.5**-0.7, -3.0)


@pytest.fixture(scope="module")
def ct():
    import paper_2506_09712_amd as ct
    ct.load()
    oracle.build(force=False)
    return ct


def _sensor(**kw):
    base = dict(thickness_um=320.0, v_bias=150.0, v_dep=29.6, temperature_k=307.85, seed=21)
    base.update(kw)
    return Sensor(**base)


def _check(g, o, G):
    np.testing.assert_allclose(g["h"], o["h"], rtol=1e-12)
    np.testing.assert_allclose(g["t"], o["t"], rtol=1e-12)
    np.testing.assert_array_equal(g["n"], o["n"])
    np.testing.assert_allclose(g["x0"], o["x0"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(g["y0"], o["y0"], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(g["counts"], o["counts"])
    np.testing.assert_allclose(g["energy"], o["energy"], rtol=0, atol=1e-9)
    np.testing.assert_array_equal(g["counts"].sum(axis=1), g["n"])


@pytest.mark.parametrize("energy,G,pitch", [(25.0, 5, 25.0), (8.0, 3, 25.0), (60.0, 8, 10.0),
                                            (25.0, 1, 25.0)])
def test_generator_matches_oracle(ct, energy, G, pitch):
    s = _sensor(grid_n=G, pitch_um=pitch)
    gen = GenParams(energy_kev=energy, atten_um=1200.0, p_alpha=PA, p_beta=PB)
    g = ct.generate(s, gen, 300, first_event_id=1000)
    o = oracle.generator.generate(s, gen, 300, first_event_id=1000)
    _check(g, o, G)


def test_generator_edge_cases(ct):
    s = _sensor()
    # no Fano fluctuation and no noise: exact carrier counts and energies
    gen = GenParams(energy_kev=25.0, fano=0.0, noise_kev=0.0, atten_um=300.0, p_alpha=PA, p_beta=PB)
    g = ct.generate(s, gen, 64, first_event_id=2**32 - 10)  # event ids wrap at 2^32
    o = oracle.generator.generate(s, gen, 64, first_event_id=2**32 - 10)
    _check(g, o, 5)
    assert np.all(g["n"] == round(25000.0 / s.pair_energy_ev))
    # a tiny energy: events with no carrier or one
    gen = GenParams(energy_kev=0.004, fano=0.13, atten_um=300.0, p_alpha=PA, p_beta=PB)
    g = ct.generate(s, gen, 200)
    o = oracle.generator.generate(s, gen, 200)
    _check(g, o, 5)
    assert set(np.unique(g["n"])) <= {0, 1, 2}
    # a point-like cloud: everything in the central pixel
    gen = GenParams(energy_kev=25.0, atten_um=300.0, p_alpha=(1e-9, 0, 0, 0), p_beta=PB)
    g = ct.generate(s, gen, 100)
    assert np.all(g["counts"][:, 12] == g["n"])


def test_million_events(ct):
    """One million 25 keV events in one launch: every carrier accounted for,
    Fano-distributed counts, truncated-exponential depths; sampled events
    equal the oracle's."""
    s = _sensor()
    gen = GenParams(energy_kev=25.0, atten_um=1200.0, p_alpha=PA, p_beta=PB)
    n = 1_000_000
    g = ct.generate(s, gen, n)
    np.testing.assert_array_equal(g["counts"].sum(axis=1), g["n"])
    mean_n = 25000.0 / s.pair_energy_ev
    assert g["n"].mean() == pytest.approx(mean_n, abs=5 * math.sqrt(0.13 * mean_n / n))
    assert g["n"].var() == pytest.approx(0.13 * mean_n, rel=0.01)
    H, lam = s.thickness_um, gen.atten_um
    cdf = lambda h: (1 - np.exp(-h / lam)) / (1 - math.exp(-H / lam))
    assert stats.kstest(g["h"], cdf).pvalue > 1e-4
    for e in (0, 123456, 999999):
        o = oracle.generator.generate(s, gen, 1, first_event_id=e)
        sl = {k: v[e:e + 1] for k, v in g.items()}
        _check(sl, o, 5)


def test_generator_error_paths(ct):
    gen = GenParams(energy_kev=25.0, atten_um=300.0, p_alpha=PA, p_beta=PB)
    for s, gp in ((_sensor(grid_n=9), gen),
                  (_sensor(), GenParams(energy_kev=25.0, p_alpha=PA, p_beta=(0.8, 0.5, -0.7, 0, -3))),
                  (_sensor(), GenParams(energy_kev=25.0, p_alpha=(-1.0, 0, 0, 0), p_beta=PB)),
                  (_sensor(), GenParams(energy_kev=0.0, p_alpha=PA, p_beta=PB)),
                  (_sensor(v_dep=160.0, drift=False), gen)):
        with pytest.raises(ct.CtError) as e:
            ct.generate(s, gp, 10)
        assert e.value.status == -1
    assert ct.generate(_sensor(), gen, 0)["counts"].shape == (0, 26)
