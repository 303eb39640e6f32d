"""Parity of the two-species path (holes and electrons, Sec. 2.1) with the
FP64 CPU oracle, through the C ABI.

Same tolerances as the hole-only path: integers (collection steps, pixel
counts) exact; FP64 endpoints of every carrier, holes and electrons, within
0.01 um; FP32 pixel fractions within 1e-3; the field of a fixed state within
the bound derived from the arithmetic of each mode.
"""
import numpy as np
import pytest

import oracle
from test_gpu_parity import (ENDPOINT_TOL_UM, FP32, FP64, FRACTION_TOL, _event_slice,
                             assert_fp32_parity, assert_fp64_parity, field_error_bound, gpu_run)
from workloads import Batch, Sensor, batch_8kev_eh, explicit_batch, single_8kev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ct():
    import paper_2506_09712_amd as ct
    ct.load()
    oracle.build(force=False)
    return ct


def _holes_in_pixels(r, n_holes):
    np.testing.assert_array_equal(r["pix"].sum(axis=1), n_holes)


@pytest.mark.parametrize("nh,ne", [(1, 1), (7, 3), (255, 256), (300, 0), (0, 40), (1000, 1000)])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_mixed_field_matches_oracle(ct, nh, ne, prec):
    rng = np.random.default_rng(nh * 1000 + ne)
    h = rng.normal(size=(nh, 3)) * [1.0, 1.5, 0.8] + [4.0, -3.0, 120.0]
    e = rng.normal(size=(ne, 3)) * [1.2, 1.0, 0.9] + [4.5, -3.0, 121.0]
    s = Sensor(softening_um=0.01, electrons=True)
    xyz = np.concatenate([h, e])
    q = np.concatenate([np.ones(nh), -np.ones(ne)])
    ref = oracle.field_q(s, xyz, q)
    b = explicit_batch([h], electrons_per_event=[e])
    for launch in [None, (1, 128, 128), (2, 256, 256), (1, 64, 64)]:
        # the tile of an item's targets (the frame of its FP32 coordinates)
        frame = 256 if launch is None or prec == FP64 else launch[0] * launch[1]
        bound = field_error_bound(xyz, s.softening_um, oracle.coulomb_k(s), prec == FP32,
                                  frame_tile=frame)
        with ct.Simulator(s, prec, launch=launch) as sim:
            sim.seed(b)
            E = sim.field()
        if nh == 0:  # an event with no hole has ended before its first step
            assert np.all(np.isnan(E))
            continue
        err = np.abs(E - ref).max(axis=1)
        assert np.all(err <= bound + 1e-300), (launch, (err / np.maximum(bound, 1e-300)).max())


def test_single_8kev_pairs_fp64_and_fp32(ct):
    s, b = single_8kev(seed=0)
    s = s.replace(electrons=True)
    o = oracle.run(s, b)
    assert o["n"][0] == 4444
    g = gpu_run(ct, s, b, FP64)
    err = assert_fp64_parity(g, o, "single_8kev pairs fp64")
    assert g["pairs"] == o["pairs"] and g["hole_steps"] == o["hole_steps"]
    assert np.array_equal(g["steps"], o["steps"])
    _holes_in_pixels(g, [2222])
    g32 = gpu_run(ct, s, b, FP32)
    assert g32["stats"].newton_pairs == 1  # charged Newton pairs
    df = assert_fp32_parity(g32, o, "single_8kev pairs fp32")
    _holes_in_pixels(g32, [2222])
    g1 = gpu_run(ct, s, b, FP32, options=ct.CT_OPT_ONE_SIDED)
    assert g1["stats"].newton_pairs == 0
    df1 = assert_fp32_parity(g1, o, "single_8kev pairs fp32, every ordered pair")
    _holes_in_pixels(g1, [2222])
    print(f"single_8kev with electrons: fp64 endpoint error {err:.2e} um, fp32 fraction {df:.2e} "
          f"(Newton pairs), {df1:.2e} (every ordered pair)")


@pytest.mark.parametrize("launch", [None, (1, 128, 128), (2, 256, 256), (4, 256, 1024), (1, 64, 64)])
def test_ragged_two_species_all_launches(ct, launch):
    rng = np.random.default_rng(33)
    sizes = [(0, 0), (1, 0), (0, 2), (2, 1), (63, 64), (65, 1), (300, 300), (700, 1025)]
    hs, es = [], []
    for nh, ne in sizes:
        c = [rng.uniform(-10, 10), rng.uniform(-10, 10), rng.uniform(5, 60)]
        hs.append(rng.normal(size=(nh, 3)) * 1.2 + c)
        es.append(rng.normal(size=(ne, 3)) * 1.2 + c)
    s = Sensor(seed=9, electrons=True)
    b = explicit_batch(hs, first_event_id=100, electrons_per_event=es)
    o = oracle.run(s, b)
    g = gpu_run(ct, s, b, FP64, launch=launch)
    assert_fp64_parity(g, o, f"ragged two-species fp64 {launch}")
    g32 = gpu_run(ct, s, b, FP32, launch=launch)
    assert_fp32_parity(g32, o, f"ragged two-species fp32 {launch}")
    _holes_in_pixels(g32, [nh for nh, _ in sizes])


def test_batch_8kev_eh_sampled_events(ct):
    """The two-species bench batch (256 events x 4444 carriers) in one run;
    sampled events against the oracle."""
    s, b = batch_8kev_eh(n_events=256, seed=0)
    g64 = gpu_run(ct, s, b, FP64)
    g32 = gpu_run(ct, s, b, FP32)
    _holes_in_pixels(g64, b.n_carriers)
    _holes_in_pixels(g32, b.n_carriers)
    worst64, worst32 = 0.0, 0.0
    for e in (0, 97, 255):
        o = oracle.run(s, b.event(e))
        worst64 = max(worst64, assert_fp64_parity(_event_slice(g64, e), o, f"eh event {e} fp64"))
        worst32 = max(worst32, assert_fp32_parity(_event_slice(g32, e), o, f"eh event {e} fp32"))
    print(f"batch_8kev_eh: fp64 worst endpoint {worst64:.2e} um; fp32 worst fraction {worst32:.2e}")


def test_two_species_batch_equals_alone_and_reruns_bitwise(ct):
    s, b = batch_8kev_eh(n_events=4, seed=2)
    b = Batch(b.energy_kev, [600, 900, 300, 1200], b.sigma_um, b.n_deposits, b.deposits,
              first_event_id=40)
    for prec in (FP64, FP32):
        g = gpu_run(ct, s, b, prec)
        again = gpu_run(ct, s, b, prec)
        np.testing.assert_array_equal(g["xyz"], again["xyz"])
        for e in range(4):
            a = gpu_run(ct, s, b.event(e), prec)
            sl = _event_slice(g, e)
            np.testing.assert_array_equal(a["xyz"], sl["xyz"])
            np.testing.assert_array_equal(a["cstep"], sl["cstep"])
            np.testing.assert_array_equal(a["pix"], sl["pix"])


def test_pair_approach_through_abi(ct):
    """Closed form through the library: an electron-hole pair closes as
    r^3 = r0^3 - 3 (mu_h + mu_e) K t (constant mobilities, no drift or
    diffusion), and the mobility-weighted point stays put."""
    mu_h, mu_e, r0, dt, steps = 48.0, 140.0, 0.6, 0.01, 150
    s = Sensor(electrons=True, repulsion=True, drift=False, diffusion=False, mobility="constant",
               mu0_override=mu_h, mu0_e_override=mu_e, softening_um=0.0, dt_ns=dt)
    b = explicit_batch([[[-r0 / 2, 0.0, 100.0]]], electrons_per_event=[[[r0 / 2, 0.0, 100.0]]])
    K = oracle.coulomb_k(s)
    exact = (r0**3 - 3 * (mu_h + mu_e) * K * dt * steps) ** (1 / 3)
    for prec in (FP64, FP32):
        g = gpu_run(ct, s, b, prec, max_steps=steps)
        assert g["status"] == -5
        p = g["xyz"]
        assert abs((p[1, 0] - p[0, 0]) - exact) / exact < 1e-3
        centre = (mu_e * p[0, 0] + mu_h * p[1, 0]) / (mu_h + mu_e)
        assert centre == pytest.approx((mu_e * (-r0 / 2) + mu_h * (r0 / 2)) / (mu_h + mu_e), abs=1e-9)


def test_two_species_error_paths(ct):
    s = Sensor()  # no electron species
    b = explicit_batch([[[0, 0, 10.0]]], electrons_per_event=[[[0, 0, 11.0]]])
    with ct.Simulator(s, FP64) as sim:
        with pytest.raises(ct.CtError) as e:
            sim.seed(b)
        assert e.value.status == -1
    s2 = Sensor(electrons=True)
    _, bb = single_8kev()
    bad = Batch(bb.energy_kev, bb.n_carriers, bb.sigma_um, bb.n_deposits, bb.deposits,
                n_electrons=[5])  # a cloud event has one electron per hole
    with ct.Simulator(s2, FP64) as sim:
        with pytest.raises(ct.CtError) as e:
            sim.seed(bad)
        assert e.value.status == -1
