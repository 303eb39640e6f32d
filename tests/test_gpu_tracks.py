"""Track events through the C ABI (ct_event_desc.seg_len_um > 0): the
library draws each track's walk on the device (k_track) and seeds its
carriers around the midpoints; parity with the oracle, which draws the same
walk from the same definition.

Bars as for every event kind: seeding positions within 1e-10 um (the walk
accumulates a few FP64 roundings per segment, fused on the device and not in
the oracle), collection at seeding and pixels exact; complete runs with FP64
endpoints within 0.01 um, the same collection steps and pixels; FP32 pixel
fractions within 1e-3.
"""
import numpy as np
import pytest

import oracle
from workloads import Batch, Sensor, track_walks
from test_gpu_parity import (FP32, FP64, _event_slice, assert_fp32_parity, assert_fp64_parity,
                             gpu_run)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ct():
    import paper_2506_09712_amd as ct
    ct.load()
    oracle.build(force=False)
    return ct


def _seeded(ct, s, b, prec):
    with ct.Simulator(s.replace(max_steps=1), prec) as sim:
        sim.seed(b)
        return sim.collect()


def test_track_deposits_match_oracle(ct):
    """Width 0: every carrier sits on its deposit, so the seeded positions are
    the deposits the device computed; folding at both faces included (thin
    sensor, segments longer than it)."""
    for H, seg, start_z in ((320.0, 5.0, 320.0), (1.3, 5.0, 1.3), (320.0, 7.5, 2.0)):
        s = Sensor(thickness_um=H, v_bias=150.0, v_dep=60.0, seed=21)
        B = 6
        rng = np.random.default_rng(int(H * 10))
        start = np.column_stack([rng.uniform(-12.5, 12.5, (B, 2)), np.full(B, start_z)])
        nseg = [1, 2, 7, 40, 63, 100]
        b = Batch(energy_kev=np.full(B, 10.0), n_carriers=[n * 3 for n in nseg],
                  sigma_um=np.zeros(B), n_deposits=nseg, deposits=start, first_event_id=900,
                  seg_len_um=np.full(B, seg))
        for prec in (FP64, FP32):
            g = _seeded(ct, s, b, prec)
            o = oracle.run(s.replace(max_steps=0), b)
            np.testing.assert_array_equal(g["cstep"], o["cstep"])
            np.testing.assert_array_equal(g["pix"], o["pix"])
            np.testing.assert_allclose(g["xyz"], o["xyz"], rtol=0, atol=1e-10)
            off = g["offsets"]
            for e in range(B):
                dep = oracle.track_deposits(s, b, e)
                sl = g["xyz"][off[e]:off[e + 1]]
                alive = g["cstep"][off[e]:off[e + 1]] < 0
                k = np.arange(len(sl)) % nseg[e]
                np.testing.assert_allclose(sl[alive], dep[k][alive], rtol=0, atol=1e-10)


def test_track_seeding_with_width_matches_oracle(ct):
    s, b = track_walks(n_events=3, seed=4, n_segments=40, n_carriers=4000)
    for prec in (FP64, FP32):
        g = _seeded(ct, s, b, prec)
        o = oracle.run(s.replace(max_steps=0), b)
        np.testing.assert_array_equal(g["cstep"], o["cstep"])
        np.testing.assert_allclose(g["xyz"], o["xyz"], rtol=0, atol=1e-10)


@pytest.mark.parametrize("electrons", [False, True])
def test_track_full_runs_match_oracle(ct, electrons):
    """Complete runs of short tracks (12 segments of 5 um, 3000 holes) next to
    a cloud event and an explicit one, in one batch; each event against the
    oracle run alone."""
    s, tb = track_walks(n_events=2, seed=8, n_segments=12, n_carriers=3000)
    s = s.replace(electrons=electrons)
    rng = np.random.default_rng(3)
    ex = rng.normal(size=(300, 3)) * 1.5 + [2.0, -4.0, 60.0]
    b = Batch(energy_kev=[tb.energy_kev[0], 8.0, tb.energy_kev[1], 0.0],
              n_carriers=[3000, 1500, 3000, 300], sigma_um=[0.5, 1.0, 0.5, 0.0],
              n_deposits=[12, 1, 12, 0],
              deposits=np.vstack([tb.deposits[0], [1.0, 2.0, 150.0], tb.deposits[1]]),
              xyz=np.vstack([ex, ex + [0.0, 0.0, 1.0]]) if electrons else ex,
              n_electrons=[-1, -1, -1, 300 if electrons else 0],
              seg_len_um=[5.0, 0.0, 5.0, 0.0], first_event_id=40)
    g64 = gpu_run(ct, s, b, FP64)
    g32 = gpu_run(ct, s, b, FP32)
    worst = 0.0
    for e in range(4):
        o = oracle.run(s, b.event(e))
        worst = max(worst, assert_fp64_parity(_event_slice(g64, e), o, f"event {e} fp64"))
        assert_fp32_parity(_event_slice(g32, e), o, f"event {e} fp32")
    print(f"tracks (electrons={electrons}): FP64 worst endpoint {worst:.2e} um")


def test_track_batch_equals_alone_bitwise(ct):
    s, b = track_walks(n_events=3, seed=2, n_segments=20, n_carriers=2500)
    for prec in (FP64, FP32):
        g = gpu_run(ct, s, b, prec)
        for e in range(3):
            a = gpu_run(ct, s, b.event(e), prec)
            sl = _event_slice(g, e)
            np.testing.assert_array_equal(a["xyz"], sl["xyz"])
            np.testing.assert_array_equal(a["cstep"], sl["cstep"])
            np.testing.assert_array_equal(a["pix"], sl["pix"])
