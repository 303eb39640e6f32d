"""Pins of the oracle's track events: an event described by its start point,
whose deposits are the midpoints of a walk of straight segments (the
reading of the deposit-based seeding of Algorithm 1 for an extended track;
the paper has no track model).

The walk: segment 0 points along -z, segment k >= 1 along the isotropic unit
vector of the Philox block at counter (k, 0, event id, 3) with
cos(theta) = 1 - 2 u0 and phi = 2 pi u1; walk points and midpoints are folded
back into [0, H].  Each property below is checked against something other
than the oracle itself: the geometry of the walk reconstructed from its
midpoints, rocRAND's Philox for the directions, the uniform law of cos(theta)
and phi, and the seeding convention of multi-deposit events.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
from workloads import Batch, Sensor, track_walks
from test_oracle_pins import rocrand_philox  # noqa: F401  (fixture)


def _track(start, n_segments, seg_len, H=320.0, seed=5, first_event_id=0, n_carriers=None,
           sigma=0.0):
    s = Sensor(thickness_um=H, v_bias=150.0, v_dep=60.0, dt_ns=0.05, seed=seed)
    B = len(start)
    n = n_segments if n_carriers is None else n_carriers
    b = Batch(energy_kev=np.full(B, 10.0), n_carriers=np.full(B, n), sigma_um=np.full(B, sigma),
              n_deposits=np.full(B, n_segments), deposits=np.asarray(start, dtype=np.float64),
              first_event_id=first_event_id, seg_len_um=np.full(B, seg_len))
    return s, b


def _walk_points(start, mids):
    """Walk points p_0..p_n from the midpoints when nothing was folded:
    p_{k+1} = 2 m_k - p_k."""
    p = [np.asarray(start, dtype=np.float64)]
    for m in mids:
        p.append(2.0 * m - p[-1])
    return np.array(p)


def test_walk_geometry_without_folding():
    # a sensor thick enough that a 40 x 5 um walk from its middle never leaves it
    H = 10000.0
    start = [[1.5, -2.0, 0.5 * H]]
    s, b = _track(start, 40, 5.0, H=H)
    mids = oracle.track_deposits(s, b, 0)
    assert mids.shape == (40, 3)
    np.testing.assert_allclose(mids[0], [1.5, -2.0, 0.5 * H - 2.5], rtol=0, atol=1e-12)
    p = _walk_points(start[0], mids)
    seg = np.linalg.norm(np.diff(p, axis=0), axis=1)
    np.testing.assert_allclose(seg, 5.0, rtol=1e-12)
    # later segments are not all along -z
    d = np.diff(p, axis=0) / 5.0
    assert np.abs(d[1:, 2]).max() < 1.0 and np.abs(d[1:, :2]).max() > 0.5


def test_walk_directions_from_rocrand_philox(rocrand_philox):  # noqa: F811
    H = 10000.0
    seed, eid = 0x0123_4567_89AB_CDEF, 77
    start = [[0.0, 0.0, 0.5 * H]]
    s, b = _track(start, 24, 3.0, H=H, seed=seed, first_event_id=eid)
    mids = oracle.track_deposits(s, b, 0)
    rows = [(k, 0, eid, 3, seed & 0xFFFFFFFF, seed >> 32) for k in range(1, 24)]
    w = rocrand_philox(rows).astype(np.float64)
    u0, u1 = (w[:, 0] + 0.5) / 2.0**32, (w[:, 1] + 0.5) / 2.0**32
    c = 1.0 - 2.0 * u0
    sn = np.sqrt(1.0 - c * c)
    d = np.column_stack([sn * np.cos(2 * np.pi * u1), sn * np.sin(2 * np.pi * u1), c])
    d = np.vstack([[0.0, 0.0, -1.0], d])
    p = np.asarray(start[0], dtype=np.float64)
    for k in range(24):
        np.testing.assert_allclose(mids[k], p + 1.5 * d[k], rtol=0, atol=1e-9)
        p = p + 3.0 * d[k]


def test_directions_are_isotropic():
    H = 1e6
    B = 1500
    start = np.column_stack([np.zeros(B), np.zeros(B), np.full(B, 0.5 * H)])
    s, b = _track(start, 20, 1.0, H=H, seed=11)
    d = []
    for e in range(B):
        p = _walk_points(start[e], oracle.track_deposits(s, b, e))
        d.append(np.diff(p, axis=0)[1:])  # segment 0 is fixed
    d = np.concatenate(d)
    assert d.shape == (B * 19, 3)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, rtol=1e-9)
    # cos(theta) uniform on [-1, 1], phi uniform on [0, 2 pi)
    assert stats.kstest(d[:, 2], stats.uniform(-1, 2).cdf).pvalue > 1e-3
    phi = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2 * np.pi)
    assert stats.kstest(phi, stats.uniform(0, 2 * np.pi).cdf).pvalue > 1e-3
    assert np.abs(d.mean(axis=0)).max() < 4.0 / np.sqrt(len(d))
    # events differ (the event id is in the counter)
    assert not np.allclose(oracle.track_deposits(s, b, 0), oracle.track_deposits(s, b, 1))


def test_folding_at_both_faces():
    # from z = 2 um the first 5 um segment leaves the pixel side: the walk
    # point folds to 3 um and the midpoint (-0.5) to 0.5 um
    s, b = _track([[0.0, 0.0, 2.0]], 3, 5.0, H=320.0)
    mids = oracle.track_deposits(s, b, 0)
    np.testing.assert_allclose(mids[0], [0.0, 0.0, 0.5], atol=1e-12)
    # a sensor thinner than a segment folds many times: every deposit stays
    # inside, and the lateral steps are those of the unfolded walk
    H = 1.3
    B = 50
    start = np.column_stack([np.zeros(B), np.zeros(B), np.full(B, H)])
    s, b = _track(start, 30, 5.0, H=H)
    for e in range(B):
        m = oracle.track_deposits(s, b, e)
        assert np.all((m[:, 2] >= 0.0) & (m[:, 2] <= H))
        lat = np.linalg.norm(np.diff(_walk_points(start[e], m)[:, :2], axis=0), axis=1)
        assert np.all(lat <= 5.0 + 1e-9)


def test_track_carriers_sit_on_their_deposits():
    # width 0: carrier i sits exactly on deposit i mod n_segments after seeding
    s, b = _track([[3.0, 4.0, 300.0]], 8, 5.0, n_carriers=37)
    mids = oracle.track_deposits(s, b, 0)
    r = oracle.run(s.replace(max_steps=0), b)
    assert r["status"] == -5
    np.testing.assert_array_equal(r["xyz"], mids[np.arange(37) % 8])
    # with a width, the cloud of each deposit is centred on it
    s, b = _track([[3.0, 4.0, 300.0]], 4, 5.0, n_carriers=40000, sigma=0.5)
    r = oracle.run(s.replace(max_steps=0), b)
    mids = oracle.track_deposits(s, b, 0)
    for k in range(4):
        pts = r["xyz"][k::4]
        np.testing.assert_allclose(pts.mean(axis=0), mids[k], atol=5 * 0.5 / np.sqrt(len(pts)))
        np.testing.assert_allclose(pts.std(axis=0), 0.5, rtol=0.03)


def test_track_walks_workload_and_rejections():
    s, b = track_walks(n_events=4, n_segments=40)
    assert b.deposits.shape == (4, 3) and np.all(b.n_deposits == 40)
    assert np.all(b.deposits[:, 2] == s.thickness_um)
    assert np.all(oracle.carrier_counts(s, b) == 55556)
    one = b.event(2)
    np.testing.assert_array_equal(one.deposits, b.deposits[2:3])
    np.testing.assert_array_equal(oracle.track_deposits(s, b, 2), oracle.track_deposits(s, one, 0))
    for bad in (-1.0, np.inf, np.nan):
        rows = 1 if bad > 0 else 4  # a track's one start row, else one row per deposit
        bb = Batch(energy_kev=[10.0], n_carriers=[8], sigma_um=[0.0], n_deposits=[4],
                   deposits=np.tile([0.0, 0.0, 100.0], (rows, 1)), seg_len_um=[bad])
        assert oracle.run(s, bb)["status"] == -1, bad
