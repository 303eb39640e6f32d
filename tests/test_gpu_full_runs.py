"""Complete runs of the large workloads against the FP64 oracle (Algorithm 1,
the whole loop, through the C ABI):

* mixed_energy (1024 events of 1667-6111 holes, 450 um at 200 V): the whole
  batch in one launch per precision; 8 events of each energy against the
  oracle, which runs them at test time;
* gamma_60kev (64 events of 16,667 holes) and track_200kev (16 events of
  55,556 holes): the whole batch per precision; sampled events against
  complete oracle runs stored in tests/golden/oracle_<workload>.npz, written
  by tests/golden/make_large_golden.py (which calls only the oracle, since
  one such event takes the oracle minutes).

Bars (per event): FP64 - endpoints within 0.01 um of the oracle, the same
collection step for every carrier, the same pixel counts and step count;
FP32 - pixel charge fractions within 1e-3.  The FP32 endpoint error
distribution is printed.
"""
import os

import numpy as np
import pytest

import oracle
from workloads import gamma_60kev, mixed_energy, track_200kev
from test_gpu_parity import (ENDPOINT_TOL_UM, FP32, FP64, FRACTION_TOL, _event_slice,
                             assert_fp32_parity, assert_fp64_parity, endpoint_error_stats,
                             fractions, gpu_run)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ct():
    import paper_2506_09712_amd as ct
    ct.load()
    oracle.build(force=False)
    return ct


@pytest.fixture(scope="module")
def mixed(ct):
    s, b = mixed_energy(n_events=1024, seed=0)
    g64 = gpu_run(ct, s, b, FP64)
    g32 = gpu_run(ct, s, b, FP32)
    assert g64["status"] == 0 and g32["status"] == 0
    np.testing.assert_array_equal(g64["pix"].sum(axis=1), b.n_carriers)
    np.testing.assert_array_equal(g32["pix"].sum(axis=1), b.n_carriers)
    return s, b, g64, g32


@pytest.mark.parametrize("energy", [6.0, 12.0, 17.5, 22.0])
def test_mixed_energy_full_runs_vs_oracle(ct, mixed, energy):
    s, b, g64, g32 = mixed
    picks = np.flatnonzero(b.energy_kev == energy)[:8]
    assert len(picks) == 8
    worst64, worst32, d32 = 0.0, 0.0, []
    for e in picks:
        o = oracle.run(s, b.event(int(e)))
        worst64 = max(worst64, assert_fp64_parity(_event_slice(g64, e), o, f"mixed event {e} fp64"))
        assert np.array_equal(g64["steps"][e:e + 1], o["steps"]), e
        g = _event_slice(g32, e)
        worst32 = max(worst32, assert_fp32_parity(g, o, f"mixed event {e} fp32"))
        d32.append(np.hypot(*(g["xyz"][:, :2] - o["xyz"][:, :2]).T))
    d32 = np.concatenate(d32)
    print(f"mixed_energy {energy} keV, events {picks.tolist()}: FP64 worst endpoint {worst64:.2e} um; "
          f"FP32 worst fraction {worst32:.2e}, endpoints max {d32.max():.2e} / p99 "
          f"{np.percentile(d32, 99):.2e} um")


LARGE = {"gamma_60kev": (gamma_60kev, 64), "track_200kev": (track_200kev, 16)}


@pytest.mark.parametrize("name", list(LARGE))
def test_large_workload_full_runs_vs_stored_oracle(ct, name):
    make, n_events = LARGE[name]
    path = os.path.join(GOLDEN, f"oracle_{name}.npz")
    z = np.load(path)  # plain arrays: no pickled objects are loaded
    s, b = make(n_events=n_events, seed=0)
    g64 = gpu_run(ct, s, b, FP64)
    g32 = gpu_run(ct, s, b, FP32)
    assert g64["status"] == 0 and g32["status"] == 0
    np.testing.assert_array_equal(g64["pix"].sum(axis=1), b.n_carriers)
    np.testing.assert_array_equal(g32["pix"].sum(axis=1), b.n_carriers)
    for e in z["events"].tolist():
        # the workload generator still draws the stored event
        assert int(b.n_carriers[e]) == int(z[f"e{e}_n"])
        np.testing.assert_array_equal(b.event(e).deposits, z[f"e{e}_deposits"])
        assert int(z[f"e{e}_status"]) == 0
        off = g64["offsets"]
        sl = slice(int(off[e]), int(off[e + 1]))
        # FP64: endpoints, collection steps, pixels and steps
        np.testing.assert_array_equal(g64["cstep"][sl], z[f"e{e}_cstep"], err_msg=f"{name} {e}")
        err = np.abs(g64["xyz"][sl, :2] - z[f"e{e}_xy"]).max()
        assert err <= ENDPOINT_TOL_UM, (name, e, err)
        np.testing.assert_array_equal(g64["pix"][e], z[f"e{e}_pix"])
        assert int(g64["steps"][e]) == int(z[f"e{e}_steps"])
        # FP32: pixel fractions
        n = int(z[f"e{e}_n"])
        df = np.abs(g32["pix"][e] - z[f"e{e}_pix"]).max() / n
        assert df <= FRACTION_TOL, (name, e, df)
        d = np.hypot(*(g32["xyz"][sl, :2] - z[f"e{e}_xy"]).T)
        same = np.mean(g32["cstep"][sl] == z[f"e{e}_cstep"])
        print(f"{name} event {e}: FP64 endpoint error {err:.2e} um; FP32 fractions {df:.2e}, "
              f"endpoints max {d.max():.2e} / p99 {np.percentile(d, 99):.2e} / mean {d.mean():.2e} um, "
              f"collection steps equal {same:.5f}")
