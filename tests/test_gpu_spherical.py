"""Parity of the simplified spherical model (Sec. 2.2, Eq. 7) on the GPU with
the FP64 CPU oracle, through the C ABI.

Same bar as the brute-force path: integers (collection steps, pixel counts,
step and pair counts) exact; FP64 endpoints within 0.01 um.  The model is
evaluated in FP64 in both precision modes, so a CT_FP32 context must give
the same bits as a CT_FP64 one.  The field of a fixed state: the enclosed
counts are integers decided by comparing squared distances, which both sides
compute the same way from centres that differ only in summation order, so
with distinct distances the counts agree and the field agrees to rounding
(1e-10 of the event's largest field, written below).
"""
import math

import numpy as np
import pytest

import oracle
from test_gpu_parity import FP32, FP64, _event_slice, assert_fp64_parity, gpu_run
from workloads import Sensor, batch_8kev, explicit_batch, gamma_60kev, single_8kev, track_200kev

pytestmark = pytest.mark.gpu

FIELD_RTOL = 1e-10


@pytest.fixture(scope="module")
def ct():
    import paper_2506_09712_amd as ct
    ct.load()
    oracle.build(force=False)
    return ct


def _sph(s: Sensor) -> Sensor:
    return s.replace(spherical=True)


def _clouds(sizes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        c = [rng.uniform(-10, 10), rng.uniform(-10, 10), rng.uniform(20, 200)]
        out.append(rng.normal(size=(n, 3)) * rng.uniform(0.3, 3.0, 3) + c)
    return out


def test_spherical_field_matches_oracle(ct):
    sizes = [1, 2, 3, 64, 511, 512, 513, 3000, 20000]
    clouds = _clouds(sizes, 3)
    s = _sph(Sensor(softening_um=0.01))
    b = explicit_batch(clouds)
    fields = {}
    for prec in (FP64, FP32):
        with ct.Simulator(s, prec) as sim:
            sim.seed(b)
            fields[prec] = sim.field()
    np.testing.assert_array_equal(fields[FP64], fields[FP32])  # FP64 in both modes
    E = fields[FP64]
    o = 0
    for n, xyz in zip(sizes, clouds):
        ref = oracle.field_spherical(s, xyz)
        got = E[o:o + n]
        o += n
        # n = 1: no field; n = 2: the two holes are equidistant from their
        # centre up to the rounding of the centre, which both sides compute
        # alike (a + b, halved), so they break the tie the same way
        assert np.abs(got - ref).max() <= FIELD_RTOL * np.abs(ref).max(), n
        if n == 1:
            assert np.all(got == 0.0)


def test_hand_worked_case_through_abi(ct):
    """x = -3, -1, 0, 4 on a line (centre exactly at x = 0) enclose 2, 1, 0
    and 3 holes: E = -2K/9, -K, 0, 3K/16 along x with s = 0."""
    s = _sph(Sensor(softening_um=0.0))
    K = oracle.coulomb_k(s)
    xyz = np.array([[-3.0, 0, 50], [-1.0, 0, 50], [0.0, 0, 50], [4.0, 0, 50]])
    with ct.Simulator(s, FP64) as sim:
        sim.seed(explicit_batch([xyz]))
        E = sim.field()
    np.testing.assert_allclose(E[:, 0], [-2 * K / 9, -K, 0.0, 3 * K / 16], rtol=1e-13, atol=0)
    assert np.all(E[:, 1:] == 0.0)


def _disc(M, seed, z0=128.0):
    rng = np.random.default_rng(seed)
    r = np.sort(rng.uniform(0.5, 3.0, M))
    ang = rng.uniform(0, 2 * np.pi, M)
    p = np.stack([r * np.cos(ang), r * np.sin(ang)], axis=1)
    xyz = np.zeros((2 * M, 3))
    xyz[0::2, :2] = p
    xyz[1::2, :2] = -p
    xyz[:, 2] = z0
    return xyz


def test_symmetric_disc_closed_form_through_abi(ct):
    """Point-symmetric disc, partners adjacent: the library's centre stays
    exact (partners cancel in the first level of its reduction), so every
    hole keeps its enclosed count 2 (pairs inside): r^3 = r0^3 + 3 mu K Q t
    to Euler's first-order error, partners stay exact mirrors, and the result
    matches the oracle."""
    M, mu, dt, steps = 50, 200.0, 0.01, 150
    xyz0 = _disc(M, 4)
    s = _sph(Sensor(repulsion=True, drift=False, diffusion=False, mobility="constant",
                    mu0_override=mu, softening_um=0.0, dt_ns=dt))
    b = explicit_batch([xyz0])
    g = gpu_run(ct, s, b, FP64, max_steps=steps)
    assert g["status"] == -5
    p = g["xyz"]
    np.testing.assert_array_equal(p[0::2], -p[1::2] + [0, 0, 256.0])
    assert np.all(p[:, 2] == 128.0)
    K = oracle.coulomb_k(s)
    r0 = np.linalg.norm(xyz0[:, :2], axis=1)
    Q = 2 * (np.arange(2 * M) // 2)
    exact = (r0**3 + 3 * mu * K * Q * dt * steps) ** (1 / 3)
    r = np.linalg.norm(p[:, :2], axis=1)
    assert np.abs(r / exact - 1).max() < 2e-3
    o = oracle.run(s.replace(max_steps=steps), b)
    assert np.abs(p - o["xyz"]).max() < 1e-9


def test_single_8kev_spherical_parity(ct):
    s, b = single_8kev(seed=0)
    s = _sph(s)
    o = oracle.run(s, b)
    g = gpu_run(ct, s, b, FP64)
    err = assert_fp64_parity(g, o, "single_8kev spherical")
    assert g["pairs"] == o["pairs"] and g["hole_steps"] == o["hole_steps"]
    np.testing.assert_array_equal(g["steps"], o["steps"])
    np.testing.assert_array_equal(g["pix"].sum(axis=1), [2222])
    print(f"single_8kev spherical: fp64 endpoint error {err:.2e} um")


def test_ragged_spherical_batch(ct):
    sizes = [0, 1, 2, 3, 511, 512, 513, 1500]
    clouds = _clouds(sizes, 8)
    s = _sph(Sensor(seed=4))
    b = explicit_batch(clouds, first_event_id=77)
    o = oracle.run(s, b)
    g = gpu_run(ct, s, b, FP64)
    assert_fp64_parity(g, o, "ragged spherical")
    np.testing.assert_array_equal(g["steps"], o["steps"])
    np.testing.assert_array_equal(g["pix"].sum(axis=1), sizes)


def test_batch_8kev_spherical_sampled_events(ct):
    s, b = batch_8kev(n_events=256, seed=0)
    s = _sph(s)
    g = gpu_run(ct, s, b, FP64)
    np.testing.assert_array_equal(g["pix"].sum(axis=1), b.n_carriers)
    worst = 0.0
    for e in (0, 131, 255):
        o = oracle.run(s, b.event(e))
        worst = max(worst, assert_fp64_parity(_event_slice(g, e), o, f"spherical event {e}"))
    print(f"batch_8kev spherical: worst endpoint error {worst:.2e} um")


@pytest.mark.parametrize("make,n_ev", [(gamma_60kev, 2), (track_200kev, 1)])
def test_large_events_spherical(ct, make, n_ev):
    """16,667-hole clouds and a 55,556-hole track (many holes per thread,
    many per bin near the centre of a track)."""
    s, b = make(seed=1)
    s = _sph(s)
    b = b.head(n_ev)
    o = oracle.run(s, b)
    g = gpu_run(ct, s, b, FP64)
    assert_fp64_parity(g, o, f"{b.name} spherical")
    np.testing.assert_array_equal(g["steps"], o["steps"])


def test_spherical_resume_reproducible_and_batch_independent(ct):
    s, b = batch_8kev(n_events=6, seed=5)
    s = _sph(s)
    ref = gpu_run(ct, s, b, FP64)
    with ct.Simulator(s, FP64) as sim:  # the same run in calls of 37 steps
        sim.seed(b)
        while True:
            st, _, _ = sim.step(37)
            if st == 0:
                break
            assert st == -5
        r = sim.collect()
    for k in ("xyz", "cstep", "pix", "steps"):
        np.testing.assert_array_equal(r[k], ref[k])
    again = gpu_run(ct, s, b, FP32)
    np.testing.assert_array_equal(again["xyz"], ref["xyz"])
    for e in (0, 4):
        alone = gpu_run(ct, s, b.event(e), FP64)
        np.testing.assert_array_equal(alone["xyz"], _event_slice(ref, e)["xyz"])


def test_spherical_without_repulsion_is_the_brute_force_path(ct):
    s, b = batch_8kev(n_events=3, seed=2)
    s = s.replace(repulsion=False)
    a = gpu_run(ct, s, b, FP64)
    c = gpu_run(ct, _sph(s), b, FP64)
    for k in ("xyz", "cstep", "pix", "steps"):
        np.testing.assert_array_equal(a[k], c[k])


def test_spherical_error_paths(ct):
    with pytest.raises(ct.CtError) as e:
        ct.Simulator(_sph(Sensor(electrons=True)), FP64)
    assert e.value.status == -1


def test_shared_events_mixed_batch(ct):
    """Events above 8192 holes are shared by several workgroups (contiguous
    slices, barriers between the ranking phases); smaller ones keep one.  A
    batch mixing both, with an empty and a one-hole event, meets the oracle:
    exact steps and pixel counts, FP64 endpoints within 0.01 um."""
    sizes = [9000, 0, 1, 2600, 20000, 8192, 8193]
    clouds = _clouds(sizes, 21)
    s = _sph(Sensor(seed=6))
    b = explicit_batch(clouds, first_event_id=300)
    o = oracle.run(s, b)
    g = gpu_run(ct, s, b, FP64)
    assert_fp64_parity(g, o, "shared spherical batch")
    np.testing.assert_array_equal(g["steps"], o["steps"])
    np.testing.assert_array_equal(g["pix"], o["pix"])
    assert g["pairs"] == o["pairs"] and g["hole_steps"] == o["hole_steps"]


def test_shared_event_resume_batch_independent(ct):
    """A shared event (16,667 holes) gives the same bits when stepped in calls
    of 29 steps, alone or in a batch with other events, and in a CT_FP32
    context."""
    s, b = gamma_60kev(seed=3)
    s = _sph(s)
    b = b.head(3)
    ref = gpu_run(ct, s, b, FP64)
    with ct.Simulator(s, FP64) as sim:
        sim.seed(b)
        while True:
            st, _, _ = sim.step(29)
            if st == 0:
                break
            assert st == -5
        r = sim.collect()
    for k in ("xyz", "cstep", "pix", "steps"):
        np.testing.assert_array_equal(r[k], ref[k])
    np.testing.assert_array_equal(gpu_run(ct, s, b, FP32)["xyz"], ref["xyz"])
    alone = gpu_run(ct, s, b.event(1), FP64)
    np.testing.assert_array_equal(alone["xyz"], _event_slice(ref, 1)["xyz"])


def test_spherical_empty_and_degenerate(ct):
    """Empty batch; an empty event, an event collected at seeding and a lone
    hole (no enclosed holes: drift and diffusion only); and a shared event
    (9000 carriers, so 2 workgroups) of which only 10 holes are still
    drifting after seeding, so that most slices are empty.  Against the
    oracle: exact steps and pixels, FP64 endpoints within 0.01 um."""
    s = _sph(Sensor(seed=13))
    with ct.Simulator(s, FP64) as sim:
        sim.seed(explicit_batch([]))
        assert sim.step(0)[0] == 0
    rng = np.random.default_rng(5)
    big = np.column_stack([rng.normal(0, 2, 9000), rng.normal(0, 2, 9000), np.full(9000, -1.0)])
    big[:10, 2] = rng.uniform(40, 60, 10)
    events = [np.zeros((0, 3)), np.array([[0.0, 0.0, -1.0]]), np.array([[1.0, 2.0, 30.0]]), big]
    b = explicit_batch(events, first_event_id=40)
    o = oracle.run(s, b)
    g = gpu_run(ct, s, b, FP64)
    assert_fp64_parity(g, o, "degenerate spherical")
    np.testing.assert_array_equal(g["steps"], o["steps"])
    np.testing.assert_array_equal(g["pix"], o["pix"])
    np.testing.assert_array_equal(g["pix"].sum(axis=1), [0, 1, 1, 9000])
