"""ct_seed_events_noalloc, the seeding entry point for callers that cannot
allocate device memory, through the C ABI: its runs must equal those of
ct_seed_events on the same inputs bit for bit (the same kernels run; only
the queue memory differs), for two seedings of one context in a row (the
second batch smaller), for a batch whose queue only fits the scratch with
fewer tickets (events parked and run again), in both precisions.  Also: the
scratch taken over by another context, a batch too large for the scratch,
and the refusals (no bound workspace, autotuning)."""
import numpy as np
import pytest

from workloads import batch_8kev, explicit_batch, Sensor

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
CT_ESTATE, CT_EINVAL, CT_ENOMEM = -2, -1, -3


@pytest.fixture(scope="module")
def ct():
    import paper_2506_09712_amd as ct
    ct.load()
    return ct


def _same(a, b, tag):
    for k in ("xyz", "cstep", "pix", "steps"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"{tag}: {k}")
    assert a["pairs"] == b["pairs"] and a["hole_steps"] == b["hole_steps"], tag


def _run_normal(ct, s, b, prec):
    with ct.Simulator(s, prec) as sim:
        sim.seed(b)
        st, _, _ = sim.step(0)
        r = sim.collect()
    assert st == 0
    return r


def test_noalloc_equals_ct_seed_events_twice(ct):
    s, big = batch_8kev(n_events=48, seed=3)
    small = big.head(5)
    for prec in (FP64, FP32):
        ref_big, ref_small = _run_normal(ct, s, big, prec), _run_normal(ct, s, small, prec)
        with ct.Simulator(s, prec) as sim:  # one context, two seedings in a row
            out = []
            for b in (big, small):
                sim.seed(b, noalloc=True)
                st, _, _ = sim.step(0)
                assert st == 0
                out.append(sim.collect())
        _same(out[0], ref_big, f"prec {prec}, first call")
        _same(out[1], ref_small, f"prec {prec}, second (smaller) call")


def test_noalloc_with_a_shortened_queue(ct):
    """Batches whose partial fields fill most of the scratch: the queue is
    shortened to what is left.  256 events of 2222 holes still hold the whole
    run; 7 events of 16,667 holes (112 MB of partial fields) park events and
    run them again.  The results are unchanged."""
    from workloads import gamma_60kev
    for make, n, parks in ((batch_8kev, 256, False), (gamma_60kev, 7, True)):
        s, b = make(n_events=n, seed=0)
        ref = _run_normal(ct, s, b, FP32)
        with ct.Simulator(s, FP32, options=ct.CT_OPT_TIMING) as sim:
            sim.seed(b, noalloc=True)
            st, _, _ = sim.step(0)
            r = sim.collect()
        assert st == 0
        _same(r, ref, f"{make.__name__} x {n}")
        if parks:
            assert r["stats"].field_launches > 1  # parked events ran again


def test_noalloc_scratch_taken_over_and_refusals(ct):
    s = Sensor(seed=5)
    rng = np.random.default_rng(2)
    ev = explicit_batch([rng.normal(size=(300, 3)) + [0, 0, 40.0]])
    a = ct.Simulator(s, FP64)
    b = ct.Simulator(s, FP64)
    try:
        a.seed(ev, noalloc=True)
        b.seed(ev, noalloc=True)  # takes the device's scratch over
        with pytest.raises(ct.CtError) as e:
            a.step(0)
        assert e.value.status == CT_ESTATE
        with pytest.raises(ct.CtError) as e:
            a.collect()
        assert e.value.status == CT_ESTATE
        st, _, _ = b.step(0)
        assert st == 0
        ref = b.collect()
        a.seed(ev, noalloc=True)  # seeded again: the scratch is a's
        st, _, _ = a.step(0)
        assert st == 0
        _same(a.collect(), ref, "after taking the scratch back")
        with pytest.raises(ct.CtError) as e:
            b.step(0)
        assert e.value.status == CT_ESTATE
        b.seed(ev)  # the usual seeding leaves the scratch alone
        assert b.step(0)[0] == 0
    finally:
        a.close()
        b.close()
    # a batch whose queue cannot fit the scratch (its workspace is bound and
    # large enough): refused before anything changes
    from paper_2506_09712_amd.binding import EventDescs
    big = explicit_batch([rng.normal(size=(55556, 3)) * 20 + [0, 0, 150.0]])
    with ct.Simulator(s, FP32) as sim:
        sim.seed(big)  # binds a workspace large enough for the big batch
        sim.seed(ev, noalloc=True)
        with pytest.raises(ct.CtError) as e:
            ct.ct_seed_events_noalloc(sim.ctx, EventDescs(big), 0)
        assert e.value.status == CT_ENOMEM
        assert sim.step(0)[0] == 0  # the earlier batch is still there
    # no bound workspace; autotuning
    with ct.Simulator(s, FP64, use_torch=False) as sim:
        with pytest.raises(ct.CtError) as e:
            sim.seed(ev, noalloc=True)
        assert e.value.status == CT_ESTATE
    with ct.Simulator(s, FP32, options=ct.CT_OPT_AUTOTUNE) as sim:
        with pytest.raises(ct.CtError) as e:
            sim.seed(ev, noalloc=True)
        assert e.value.status == CT_EINVAL
