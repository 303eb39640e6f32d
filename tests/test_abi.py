"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/ct.h declares, validates parameters and events, and
reports CT_EDEVICE on a host without a gfx950 device."""
import math
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ct.h")


@pytest.fixture(scope="module")
def ct():
    import paper_2506_09712_amd as ct
    from paper_2506_09712_amd.binding import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_2506_09712_amd.build import build
        build()
    ct.load()
    return ct


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ct_[a-z_]+)\s*\(", src)))


def test_header_compiles_as_c99():
    out = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", HEADER],
                         capture_output=True, text=True)
    assert out.returncode == 0, out.stderr


def test_library_exports_every_declared_function(ct):
    declared = _declared_functions()
    assert set(declared) == set(ct.EXPORTS)
    lib = ct.load()
    for name in declared:
        assert hasattr(lib, name), name
    from paper_2506_09712_amd.binding import LIB_PATH
    nm = subprocess.run(["nm", "-D", "--defined-only", LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (ct_[a-z_]+)", nm))
    assert set(declared) <= exported


def test_struct_layout_matches_header(ct):
    """Sizes of the ABI structs as a C compiler lays them out."""
    from paper_2506_09712_amd.binding import ct_event_desc, ct_run_stats, ct_sensor_params
    import ctypes as C
    prog = ('#include <stdio.h>\n#include "ct.h"\nint main(void){printf("%zu %zu %zu\\n",'
            'sizeof(ct_sensor_params), sizeof(ct_event_desc), sizeof(ct_run_stats));return 0;}')
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(prog)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o",
                        os.path.join(d, "s")], check=True)
        out = subprocess.run([os.path.join(d, "s")], capture_output=True, text=True).stdout.split()
    assert [int(v) for v in out] == [C.sizeof(ct_sensor_params), C.sizeof(ct_event_desc),
                                     C.sizeof(ct_run_stats)]


def test_no_device_is_reported_not_crashed(ct):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from workloads import single_8kev
    s, _ = single_8kev()
    with pytest.raises(ct.CtError) as e:
        ct.ct_init_sensor(ct.make_params(s))
    assert e.value.status == -4  # CT_EDEVICE


def test_parameter_validation(ct):
    from workloads import Sensor
    bad = [dict(v_bias=50.0, v_dep=60.0), dict(dt_ns=0.0), dict(thickness_um=-1.0),
           dict(grid_n=0), dict(softening_um=-0.1), dict(temperature_k=0.0), dict(max_steps=0),
           dict(mu0_override=-3.0)]
    for kw in bad:
        p = ct.make_params(Sensor(**kw))
        with pytest.raises(ct.CtError) as e:
            ct.ct_init_sensor(p)
        assert e.value.status == -1, kw
    p = ct.make_params(Sensor())
    p.abi_version = 99
    with pytest.raises(ct.CtError) as e:
        ct.ct_init_sensor(p)
    assert e.value.status == -1
    for bits in (2, 16, 1 << 20):  # only CT_OPT_TIMING, CT_OPT_AUTOTUNE and CT_OPT_ONE_SIDED exist
        p = ct.make_params(Sensor())
        p.options = bits
        with pytest.raises(ct.CtError) as e:
            ct.ct_init_sensor(p)
        assert e.value.status == -1, bits


def test_carrier_counts_follow_algorithm1(ct):
    """N = round(1000 E / w) (Algorithm 1) as the library derives it."""
    import json
    from workloads import Batch, Sensor
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "alg1_init.json")))
    for case in g["carrier_count"]:
        p = ct.make_params(Sensor(pair_energy_ev=case["w_ev"]))
        b = Batch([case["E_kev"]], [0], [1.0], [1], [[0, 0, 10]])
        assert ct.ct_event_carriers(p, ct.EventDescs(b))[0] == case["N"]


def test_workspace_bytes_grow_with_batch(ct):
    from workloads import batch_8kev
    s, b = batch_8kev(n_events=16)
    p = ct.make_params(s)
    small = ct.ct_workspace_bytes(p, ct.EventDescs(b.head(4)))
    big = ct.ct_workspace_bytes(p, ct.EventDescs(b))
    assert 0 < small < big
    assert big >= 16 * 2222 * (6 * 8 + 3 * 8)  # positions twice + endpoints, FP64


def test_invalid_events_rejected(ct):
    from workloads import Batch, Sensor
    p = ct.make_params(Sensor())
    b = Batch([8.0], [10], [1.0], [1], [[0, 0, 10]])
    d = ct.EventDescs(b)
    d.arr[0].deposits = None
    with pytest.raises(ct.CtError) as e:
        ct.ct_event_carriers(p, d)
    assert e.value.status == -1


def test_track_events_validated_on_the_host(ct):
    """A track (seg_len_um > 0) lists one start point and n_deposits >= 1
    segments; a negative or non-finite length is rejected, as is a track
    with no segment."""
    from workloads import Batch, Sensor, track_walks
    s, b = track_walks(n_events=3, n_segments=40)
    p = ct.make_params(s)
    assert list(ct.ct_event_carriers(p, ct.EventDescs(b))) == [55556] * 3
    # the workspace holds the 40 deposits of each track, not just its start
    flat = Batch(b.energy_kev, b.n_carriers, b.sigma_um, b.n_deposits, np.zeros((120, 3)))
    assert ct.ct_workspace_bytes(p, ct.EventDescs(b)) >= ct.ct_workspace_bytes(p, ct.EventDescs(flat))
    for bad in (-1.0, float("inf"), float("nan")):
        d = ct.EventDescs(b)
        d.arr[1].seg_len_um = bad
        with pytest.raises(ct.CtError) as e:
            ct.ct_event_carriers(p, d)
        assert e.value.status == -1 and "seg_len_um" in str(e.value), bad
    d = ct.EventDescs(Batch([10.0], [5], [0.0], [1], [[0, 0, 10.0]]))
    d.arr[0].n_deposits = 0
    d.arr[0].seg_len_um = 5.0
    with pytest.raises(ct.CtError) as e:
        ct.ct_event_carriers(p, d)
    assert e.value.status == -1
