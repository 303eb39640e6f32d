"""ctypes wrapper of the FP64 CPU oracle (``ct_oracle.c``).

Test infrastructure only: the test suite, the smoke check and the CPU
baseline leg of the benchmark load it.  It never imports the library package
and the library never imports it; both consume the seeded inputs of
``workloads``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ct_oracle.c")
_LIB = os.path.join(_HERE, "libct_oracle.so")

OK, EINVAL, EMAXSTEPS, ENONFINITE = 0, -1, -5, -6
REPULSION, DRIFT, DIFFUSION, ELECTRONS, SPHERICAL = 1, 2, 4, 8, 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE FP64: no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OcParams(C.Structure):
    _fields_ = [
        ("thickness_um", C.c_double), ("v_bias", C.c_double), ("v_dep", C.c_double),
        ("temperature_k", C.c_double), ("pitch_um", C.c_double), ("grid_n", C.c_int32),
        ("dt_ns", C.c_double), ("softening_um", C.c_double), ("eps_r", C.c_double),
        ("pair_energy_ev", C.c_double), ("mobility", C.c_int32),
        ("mu0_override", C.c_double), ("ec_override", C.c_double), ("beta_override", C.c_double),
        ("physics", C.c_uint32), ("seed", C.c_uint64), ("max_steps", C.c_int64),
        ("mu0_e_override", C.c_double), ("ec_e_override", C.c_double),
        ("beta_e_override", C.c_double),
    ]


class OcEvent(C.Structure):
    _fields_ = [
        ("energy_kev", C.c_double), ("n_carriers", C.c_int32), ("n_deposits", C.c_int32),
        ("sigma_um", C.c_double), ("deposits", C.POINTER(C.c_double)),
        ("xyz", C.POINTER(C.c_double)), ("ids", C.POINTER(C.c_int32)), ("start_step", C.c_int64),
        ("n_electrons", C.c_int32), ("seg_len_um", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        dp, ip, up = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_uint32)
        L.oc_philox4x32_10.argtypes = [up, up, up]
        L.oc_normals3.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, dp]
        L.oc_philox_many.argtypes = [C.c_uint64, C.c_int64, up, up]
        L.oc_normals_many.argtypes = [C.c_uint64, C.c_int64, up, dp]
        L.oc_coulomb_k.argtypes = [C.POINTER(OcParams)]
        L.oc_coulomb_k.restype = C.c_double
        L.oc_thermal_voltage.argtypes = [C.POINTER(OcParams)]
        L.oc_thermal_voltage.restype = C.c_double
        L.oc_mobility_params.argtypes = [C.POINTER(OcParams), dp]
        L.oc_mobility_params_of.argtypes = [C.POINTER(OcParams), C.c_int, dp]
        L.oc_mobility_of.argtypes = [C.POINTER(OcParams), C.c_int, C.c_double]
        L.oc_mobility_of.restype = C.c_double
        L.oc_field_spherical.argtypes = [C.POINTER(OcParams), C.c_int64, dp, dp]
        L.oc_field_q.argtypes = [C.POINTER(OcParams), C.c_int64, dp, dp, dp]
        L.oc_electron_count.argtypes = [C.POINTER(OcParams), C.POINTER(OcEvent)]
        L.oc_electron_count.restype = C.c_int32
        L.oc_mobility.argtypes = [C.POINTER(OcParams), C.c_double]
        L.oc_mobility.restype = C.c_double
        L.oc_drift_field.argtypes = [C.POINTER(OcParams), C.c_double]
        L.oc_drift_field.restype = C.c_double
        L.oc_field.argtypes = [C.POINTER(OcParams), C.c_int64, dp, dp]
        L.oc_field_targets.argtypes = [C.POINTER(OcParams), C.c_int64, dp, C.c_int64,
                                       C.POINTER(C.c_int64), dp]
        L.oc_carrier_count.argtypes = [C.POINTER(OcParams), C.POINTER(OcEvent)]
        L.oc_carrier_count.restype = C.c_int32
        L.oc_track_deposits.argtypes = [C.POINTER(OcParams), C.POINTER(OcEvent), C.c_uint64, dp]
        L.oc_track_deposits.restype = None
        L.oc_initial_sigma.argtypes = [C.POINTER(OcEvent)]
        L.oc_initial_sigma.restype = C.c_double
        L.oc_pixel_bin.argtypes = [C.POINTER(OcParams), C.c_double, C.c_double]
        L.oc_pixel_bin.restype = C.c_int32
        L.oc_run.argtypes = [C.POINTER(OcParams), C.POINTER(OcEvent), C.c_int32, C.c_uint64,
                             ip, dp, ip, C.POINTER(C.c_int64), C.POINTER(C.c_uint64),
                             C.POINTER(C.c_uint64)]
        L.oc_run.restype = C.c_int
        L.oc_set_threads.argtypes = [C.c_int]
        L.oc_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def params(sensor) -> OcParams:
    flags = (REPULSION if sensor.repulsion else 0) | (DRIFT if sensor.drift else 0) | \
            (DIFFUSION if sensor.diffusion else 0) | (ELECTRONS if sensor.electrons else 0) | \
            (SPHERICAL if sensor.spherical else 0)
    mob = {"jacoboni": 0, "constant": 1}[sensor.mobility]
    return OcParams(sensor.thickness_um, sensor.v_bias, sensor.v_dep, sensor.temperature_k,
                    sensor.pitch_um, sensor.grid_n, sensor.dt_ns, sensor.softening_um, sensor.eps_r,
                    sensor.pair_energy_ev, mob, sensor.mu0_override, sensor.ec_override,
                    sensor.beta_override, flags, sensor.seed, sensor.max_steps,
                    sensor.mu0_e_override, sensor.ec_e_override, sensor.beta_e_override)


def set_threads(n: int) -> None:
    lib().oc_set_threads(int(n))


def threads() -> int:
    return int(lib().oc_get_threads())


def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().oc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def normals3(seed: int, c0: int, c1: int, c2: int, c3: int) -> np.ndarray:
    o = (C.c_double * 3)()
    lib().oc_normals3(seed, c0, c1, c2, c3, o)
    return np.array(list(o))


def philox_many(seed: int, ctr: np.ndarray) -> np.ndarray:
    """Philox4x32-10 blocks [n, 4] for counters [n, 4] under a 64-bit seed."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().oc_philox_many(int(seed), ctr.shape[0], ctr.ctypes.data_as(C.POINTER(C.c_uint32)),
                         out.ctypes.data_as(C.POINTER(C.c_uint32)))
    return out


def normals_many(seed: int, ctr: np.ndarray) -> np.ndarray:
    """Box-Muller normals [n, 3] for counters [n, 4]."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty((ctr.shape[0], 3))
    lib().oc_normals_many(int(seed), ctr.shape[0], ctr.ctypes.data_as(C.POINTER(C.c_uint32)),
                          _dp(out))
    return out


def coulomb_k(sensor) -> float:
    return float(lib().oc_coulomb_k(C.byref(params(sensor))))


def thermal_voltage(sensor) -> float:
    return float(lib().oc_thermal_voltage(C.byref(params(sensor))))


def mobility_params(sensor, electron: bool = False) -> tuple:
    """(mu0 [um^2/(V ns)], Ec [V/um], beta) of holes or electrons."""
    o = (C.c_double * 3)()
    lib().oc_mobility_params_of(C.byref(params(sensor)), int(electron), o)
    return tuple(o)


def mobility(sensor, e_mag: float, electron: bool = False) -> float:
    return float(lib().oc_mobility_of(C.byref(params(sensor)), int(electron), float(e_mag)))


def drift_field(sensor, z: float) -> float:
    return float(lib().oc_drift_field(C.byref(params(sensor)), float(z)))


def pixel_bin(sensor, x: float, y: float) -> int:
    return int(lib().oc_pixel_bin(C.byref(params(sensor)), float(x), float(y)))


def field(sensor, xyz: np.ndarray) -> np.ndarray:
    """Repulsion field (V/um) of the carriers at xyz [n, 3] on each other."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    E = np.zeros_like(xyz)
    lib().oc_field(C.byref(params(sensor)), xyz.shape[0], _dp(xyz), _dp(E))
    return E


def field_q(sensor, xyz: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Field (V/um) of carriers with charges q (+1 hole, -1 electron) on each other."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    E = np.zeros_like(xyz)
    lib().oc_field_q(C.byref(params(sensor)), xyz.shape[0], _dp(xyz), _dp(q), _dp(E))
    return E


def field_spherical(sensor, xyz: np.ndarray) -> np.ndarray:
    """Eq. 7 field (V/um) of the holes at xyz [n, 3] on each other: the holes
    strictly closer to their mean position, concentrated there."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    E = np.zeros_like(xyz)
    lib().oc_field_spherical(C.byref(params(sensor)), xyz.shape[0], _dp(xyz), _dp(E))
    return E


def field_at(sensor, xyz: np.ndarray, targets) -> np.ndarray:
    """Repulsion field on the listed carriers only ([len(targets), 3])."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(targets, dtype=np.int64)
    E = np.zeros((len(t), 3))
    lib().oc_field_targets(C.byref(params(sensor)), xyz.shape[0], _dp(xyz), len(t),
                           t.ctypes.data_as(C.POINTER(C.c_int64)), _dp(E))
    return E


def _events(batch):
    B = batch.n_events
    evs = (OcEvent * max(B, 1))()
    doff = batch.dep_offsets()
    xo = 0
    keep = []
    for b in range(B):
        nd = int(batch.n_deposits[b])
        dep = np.ascontiguousarray(batch.deposits[doff[b]:doff[b + 1]]) if nd > 0 else None
        xyz = None
        if nd == 0:
            n = int(batch.n_carriers[b]) + max(int(batch.n_electrons[b]), 0)
            xyz = np.ascontiguousarray(batch.xyz[xo:xo + n])
            xo += n
        keep += [dep, xyz]
        evs[b] = OcEvent(float(batch.energy_kev[b]), int(batch.n_carriers[b]), nd,
                         float(batch.sigma_um[b]), _dp(dep), _dp(xyz), None,
                         int(batch.start_step[b]), int(batch.n_electrons[b]),
                         float(batch.seg_len_um[b]))
    return evs, keep


def track_deposits(sensor, batch, b: int = 0) -> np.ndarray:
    """The deposits of track event b ([n_deposits, 3]): the midpoints of the
    walk the oracle draws from the event's start point."""
    evs, keep = _events(batch)
    out = np.zeros((int(batch.n_deposits[b]), 3))
    lib().oc_track_deposits(C.byref(params(sensor)), C.byref(evs[b]),
                            C.c_uint64(batch.first_event_id + b), _dp(out))
    return out


def hole_counts(sensor, batch) -> np.ndarray:
    evs, keep = _events(batch)
    p = params(sensor)
    return np.array([lib().oc_carrier_count(C.byref(p), C.byref(evs[b]))
                     for b in range(batch.n_events)], dtype=np.int64)


def electron_counts(sensor, batch) -> np.ndarray:
    evs, keep = _events(batch)
    p = params(sensor)
    return np.array([lib().oc_electron_count(C.byref(p), C.byref(evs[b]))
                     for b in range(batch.n_events)], dtype=np.int64)


def carrier_counts(sensor, batch) -> np.ndarray:
    """Carriers of each event: its holes and (with the electron species) electrons."""
    return np.maximum(hole_counts(sensor, batch), 0) + np.maximum(electron_counts(sensor, batch), 0)


def initial_sigma(batch, b: int = 0) -> float:
    evs, keep = _events(batch)
    return float(lib().oc_initial_sigma(C.byref(evs[b])))


def run(sensor, batch, threads: Optional[int] = None) -> dict:
    """Simulate every event of the batch; returns the oracle's outputs."""
    if threads is not None:
        set_threads(threads)
    p = params(sensor)
    evs, keep = _events(batch)
    n = carrier_counts(sensor, batch)
    off = np.zeros(batch.n_events + 1, dtype=np.int64)
    np.cumsum(np.maximum(n, 0), out=off[1:])
    G1 = sensor.grid_n * sensor.grid_n + 1
    pix = np.zeros((batch.n_events, G1), dtype=np.int32)
    xyz = np.zeros((int(off[-1]), 3), dtype=np.float64)
    cstep = np.zeros(int(off[-1]), dtype=np.int32)
    steps = np.zeros(batch.n_events, dtype=np.int64)
    pairs, hsteps = C.c_uint64(0), C.c_uint64(0)
    st = lib().oc_run(C.byref(p), evs, batch.n_events, batch.first_event_id,
                      pix.ctypes.data_as(C.POINTER(C.c_int32)), _dp(xyz),
                      cstep.ctypes.data_as(C.POINTER(C.c_int32)),
                      steps.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(pairs), C.byref(hsteps))
    return {"status": int(st), "pix": pix, "xyz": xyz, "cstep": cstep, "steps": steps,
            "pairs": int(pairs.value), "hole_steps": int(hsteps.value), "offsets": off, "n": n,
            "n_holes": np.maximum(hole_counts(sensor, batch), 0)}
