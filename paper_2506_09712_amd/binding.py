"""ctypes binding of libct.so (include/ct.h).

The functions keep the C names (ct_init_sensor, ct_seed_events, ct_step,
ct_collect, ...); this module only marshals arguments.  PyTorch, when it is
importable, provides the HIP stream and the device workspace; every step of
the simulation runs in the library's HIP kernels.  There is no fallback:
if libct.so is missing or no gfx950 device is present the calls fail.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional

import numpy as np

try:  # torch first, so that libct.so binds to the HIP runtime torch already loaded
    import torch  # noqa: F401
    _HAVE_TORCH = True
except Exception:  # pragma: no cover - torch is part of the image
    torch = None
    _HAVE_TORCH = False

_PKG = os.path.dirname(os.path.abspath(__file__))
# CT_LIBRARY selects another build of the same library (e.g. a variant of the
# kernels compiled with different tuning macros)
LIB_PATH = os.environ.get("CT_LIBRARY") or os.path.join(_PKG, "libct.so")

CT_ABI_VERSION = 3
CT_OK, CT_EINVAL, CT_ESTATE, CT_ENOMEM, CT_EDEVICE, CT_EMAXSTEPS, CT_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
CT_FP64, CT_FP32 = 0, 1
CT_MOB_JACOBONI, CT_MOB_CONSTANT = 0, 1
CT_REPULSION, CT_DRIFT, CT_DIFFUSION, CT_ELECTRONS, CT_SPHERICAL = 1, 2, 4, 8, 16
CT_OPT_TIMING = 1
CT_OPT_AUTOTUNE = 4
CT_OPT_ONE_SIDED = 8

_STATUS = {0: "CT_OK", -1: "CT_EINVAL", -2: "CT_ESTATE", -3: "CT_ENOMEM", -4: "CT_EDEVICE",
           -5: "CT_EMAXSTEPS", -6: "CT_ENONFINITE"}


class CtError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


class ct_sensor_params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("thickness_um", C.c_double), ("v_bias", C.c_double),
        ("v_dep", C.c_double), ("temperature_k", C.c_double), ("pitch_um", C.c_double),
        ("grid_n", C.c_int32), ("dt_ns", C.c_double), ("softening_um", C.c_double),
        ("eps_r", C.c_double), ("pair_energy_ev", C.c_double), ("mobility", C.c_int32),
        ("mu0_override", C.c_double), ("ec_override", C.c_double), ("beta_override", C.c_double),
        ("physics_flags", C.c_uint32), ("precision", C.c_int32), ("seed", C.c_uint64),
        ("max_steps", C.c_int64), ("hip_stream", C.c_void_p), ("device", C.c_int32),
        ("options", C.c_uint32), ("mu0_e_override", C.c_double), ("ec_e_override", C.c_double),
        ("beta_e_override", C.c_double),
    ]


class ct_event_desc(C.Structure):
    _fields_ = [
        ("energy_kev", C.c_double), ("n_carriers", C.c_int32), ("n_deposits", C.c_int32),
        ("sigma_um", C.c_double), ("deposits", C.POINTER(C.c_double)),
        ("xyz", C.POINTER(C.c_double)), ("ids", C.POINTER(C.c_int32)), ("start_step", C.c_int64),
        ("n_electrons", C.c_int32), ("seg_len_um", C.c_double),
    ]


class ct_gen_params(C.Structure):
    _fields_ = [
        ("energy_kev", C.c_double), ("fano", C.c_double), ("noise_kev", C.c_double),
        ("atten_um", C.c_double), ("p_alpha", C.c_double * 4), ("p_beta", C.c_double * 5),
    ]


class ct_run_stats(C.Structure):
    _fields_ = [
        ("steps", C.c_int64), ("pairs", C.c_uint64), ("n_total", C.c_int64), ("n_active", C.c_int64),
        ("field_launches", C.c_int64), ("field_kernel_ms", C.c_double), ("step_wall_ms", C.c_double),
        ("targets_per_thread", C.c_int32), ("block_size", C.c_int32), ("chunk_len", C.c_int32),
        ("workgroups", C.c_int32), ("hole_steps", C.c_uint64),
        ("newton_pairs", C.c_int32), ("reserved", C.c_int32),
    ]


EXPORTS = ["ct_init_sensor", "ct_event_carriers", "ct_workspace_bytes", "ct_bind_workspace",
           "ct_seed_events", "ct_seed_events_noalloc", "ct_step", "ct_collect", "ct_field", "ct_philox", "ct_set_launch",
           "ct_destroy", "ct_last_error", "ct_generate"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libct.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2506_09712_amd.build.build()")
    L = C.CDLL(path)
    P = C.POINTER
    st = C.c_int
    L.ct_init_sensor.argtypes = [P(ct_sensor_params), P(C.c_void_p)]
    L.ct_init_sensor.restype = st
    L.ct_event_carriers.argtypes = [P(ct_sensor_params), P(ct_event_desc), C.c_int32, P(C.c_int32)]
    L.ct_event_carriers.restype = st
    L.ct_workspace_bytes.argtypes = [P(ct_sensor_params), P(ct_event_desc), C.c_int32]
    L.ct_workspace_bytes.restype = C.c_size_t
    L.ct_bind_workspace.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    L.ct_bind_workspace.restype = st
    L.ct_seed_events.argtypes = [C.c_void_p, P(ct_event_desc), C.c_int32, C.c_uint64]
    L.ct_seed_events.restype = st
    L.ct_seed_events_noalloc.argtypes = [C.c_void_p, P(ct_event_desc), C.c_int32, C.c_uint64]
    L.ct_seed_events_noalloc.restype = st
    L.ct_step.argtypes = [C.c_void_p, C.c_int64, P(C.c_int64), P(C.c_int64)]
    L.ct_step.restype = st
    L.ct_collect.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_double), P(C.c_int32), P(C.c_int64),
                             P(ct_run_stats)]
    L.ct_collect.restype = st
    L.ct_field.argtypes = [C.c_void_p, P(C.c_double)]
    L.ct_field.restype = st
    L.ct_philox.argtypes = [C.c_void_p, P(C.c_uint32), C.c_int64, P(C.c_uint32), P(C.c_double)]
    L.ct_philox.restype = st
    L.ct_set_launch.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
    L.ct_set_launch.restype = st
    L.ct_generate.argtypes = [C.c_void_p, P(ct_gen_params), C.c_int64, C.c_uint64, C.c_void_p,
                              C.c_void_p, C.c_void_p, P(C.c_float)]
    L.ct_generate.restype = st
    L.ct_destroy.argtypes = [C.c_void_p]
    L.ct_destroy.restype = None
    L.ct_last_error.argtypes = []
    L.ct_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(status: int, where: str, allow=(CT_OK,)) -> int:
    if status not in allow:
        raise CtError(status, where, load().ct_last_error().decode(errors="replace"))
    return status


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


# ------------------------------------------------------------ marshalling

def make_params(sensor, precision: int = CT_FP64, stream=None, device: int = -1,
                options: int = 0) -> ct_sensor_params:
    flags = (CT_REPULSION if sensor.repulsion else 0) | (CT_DRIFT if sensor.drift else 0) | \
        (CT_DIFFUSION if sensor.diffusion else 0) | (CT_ELECTRONS if sensor.electrons else 0) | \
        (CT_SPHERICAL if sensor.spherical else 0)
    mob = {"jacoboni": CT_MOB_JACOBONI, "constant": CT_MOB_CONSTANT}[sensor.mobility]
    return ct_sensor_params(
        CT_ABI_VERSION, sensor.thickness_um, sensor.v_bias, sensor.v_dep, sensor.temperature_k,
        sensor.pitch_um, sensor.grid_n, sensor.dt_ns, sensor.softening_um, sensor.eps_r,
        sensor.pair_energy_ev, mob, sensor.mu0_override, sensor.ec_override, sensor.beta_override,
        flags, int(precision), int(sensor.seed), int(sensor.max_steps), stream, int(device),
        int(options), sensor.mu0_e_override, sensor.ec_e_override, sensor.beta_e_override)


class EventDescs:
    """ct_event_desc[] for a workloads.Batch, keeping its arrays alive."""

    def __init__(self, batch, ids=None):
        B = batch.n_events
        self.n = B
        self.arr = (ct_event_desc * max(B, 1))()
        self._keep = []
        doff = batch.dep_offsets()
        xo = 0
        for b in range(B):
            nd = int(batch.n_deposits[b])
            dep = np.ascontiguousarray(batch.deposits[doff[b]:doff[b + 1]]) if nd > 0 else None
            xyz = None
            if nd == 0:
                n = int(batch.n_carriers[b]) + max(int(batch.n_electrons[b]), 0)
                xyz = np.ascontiguousarray(batch.xyz[xo:xo + n])
                xo += n
            idp = None
            if ids is not None and ids[b] is not None:
                ida = np.ascontiguousarray(ids[b], dtype=np.int32)
                self._keep.append(ida)
                idp = ida.ctypes.data_as(C.POINTER(C.c_int32))
            self._keep += [dep, xyz]
            self.arr[b] = ct_event_desc(float(batch.energy_kev[b]), int(batch.n_carriers[b]), nd,
                                        float(batch.sigma_um[b]), _dp(dep), _dp(xyz), idp,
                                        int(batch.start_step[b]), int(batch.n_electrons[b]),
                                        float(batch.seg_len_um[b]))


# ------------------------------------------------------------ wrappers

def ct_init_sensor(params: ct_sensor_params) -> C.c_void_p:
    ctx = C.c_void_p()
    _check(load().ct_init_sensor(C.byref(params), C.byref(ctx)), "ct_init_sensor")
    return ctx


def ct_event_carriers(params, descs: EventDescs) -> np.ndarray:
    out = np.zeros(max(descs.n, 1), dtype=np.int32)
    _check(load().ct_event_carriers(C.byref(params), descs.arr, descs.n,
                                    out.ctypes.data_as(C.POINTER(C.c_int32))), "ct_event_carriers")
    return out[:descs.n]


def ct_workspace_bytes(params, descs: EventDescs) -> int:
    return int(load().ct_workspace_bytes(C.byref(params), descs.arr, descs.n))


def ct_bind_workspace(ctx, ptr: Optional[int], nbytes: int) -> None:
    _check(load().ct_bind_workspace(ctx, C.c_void_p(ptr) if ptr else None, int(nbytes)),
           "ct_bind_workspace")


def ct_seed_events(ctx, descs: EventDescs, first_event_id: int = 0) -> None:
    _check(load().ct_seed_events(ctx, descs.arr, descs.n, int(first_event_id)), "ct_seed_events")


def ct_seed_events_noalloc(ctx, descs: EventDescs, first_event_id: int = 0) -> None:
    _check(load().ct_seed_events_noalloc(ctx, descs.arr, descs.n, int(first_event_id)),
           "ct_seed_events_noalloc")


def ct_step(ctx, max_steps: int = 0):
    done, act = C.c_int64(0), C.c_int64(0)
    st = _check(load().ct_step(ctx, int(max_steps), C.byref(done), C.byref(act)), "ct_step",
                allow=(CT_OK, CT_EMAXSTEPS))
    return st, int(done.value), int(act.value)


def ct_collect(ctx, n_events: int, n_total: int, grid_n: int, carriers: bool = True):
    """Pixel counts, event steps and stats; with carriers=True also the
    per-carrier positions and collection steps (else those are None)."""
    G1 = grid_n * grid_n + 1
    pix = np.zeros((max(n_events, 1), G1), dtype=np.int32)
    xyz = np.zeros((max(n_total, 1), 3), dtype=np.float64) if carriers else None
    cstep = np.zeros(max(n_total, 1), dtype=np.int32) if carriers else None
    esteps = np.zeros(max(n_events, 1), dtype=np.int64)
    stats = ct_run_stats()
    _check(load().ct_collect(ctx, pix.ctypes.data_as(C.POINTER(C.c_int32)), _dp(xyz),
                             cstep.ctypes.data_as(C.POINTER(C.c_int32)) if carriers else None,
                             esteps.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(stats)),
           "ct_collect")
    if carriers:
        xyz, cstep = xyz[:n_total], cstep[:n_total]
    return pix[:n_events], xyz, cstep, esteps[:n_events], stats


def ct_field(ctx, n_total: int) -> np.ndarray:
    E = np.zeros((max(n_total, 1), 3), dtype=np.float64)
    _check(load().ct_field(ctx, _dp(E)), "ct_field")
    return E[:n_total]


def ct_philox(ctx, counters: np.ndarray):
    ctr = np.ascontiguousarray(counters, dtype=np.uint32).reshape(-1, 4)
    n = ctr.shape[0]
    words = np.zeros((max(n, 1), 4), dtype=np.uint32)
    normals = np.zeros((max(n, 1), 3), dtype=np.float64)
    _check(load().ct_philox(ctx, ctr.ctypes.data_as(C.POINTER(C.c_uint32)), n,
                            words.ctypes.data_as(C.POINTER(C.c_uint32)), _dp(normals)), "ct_philox")
    return words[:n], normals[:n]


def ct_set_launch(ctx, targets_per_thread: int = 0, block_size: int = 0, chunk_len: int = 0) -> None:
    _check(load().ct_set_launch(ctx, int(targets_per_thread), int(block_size), int(chunk_len)),
           "ct_set_launch")


def make_gen_params(gen) -> ct_gen_params:
    """ct_gen_params from an object with energy_kev, fano, noise_kev, atten_um,
    p_alpha[4], p_beta[5]."""
    return ct_gen_params(float(gen.energy_kev), float(gen.fano), float(gen.noise_kev),
                         float(gen.atten_um), (C.c_double * 4)(*map(float, gen.p_alpha)),
                         (C.c_double * 5)(*map(float, gen.p_beta)))


def ct_generate(ctx, gen, n_events: int, first_event_id: int, energy_ptr: int, counts_ptr: int,
                info_ptr: int, timed: bool = False) -> Optional[float]:
    """Queue the generation of n_events events into caller-owned device
    buffers (raw pointers, 0 = not wanted); with timed, wait and return the
    kernel's duration in ms."""
    ms = C.c_float(0.0)
    g = make_gen_params(gen)
    _check(load().ct_generate(ctx, C.byref(g), int(n_events), int(first_event_id),
                              C.c_void_p(energy_ptr or None), C.c_void_p(counts_ptr or None),
                              C.c_void_p(info_ptr or None), C.byref(ms) if timed else None),
           "ct_generate")
    return float(ms.value) if timed else None


def generate(sensor, gen, n_events: int, first_event_id: int = 0, device: int = 0) -> dict:
    """Generate events on the GPU into torch buffers and return them as numpy
    arrays: energy [n, G^2], counts [n, G^2 + 1], and h, t, n, x0, y0 [n]."""
    if not _HAVE_TORCH:
        raise RuntimeError("generate() allocates its output with torch")
    G = sensor.grid_n
    dev = f"cuda:{device}"
    torch.cuda.set_device(device)
    energy = torch.empty((n_events, G * G), dtype=torch.float64, device=dev)
    counts = torch.empty((n_events, G * G + 1), dtype=torch.int32, device=dev)
    info = torch.empty((n_events, 5), dtype=torch.float64, device=dev)
    params = make_params(sensor, CT_FP64, stream=torch.cuda.current_stream(device).cuda_stream,
                         device=device)
    ctx = ct_init_sensor(params)
    try:
        ct_generate(ctx, gen, n_events, first_event_id, energy.data_ptr(), counts.data_ptr(),
                    info.data_ptr())
        torch.cuda.synchronize(device)
    finally:
        ct_destroy(ctx)
    inf = info.cpu().numpy()
    return {"energy": energy.cpu().numpy(), "counts": counts.cpu().numpy().astype(np.int64),
            "h": inf[:, 0], "t": inf[:, 1], "n": inf[:, 2].astype(np.int64), "x0": inf[:, 3],
            "y0": inf[:, 4]}


def ct_destroy(ctx) -> None:
    if ctx:
        load().ct_destroy(ctx)


# ------------------------------------------------------------ convenience

class Simulator:
    """One context: seed a batch, step it to completion, collect results.

    With use_torch=True (default when a GPU is visible to torch) the context
    runs on torch's current HIP stream and its device workspace is a torch
    allocation bound with ct_bind_workspace.
    """

    def __init__(self, sensor, precision: int = CT_FP64, device: int = 0,
                 use_torch: Optional[bool] = None,
                 options: int = 0, launch: Optional[tuple] = None):
        self.sensor = sensor
        self.precision = precision
        if use_torch is None:
            use_torch = _HAVE_TORCH and torch.cuda.is_available()
        self.use_torch = use_torch
        stream = None
        if use_torch:
            torch.cuda.set_device(device)
            stream = torch.cuda.current_stream(device).cuda_stream
        self.params = make_params(sensor, precision, stream=stream, device=device, options=options)
        self.ctx = ct_init_sensor(self.params)
        self._ws = None
        self._descs = None
        self._descs_of = None
        if launch:
            ct_set_launch(self.ctx, *launch)
        self.batch = None

    def close(self):
        if self.ctx:
            ct_destroy(self.ctx)
            self.ctx = None
        self._ws = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, targets_per_thread=0, block_size=0, chunk_len=0):
        ct_set_launch(self.ctx, targets_per_thread, block_size, chunk_len)

    def seed(self, batch, ids=None, noalloc: bool = False):
        if ids is None and self._descs is not None and self._descs_of is batch:
            descs = self._descs  # same batch object: reuse its marshalled descriptions
        else:
            descs = EventDescs(batch, ids)
        self.counts = ct_event_carriers(self.params, descs)
        if self.use_torch:
            nbytes = ct_workspace_bytes(self.params, descs) + (1 << 20)
            if self._ws is None or self._ws.numel() < nbytes:
                ct_bind_workspace(self.ctx, None, 0)
                self._ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.params.device}")
            ct_bind_workspace(self.ctx, self._ws.data_ptr(), self._ws.numel())
        (ct_seed_events_noalloc if noalloc else ct_seed_events)(self.ctx, descs, batch.first_event_id)
        self.batch = batch
        self.n_total = int(self.counts.sum())
        self._descs = descs
        self._descs_of = batch if ids is None else None

    def step(self, max_steps: int = 0):
        return ct_step(self.ctx, max_steps)

    def collect(self, carriers: bool = True) -> dict:
        pix, xyz, cstep, esteps, stats = ct_collect(self.ctx, self.batch.n_events, self.n_total,
                                                    self.sensor.grid_n, carriers)
        off = np.zeros(self.batch.n_events + 1, dtype=np.int64)
        np.cumsum(self.counts, out=off[1:])
        return {"pix": pix, "xyz": xyz, "cstep": cstep, "steps": esteps, "pairs": int(stats.pairs),
                "hole_steps": int(stats.hole_steps),
                "stats": stats, "offsets": off, "n": self.counts.astype(np.int64)}

    def field(self) -> np.ndarray:
        return ct_field(self.ctx, self.n_total)

    def run(self, batch, max_steps: int = 0) -> dict:
        self.seed(batch)
        st, done, act = self.step(max_steps)
        r = self.collect()
        r["status"] = st
        return r


def run(sensor, batch, precision: int = CT_FP64, max_steps: int = 0, **kw) -> dict:
    """Simulate a batch to completion (or max_steps) and return host results."""
    with Simulator(sensor, precision, **kw) as sim:
        return sim.run(batch, max_steps)
