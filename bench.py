"""Throughput of the batched repulsion Monte Carlo on one MI355X.

One bench step = one whole batch simulated to completion through the C ABI:
seeding of every event's initial cloud on the device, the time-step loop
(all-pairs repulsion, drift, diffusion, collection, pixel integration,
compaction) until every hole is collected, and the pixel counts copied back.

Printed as one JSON line: pair-interactions/s of the FP32-batched path
(value), events/s, the FP64-plain comparison (one event at a time, FP64
field), the roofline of the repulsion-step kernel (timed with HIP events on
the library's stream) and the FP64 CPU oracle timed on a bounded sample.

--model spherical measures the simplified spherical model (Sec. 2.2, Eq. 7)
on the same workload instead: events/s (value) and hole updates/s, the
roofline of its kernel against HBM bandwidth, and the oracle's spherical
model on a bounded sample.

--model generator measures the parameterised event generation (Sec. 4.2) on
its own workload (one million 25 keV events): events/s (value) and carriers
placed per second, the roofline of its kernel against the VALU issue rate,
and the oracle's generator on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "pair-interactions/s + events/s, FP32-batched vs FP64-plain at ≤1e-3 pixel-fraction err"
METRIC_SPHERICAL = "events/s + hole-updates/s, simplified spherical model (Eq. 7), FP64"
METRIC_GENERATOR = "events/s + carriers/s, parameterised event generation (Sec. 4.2)"
# VALU issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = one vector operation
# per lane per clock
VALU_OP_PEAK = 256 * 64 * 2.4e9
# Algorithmic vector operations per generated carrier: half a Philox4x32-10
# block (10 rounds of 2 low and 2 high 32-bit products and 4 XORs per two
# carriers: 40), 2 uniform conversions (4), two searches over the 6 pixel
# edges of a 5-pixel row (24 compares and adds), the pixel index and the
# histogram update (4)
OPS_PER_CARRIER = 72
FP32_VECTOR_PEAK = 157.3e12   # MI355X FP32 vector FLOP/s (256 CU x 128 lanes x 2 (FMA) x 2.4 GHz)
# Issue slots of one pair: 11 one-slot FP32 instructions and a v_rsq_f32 at a
# quarter of their rate; at 128 lanes per CU per clock and 2.4 GHz that bounds
# the pair loop at 256 * 128 * 2.4e9 / 15 pairs/s.
SLOTS_PER_PAIR = 15
# The Newton-pair kernel takes each unordered pair once for both holes: 3 sub,
# 3 FMA, v_rsq (4 slots), 2 mul, 3 + 3 FMA and 3 DPP lane moves = 21 slots
# for two ordered pairs (within a tile too; the parked slots of ragged tiles
# cost the same and count for nothing).
# Executed FLOP: 24 per unordered pair (FMA as 2, rsqrt as 1), 12 per ordered.
NEWTON_SLOTS_PER_PAIR = 10.5
NEWTON_EXECUTED_FLOP_PER_PAIR = 12
ISSUE_SLOTS_PER_S = 256 * 128 * 2.4e9
HBM_PEAK = 8.0e12             # MI355X HBM3E bytes/s
FLOP_PER_PAIR = 20            # N-body convention for one softened pair interaction


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch_8kev")
    ap.add_argument("--model", choices=("pairs", "spherical", "generator"), default="pairs",
                    help="pairs: the brute-force field (Eq. 4); spherical: Eq. 7; generator: "
                         "the parameterised events of Sec. 4.2")
    ap.add_argument("--events", type=int, default=0, help="override the number of events")
    ap.add_argument("--plain-events", type=int, default=32,
                    help="events of the FP64-plain comparison (rate extrapolated)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--launch", default="", help="targets_per_thread,block,chunk_len override")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time launch shapes on the seeded state")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first copy this many MiB device-to-device with torch (a reference "
                         "kernel of known traffic for hardware byte counters)")
    return ap.parse_args()


# Algorithmic HBM bytes of one hole update in the step kernel: the hole's
# FP64 position (24 B) and carrier index (4 B) read, its RNG id (4 B) read,
# the new FP64 position (24 B) written.  Sources are re-reads of the same
# event's positions, served from cache.
ALG_BYTES_PER_HOLE_STEP = 56
CSRC = os.path.join(ROOT, "paper_2506_09712_amd", "csrc")
# the sources each kernel is built from, and its committed counter summary
KERNEL_SOURCES = {
    "pairs": ("ct_kernels.hip", "ct_device.hpp", "ct_internal.hpp"),
    "spherical": ("ct_sph.hip", "ct_sph_layout.hpp", "ct_device.hpp", "ct_internal.hpp"),
    "generator": ("ct_gen.hip", "ct_device.hpp", "ct_internal.hpp"),
}
TRAFFIC_PROFILES = {
    "pairs": os.path.join(ROOT, "profiles", "k_run_newton_batch_8kev_traffic.md"),
    "spherical": os.path.join(ROOT, "profiles", "k_sph_batch_8kev_traffic.md"),
    "generator": os.path.join(ROOT, "profiles", "k_gen_generator_25kev_traffic.md"),
}


def sources_digest(model):
    """SHA-256 of the kernel's source files, concatenated in a fixed order."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[model]:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def measured_traffic(model, units_per_launch):
    """HBM bytes per kernel launch from the committed rocprofv3 counter
    summary (bytes per hole update; per event for the generator), or None when
    the kernel's sources have changed since the counters were taken."""
    path = TRAFFIC_PROFILES[model]
    try:
        text = open(path).read()
    except OSError:
        return None, "no counter summary"
    unit = "bytes_per_event" if model == "generator" else "bytes_per_hole_step"
    vals = dict(line.split(":", 1) for line in text.splitlines()
                if line.startswith((unit + ":", "kernel_sources_sha256:")))
    if vals.get("kernel_sources_sha256", "").strip() != sources_digest(model):
        return None, "kernel changed since the counters were taken"
    per = float(vals[unit])
    return per * units_per_launch, ("FETCH_SIZE and WRITE_SIZE per unit of work, scaled by a "
                                     "1 GiB copy; " + os.path.basename(path))


def simulate(ct, sim, batch):
    """Seed, step to completion, copy back pixel counts and run statistics."""
    sim.seed(batch)
    st, done, act = sim.step(0)
    if st != 0:
        raise RuntimeError(f"batch did not finish: status {st}, {act} holes left")
    return sim.collect(carriers=False)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not "
                                   "supported (events shard with no per-step exchange)",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    import paper_2506_09712_amd as ct
    from workloads import make_workload

    kw = {"n_events": a.events} if a.events else {}
    if a.model == "generator":
        return generator(a, ct, torch, kw)
    sensor, batch = make_workload(a.workload, **kw)
    launch = tuple(int(v) for v in a.launch.split(",")) if a.launch else None
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    n_holes = int(batch.n_carriers.sum())
    n_carriers = n_holes * (2 if sensor.electrons else 1)
    species = "holes and electrons" if sensor.electrons else "holes"
    print(f"bench: {a.workload} {batch.n_events} events, {n_carriers} carriers ({species}); "
          f"warmup {a.warmup}, steps {a.steps}", file=sys.stderr, flush=True)
    if a.copy_calibration_mb:
        n = a.copy_calibration_mb << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"bench: calibration copy of {a.copy_calibration_mb} MiB done", file=sys.stderr,
              flush=True)
        del src, dst

    if a.model == "spherical":
        return spherical(a, ct, torch, sensor, batch, n_holes)
    tune = ct.CT_OPT_AUTOTUNE if (a.autotune and not launch) else 0

    def timed_runs(label, extra=0):
        # HIP events around the one step-kernel run of each ct_step call
        sim = ct.Simulator(sensor, ct.CT_FP32, device=0, options=ct.CT_OPT_TIMING | tune | extra,
                           launch=launch)
        for _ in range(a.warmup):
            simulate(ct, sim, batch)
        torch.cuda.synchronize()
        pairs, kern_ms, launches, hsteps = 0, 0.0, 0, 0
        t0 = time.perf_counter()
        for _ in range(a.steps):
            r = simulate(ct, sim, batch)
            pairs += r["pairs"]
            hsteps += r["hole_steps"]
            kern_ms += r["stats"].field_kernel_ms
            launches += r["stats"].field_launches
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = r["stats"]
        sim.close()
        print(f"bench: {label}: {pairs / wall:.3e} pairs/s, {batch.n_events * a.steps / wall:.1f} "
              f"events/s", file=sys.stderr, flush=True)
        return pairs, wall, kern_ms, launches, st, hsteps

    pairs, wall, kern_ms, launches, st, hsteps = timed_runs("fp32-batched")
    value = pairs / wall
    events_per_s = batch.n_events * a.steps / wall
    traffic, traffic_note = measured_traffic("pairs", hsteps / max(launches, 1))
    achieved = FLOP_PER_PAIR * pairs / (kern_ms * 1e-3) if kern_ms > 0 else None
    newton = bool(st.newton_pairs)
    slots = NEWTON_SLOTS_PER_PAIR if newton else SLOTS_PER_PAIR
    executed = (NEWTON_EXECUTED_FLOP_PER_PAIR if newton else FLOP_PER_PAIR) * pairs / (kern_ms * 1e-3) \
        if kern_ms > 0 else None
    print(f"bench: step kernel {kern_ms / max(launches, 1):.3f} ms avg over {launches} launches, "
          f"{achieved / 1e12 if achieved else 0:.1f} TFLOP/s", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": value, "unit": "pair-interactions/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * wall / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {batch.n_events} events, "
                               f"{n_carriers} carriers ({species}), "
                               f"{sensor.thickness_um:g} um Si at {sensor.v_bias:g} V, "
                               f"dt {sensor.dt_ns:g} ns; FP32 field, FP64 state; one "
                               f"persistent step kernel per run, events stepped "
                               f"independently through a device work queue",
                   "events": batch.n_events, "holes": n_holes, "carriers": n_carriers,
                   "launch": {"targets_per_thread": st.targets_per_thread,
                              "block": st.block_size, "chunk_len": st.chunk_len,
                              "workgroups": st.workgroups}},
        "events_per_s": events_per_s,
        "pairs_per_run": pairs // a.steps,
        "hole_steps_per_run": hsteps // a.steps,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12 if achieved else None,
                     "peak": FP32_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK if achieved else None,
                     "traffic": traffic, "traffic_note": traffic_note,
                     "algorithmic_bytes_per_launch": ALG_BYTES_PER_HOLE_STEP * hsteps / max(launches, 1),
                     "hole_steps_per_launch": hsteps / max(launches, 1),
                     "kernel": f"k_run_newton<256, {'true' if n_carriers != n_holes else 'false'}>" if newton else
                               f"k_run_f32<{st.targets_per_thread},{st.block_size}>",
                     "pair_evaluation": "each unordered pair once, applied to both holes" if newton
                                        else "every ordered pair",
                     "avg_launch_ms": kern_ms / max(launches, 1),
                     "launches": launches, "flop_per_pair": FLOP_PER_PAIR,
                     "executed_tflops": executed / 1e12 if executed else None,
                     "executed_frac": executed / FP32_VECTOR_PEAK if executed else None,
                     "slots_per_pair": slots,
                     "frac_of_issue_bound": (pairs / (kern_ms * 1e-3)) / (ISSUE_SLOTS_PER_S / slots)
                     if kern_ms > 0 else None},
    }

    if not a.no_plain:
        # FP64-plain: the same events one at a time with the FP64 field; plus the
        # other two corners of precision x batching so the speedup is attributable
        n_plain = min(a.plain_events, batch.n_events)

        def rate(prec, plain):
            # one event at a time: the autotuner's launch for a single event
            # (short chunks, more work items per step) unless one is pinned
            opts = ct.CT_OPT_AUTOTUNE if (plain and not launch) else tune
            sim = ct.Simulator(sensor, prec, device=0, options=opts)
            evs = [batch.event(e) for e in range(n_plain)] if plain else [batch]
            simulate(ct, sim, evs[0])
            torch.cuda.synchronize()
            pp, t1 = 0, time.perf_counter()
            for ev in evs:
                pp += simulate(ct, sim, ev)["pairs"]
            torch.cuda.synchronize()
            w = time.perf_counter() - t1
            sim.close()
            return pp / w, (n_plain if plain else batch.n_events) / w

        p64, e64 = rate(ct.CT_FP64, True)
        out["fp64_plain"] = {"value": p64, "unit": "pair-interactions/s", "events_per_s": e64,
                             "events": n_plain}
        out["speedup_fp32_batched_vs_fp64_plain"] = value / p64
        b64, be64 = rate(ct.CT_FP64, False)
        p32, pe32 = rate(ct.CT_FP32, True)
        out["ablation"] = {"fp32_batched": value, "fp64_batched": b64, "fp32_plain": p32,
                           "fp64_plain": p64, "unit": "pair-interactions/s",
                           "plain_events": n_plain}
        if newton:
            p1, w1 = timed_runs("fp32-batched, every ordered pair", ct.CT_OPT_ONE_SIDED)[:2]
            out["ablation"]["fp32_batched_one_sided"] = p1 / w1
        print(f"bench: fp64-plain {p64:.3e}, fp64-batched {b64:.3e}, fp32-plain {p32:.3e} pairs/s",
              file=sys.stderr, flush=True)

    if not a.no_cpu_baseline:
        # endpoints of one more (untimed) run in each precision, for the error
        # of the GPU results against the oracle on the events it simulates
        gpu_runs = {}
        for label, prec in (("fp32_batched", ct.CT_FP32), ("fp64_batched", ct.CT_FP64)):
            with ct.Simulator(sensor, prec, device=0, launch=launch) as sim:
                sim.seed(batch)
                st_, _, _ = sim.step(0)
                if st_ != 0:
                    raise RuntimeError(f"{label} run did not finish: status {st_}")
                gpu_runs[label] = sim.collect(carriers=True)
        import oracle
        oracle.build(force=False)
        cpairs, t2, k = 0, time.perf_counter(), 0
        oracle_runs = []
        while k < batch.n_events and (time.perf_counter() - t2) < a.cpu_seconds:
            o = oracle.run(sensor, batch.event(k))
            cpairs += o["pairs"]
            oracle_runs.append(o)
            k += 1
        cwall = time.perf_counter() - t2
        out["cpu_baseline"] = {"value": cpairs / cwall, "unit": "pair-interactions/s",
                               "cores": oracle.threads(), "kind": "oracle",
                               "sample": f"events 0..{k - 1} of {a.workload}, each simulated "
                                         f"to completion alone ({cpairs:.3e} pairs, {cwall:.1f} s)",
                               "events_per_s": k / cwall}
        out["error_vs_oracle"] = error_vs_oracle(gpu_runs, oracle_runs)
        print(f"bench: oracle {cpairs / cwall:.3e} pairs/s on {oracle.threads()} threads",
              file=sys.stderr, flush=True)
        e32, e64 = out["error_vs_oracle"]["fp32_batched"], out["error_vs_oracle"]["fp64_batched"]
        print(f"bench: vs oracle on {k} events: FP32 endpoints max {e32['endpoint_um_max']:.2e} / "
              f"p99 {e32['endpoint_um_p99']:.2e} / mean {e32['endpoint_um_mean']:.2e} um, pixel "
              f"fractions max {e32['pixel_fraction_max_abs']:.2e}; FP64 endpoints max "
              f"{e64['endpoint_um_max']:.2e} um", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def error_vs_oracle(gpu_runs, oracle_runs):
    """Per precision: the (x, y) endpoint error of every carrier of the
    oracle's events (max, 99th percentile, mean, um), the largest pixel charge
    fraction error, and the share of carriers with the oracle's collection
    step."""
    res = {"events": len(oracle_runs)}
    for label, g in gpu_runs.items():
        off = g["offsets"]
        d, frac, same, ncar = [], 0.0, 0, 0
        for e, o in enumerate(oracle_runs):
            sl = slice(int(off[e]), int(off[e + 1]))
            d.append(np.hypot(*(g["xyz"][sl, :2] - o["xyz"][:, :2]).T))
            n = max(int(o["pix"].sum()), 1)
            frac = max(frac, float(np.abs(g["pix"][e] - o["pix"][0]).max()) / n)
            same += int((g["cstep"][sl] == o["cstep"]).sum())
            ncar += sl.stop - sl.start
        d = np.concatenate(d) if d else np.zeros(1)
        res[label] = {"endpoint_um_max": float(d.max()), "endpoint_um_p99": float(np.percentile(d, 99)),
                      "endpoint_um_mean": float(d.mean()), "pixel_fraction_max_abs": frac,
                      "collect_step_match": same / max(ncar, 1)}
    return res


def generator(a, ct, torch, kw):
    """One ct_generate launch per step into device buffers allocated once
    (inputs are the parameters only; outputs stay in HBM)."""
    from workloads import generator_25kev
    sensor, gen, n = generator_25kev(**kw)
    G = sensor.grid_n
    dev = torch.device("cuda:0")
    print(f"bench: generator_25kev {n} events, {G}x{G} pixels; warmup {a.warmup}, steps {a.steps}",
          file=sys.stderr, flush=True)
    if a.copy_calibration_mb:
        src = torch.ones(a.copy_calibration_mb << 20, dtype=torch.uint8, device=dev)
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        print(f"bench: calibration copy of {a.copy_calibration_mb} MiB done", file=sys.stderr,
              flush=True)
        del src
    energy = torch.empty((n, G * G), dtype=torch.float64, device=dev)
    counts = torch.empty((n, G * G + 1), dtype=torch.int32, device=dev)
    info = torch.empty((n, 5), dtype=torch.float64, device=dev)
    ctx = ct.ct_init_sensor(ct.make_params(sensor, ct.CT_FP64,
                                           stream=torch.cuda.current_stream(0).cuda_stream, device=0))
    ptrs = (energy.data_ptr(), counts.data_ptr(), info.data_ptr())
    for w in range(a.warmup):
        ct.ct_generate(ctx, gen, n, w * n, *ptrs)
    torch.cuda.synchronize()
    kern_ms, carriers = 0.0, 0
    t0 = time.perf_counter()
    for k in range(a.steps):
        kern_ms += ct.ct_generate(ctx, gen, n, (a.warmup + k) * n, *ptrs, timed=True)
        carriers += int(info[:, 2].sum().item())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if not a.no_cpu_baseline:
        ct.ct_generate(ctx, gen, n, 0, *ptrs)  # events 0.. again (untimed), for the oracle check
        torch.cuda.synchronize()
    ct.ct_destroy(ctx)
    events_per_s = n * a.steps / wall
    achieved = OPS_PER_CARRIER * carriers / (kern_ms * 1e-3)
    traffic, traffic_note = measured_traffic("generator", n)
    print(f"bench: generator: {events_per_s:.4g} events/s, {carriers / wall:.4g} carriers/s; k_gen "
          f"{kern_ms / a.steps:.3f} ms avg over {a.steps} launches", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC_GENERATOR, "value": events_per_s, "unit": "events/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * wall / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"generator_25kev: {n} events of {gen.energy_kev:g} keV, "
                               f"{sensor.thickness_um:g} um Si at {sensor.v_bias:g} V, V_dep "
                               f"{sensor.v_dep:g} V, {G}x{G} pixels of {sensor.pitch_um:g} um; "
                               f"Fano {gen.fano:g}, noise {gen.noise_kev:g} keV; one ct_generate "
                               f"launch per step (one wave per event)", "events": n},
        "carriers_per_s": carriers / wall,
        "carriers_per_step": carriers // a.steps,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_OP_PEAK / 1e12,
                     "unit": "Tops/s (vector lane operations)", "frac": achieved / VALU_OP_PEAK,
                     "traffic": traffic, "traffic_note": traffic_note,
                     "ops_per_carrier": OPS_PER_CARRIER, "kernel": f"k_gen<{G}>",
                     "avg_launch_ms": kern_ms / a.steps, "launches": a.steps,
                     "algorithmic_bytes_per_launch": n * (8 * G * G + 4 * (G * G + 1) + 40)},
    }
    if not a.no_cpu_baseline:
        import oracle
        import oracle.generator as og
        oracle.build(force=False)
        k, t2, chunk = 0, time.perf_counter(), 200
        oc, oe = [], []
        while (time.perf_counter() - t2) < a.cpu_seconds and k < n:
            o = og.generate(sensor, gen, chunk, first_event_id=k)
            oc.append(o["counts"])
            oe.append(o["energy"])
            k += chunk
        cwall = time.perf_counter() - t2
        gc, ge = counts[:k].cpu().numpy(), energy[:k].cpu().numpy()
        out["error_vs_oracle"] = {
            "events": k, "counts_equal": bool(np.array_equal(gc, np.concatenate(oc))),
            "energy_kev_max_abs": float(np.abs(ge - np.concatenate(oe)).max())}
        out["cpu_baseline"] = {"value": k / cwall, "unit": "events/s", "cores": 1, "kind": "oracle",
                               "sample": f"events 0..{k - 1} of generator_25kev ({cwall:.1f} s), "
                                         f"the oracle's numpy generator on one thread"}
        print(f"bench: oracle {k / cwall:.1f} events/s", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def spherical(a, ct, torch, sensor, batch, n_holes):
    """The simplified spherical model on the same workload, FP64: per run one
    k_sph_single launch (one workgroup per event) and, for events of more than
    8192 holes, one k_sph_shared launch (a group of workgroups per event)."""
    if sensor.electrons:
        raise SystemExit("the spherical model simulates holes only")
    sensor = sensor.replace(spherical=True)
    sim = ct.Simulator(sensor, ct.CT_FP64, device=0, options=ct.CT_OPT_TIMING)
    for _ in range(a.warmup):
        simulate(ct, sim, batch)
    torch.cuda.synchronize()
    kern_ms, launches, hsteps = 0.0, 0, 0
    t0 = time.perf_counter()
    for _ in range(a.steps):
        r = simulate(ct, sim, batch)
        hsteps += r["hole_steps"]
        kern_ms += r["stats"].field_kernel_ms
        launches += r["stats"].field_launches
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = r["stats"]
    shared = int(r["n"].max(initial=0)) > 8192
    sim.close()
    events_per_s = batch.n_events * a.steps / wall
    per_launch = hsteps / max(launches, 1)
    achieved = ALG_BYTES_PER_HOLE_STEP * hsteps / (kern_ms * 1e-3) if kern_ms > 0 else None
    traffic, traffic_note = measured_traffic("spherical", per_launch)
    print(f"bench: spherical: {events_per_s:.1f} events/s, {hsteps / wall:.3e} hole updates/s; "
          f"k_sph {kern_ms / max(launches, 1):.3f} ms avg over {launches} launches",
          file=sys.stderr, flush=True)
    out = {
        "metric": METRIC_SPHERICAL, "value": events_per_s, "unit": "events/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * wall / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {batch.n_events} events, {n_holes} holes, "
                               f"{sensor.thickness_um:g} um Si at {sensor.v_bias:g} V, "
                               f"dt {sensor.dt_ns:g} ns; simplified spherical model (Eq. 7), FP64; "
                               f"one workgroup per event for all of its steps (a group of "
                               f"workgroups per event of more than 8192 holes)",
                   "events": batch.n_events, "holes": n_holes,
                   "launch": {"block": st.block_size, "workgroups": st.workgroups}},
        "hole_updates_per_s": hsteps / wall,
        "hole_steps_per_run": hsteps // a.steps,
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9 if achieved else None,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK if achieved else None,
                     "traffic": traffic, "traffic_note": traffic_note,
                     "algorithmic_bytes_per_launch": ALG_BYTES_PER_HOLE_STEP * per_launch,
                     "hole_steps_per_launch": per_launch,
                     "kernel": "k_sph_single+k_sph_shared" if shared else "k_sph_single",
                     "avg_launch_ms": kern_ms / max(launches, 1), "launches": launches},
    }
    if not a.no_cpu_baseline:
        with ct.Simulator(sensor, ct.CT_FP64, device=0) as sim:  # endpoints, untimed
            sim.seed(batch)
            sim.step(0)
            gpu_run = sim.collect(carriers=True)
        import oracle
        oracle.build(force=False)
        ch, t2, k = 0, time.perf_counter(), 0
        oracle_runs = []
        while k < batch.n_events and (time.perf_counter() - t2) < a.cpu_seconds:
            o = oracle.run(sensor, batch.event(k))
            ch += o["hole_steps"]
            oracle_runs.append(o)
            k += 1
        cwall = time.perf_counter() - t2
        out["error_vs_oracle"] = error_vs_oracle({"fp64": gpu_run}, oracle_runs)
        out["cpu_baseline"] = {"value": k / cwall, "unit": "events/s", "cores": oracle.threads(),
                               "kind": "oracle",
                               "sample": f"events 0..{k - 1} of {a.workload}, spherical model, each "
                                         f"simulated to completion alone ({ch:.3e} hole updates, "
                                         f"{cwall:.1f} s)",
                               "hole_updates_per_s": ch / cwall}
        print(f"bench: oracle {k / cwall:.2f} events/s on {oracle.threads()} threads",
              file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
