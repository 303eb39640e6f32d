"""Throughput of the batched repulsion Monte Carlo on one MI355X.

One bench step = one whole batch simulated to completion through the C ABI:
seeding of every event's initial cloud on the device, the time-step loop
(all-pairs repulsion, drift, diffusion, collection, pixel integration,
compaction) until every hole is collected, and the pixel counts copied back.

The headline line measures the 256-event 8 keV batch (the configuration whose
definition states the FP32-batched vs FP64-plain comparison of the metric):
pair-interactions/s of the FP32-batched path with the autotuned launch
(value), events/s, the FP64-plain comparison (one event at a time, FP64
field) and the 2x2 ablation, the roofline of the repulsion-step kernel (timed
with HIP events on the library's stream), and the FP64 CPU oracle timed on a
bounded sample with the GPU results' error against it.  "configs" holds the
same measurements, at fewer steps, for all five workloads (single 8 keV
photon, the 8 keV batch, the uneven mixed-energy batch, 60 keV events,
200 keV electron tracks).

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

# One ALU basis for every kernel: the VALU issues one wave64 instruction per
# SIMD every 4 clocks, i.e. one vector operation per lane per clock, 256 CUs
# x 64 lanes x 2.4 GHz.  Measured on the GPU with packed FP32 disabled (as
# this library is built): v_fma_f32, v_sub_f32, v_add_u32, v_xor_b32,
# v_mul_lo_u32, v_mul_hi_u32 and FP64 compares each issue 56-60 lanes per CU
# per clock at 2.3-2.4 GHz; DPP moves and v_rsq_f32 partly co-issue with
# them.  The published FP32 vector peak (157.3 TFLOP/s) counts two FMAs per
# lane per clock, which takes packed FP32 instructions.
VALU_ISSUE_PER_S = 256 * 64 * 2.4e9
VALU_OP_PEAK = VALU_ISSUE_PER_S
# Algorithmic vector operations per generated carrier: half a Philox4x32-10
# block (10 rounds of 2 low and 2 high 32-bit products and 4 XORs per two
# carriers: 40), 2 uniform conversions (4), two searches over the 6 pixel
# edges of a 5-pixel row (24 compares and adds), the pixel index and the
# histogram update (4)
OPS_PER_CARRIER = 72
FP32_VECTOR_PEAK = 157.3e12   # MI355X FP32 vector FLOP/s (published)
# VALU lane-instructions per ordered pair in the compiled pair loops (v_rsq_f32
# included): the Newton-pair sweep of partner tiles, four targets per lane,
# issues 253 per 16 unordered pairs (per pair 3 sub, 3 FMA, v_rsq, 2 mul,
# 3 + 3 FMA, and 3 DPP lane moves per four pairs), each serving two ordered
# pairs; a tile against itself, one target per lane, 145 per 8 (about a ninth
# of the pairs of an 8 keV event); the one-sided loop 96 per 8 ordered pairs.
NEWTON_INSTR_PER_PAIR = 253 / 32
ONE_SIDED_INSTR_PER_PAIR = 12.0
# Executed FLOP: 24 per unordered pair (FMA as 2, rsqrt as 1), 12 per ordered.
NEWTON_EXECUTED_FLOP_PER_PAIR = 12
HBM_PEAK = 8.0e12             # MI355X HBM3E bytes/s
FLOP_PER_PAIR = 20            # N-body convention for one softened pair interaction

# The five workloads: name in workloads.make_workload, what the line reports
# for it, and its bounded oracle sample: the events the CPU baseline runs
# (None: as many as fit the time budget) and the steps (None: whole runs;
# else a prefix of that many steps, compared at the prefix).
CONFIGS = {
    "cfg1": dict(workload="single_8kev", plain=1, oracle_events=[0], oracle_steps=None),
    "cfg2": dict(workload="batch_8kev", plain=32, oracle_events=None, oracle_steps=None),
    "cfg3": dict(workload="mixed_energy", plain=8, oracle_events="per_energy", oracle_steps=None),
    "cfg4": dict(workload="gamma_60kev", plain=2, oracle_events=[0], oracle_steps=None),
    "cfg5": dict(workload="track_200kev", plain=1, oracle_events=[0], oracle_steps=4),
}
HEADLINE = "cfg2"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch_8kev",
                    help="--model spherical: the workload to run")
    ap.add_argument("--model", choices=("pairs", "spherical", "generator"), default="pairs",
                    help="pairs: the brute-force field (Eq. 4); spherical: Eq. 7; generator: "
                         "the parameterised events of Sec. 4.2")
    ap.add_argument("--events", type=int, default=0, help="override the number of events")
    ap.add_argument("--configs", default="all",
                    help="pairs: the other workloads measured besides the headline "
                         "(all, none, or a comma list of cfg1..cfg5)")
    ap.add_argument("--config-steps", type=int, default=2,
                    help="timed runs per extra workload (the single event: 5x as many)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU-baseline budget of the headline workload (others: 2/3 of it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="the default launch, no autotuning")
    ap.add_argument("--launch", default="", help="targets_per_thread,block,chunk_len override")
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


def measured_traffic(model, units_per_launch, chunk_len=None, max_holes=None):
    """HBM bytes per kernel launch from the committed rocprofv3 counter
    summary (bytes per hole update; per event for the generator), or None when
    the kernel's sources have changed since the counters were taken, or (pair
    kernel) when the launch splits the events' steps into other work items
    than the profiled launches did: the partial-field traffic grows with the
    number of items.  A tile of the largest event (max_holes) meets at most
    P = T // 2 + 1 tiles (T its tiles of 256), so every source chunk of P
    tiles or more gives one item per tile, the same split."""
    path = TRAFFIC_PROFILES[model]
    try:
        text = open(path).read()
    except OSError:
        return None, "no counter summary"
    unit = "bytes_per_event" if model == "generator" else "bytes_per_hole_step"
    vals = dict(line.split(":", 1) for line in text.splitlines()
                if line.startswith((unit, "kernel_sources_sha256:", "chunk_len:")))
    if vals.get("kernel_sources_sha256", "").strip() != sources_digest(model):
        return None, "kernel changed since the counters were taken"
    per = vals.get(unit)
    if chunk_len is not None:
        per = vals.get(f"{unit}_chunk{chunk_len}")
        if per is None and int(vals.get("chunk_len", -1)) == chunk_len:
            per = vals.get(unit)
        if per is None and max_holes:
            whole = (-(-int(max_holes) // 256) // 2 + 1) * 256
            if chunk_len >= whole:
                same = sorted(int(line.split(":")[0][len(unit) + 6:])
                              for line in text.splitlines()
                              if line.startswith(f"{unit}_chunk"))
                same = [c for c in same if c >= whole]
                if same:
                    per = dict(line.split(":", 1) for line in text.splitlines()
                               if line.startswith(f"{unit}_chunk{same[0]}:"))[
                        f"{unit}_chunk{same[0]}"]
        if per is None:
            return None, f"no counters taken with source chunks of {chunk_len}"
    per = float(per)
    return per * units_per_launch, ("FETCH_SIZE and WRITE_SIZE per unit of work, scaled by a "
                                     "1 GiB copy; " + os.path.basename(path))


def counted_issue(kps):
    """The step kernel's VALU lane-instructions per ordered pair and shader
    clock from the committed counter summary of the 8 keV batch (whole
    kernel: pair loop, staging, reaction sums, update, compaction), and the
    issue fraction they give at this run's rate; None when the kernel's
    sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_run_newton_batch_8kev_valu.md")
    try:
        vals = dict(line.split(":", 1) for line in open(path).read().splitlines()
                    if line.startswith(("valu_lane_instr_per_pair:", "clock_ghz:",
                                        "kernel_sources_sha256:")))
    except OSError:
        return None
    if vals.get("kernel_sources_sha256", "").strip() != sources_digest("pairs"):
        return None
    per, clk = float(vals["valu_lane_instr_per_pair"]), float(vals["clock_ghz"]) * 1e9
    return {"lane_instr_per_pair": per, "clock_ghz": clk / 1e9,
            "frac": kps * per / VALU_ISSUE_PER_S,
            "frac_at_counted_clock": kps * per / (256 * 64 * clk),
            "source": os.path.basename(path)}


def simulate(ct, sim, batch, max_steps=0):
    """Seed, step to completion (or max_steps), copy back pixel counts and run
    statistics."""
    sim.seed(batch)
    st, done, act = sim.step(max_steps)
    if st != 0 and not (max_steps and st == -5):
        raise RuntimeError(f"batch did not finish: status {st}, {act} holes left")
    return sim.collect(carriers=False)


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


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
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.copy_calibration_mb:
        n = a.copy_calibration_mb << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {a.copy_calibration_mb} MiB done")
        del src, dst
    if a.model == "spherical":
        sensor, batch = make_workload(a.workload, **kw)
        return spherical(a, ct, torch, sensor, batch, int(batch.n_carriers.sum()))
    launch = tuple(int(v) for v in a.launch.split(",")) if a.launch else None
    tune = 0 if (a.no_tune or launch) else ct.CT_OPT_AUTOTUNE

    cfg = CONFIGS[HEADLINE]
    sensor, batch = make_workload(cfg["workload"], **kw)
    head = measure(a, ct, torch, HEADLINE, sensor, batch, a.steps, a.warmup, tune, launch,
                   headline=True)
    t = head["fp32_batched"]
    n_holes = int(batch.n_carriers.sum())
    n_carriers = n_holes * (2 if sensor.electrons else 1)
    species = "holes and electrons" if sensor.electrons else "holes"
    out = {
        "metric": METRIC, "value": t["pairs_per_s"], "unit": "pair-interactions/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": t["ms_per_run"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg['workload']}: {batch.n_events} events, "
                               f"{n_carriers} carriers ({species}), "
                               f"{sensor.thickness_um:g} um Si at {sensor.v_bias:g} V, "
                               f"dt {sensor.dt_ns:g} ns; FP32 field, FP64 state; one "
                               f"persistent step kernel per run, events stepped "
                               f"independently through a device work queue; autotuned launch",
                   "events": batch.n_events, "holes": n_holes, "carriers": n_carriers,
                   "headline": "the 256-event 8 keV batch: the configuration whose definition "
                               "states the metric's FP32-batched vs FP64-plain comparison; every "
                               "workload is reported under 'configs'",
                   "launch": t["launch"]},
        "events_per_s": t["events_per_s"],
        "pairs_per_run": t["pairs_per_run"],
        "hole_steps_per_run": t["hole_steps_per_run"],
        "roofline": head["roofline"],
    }
    for k in ("default_launch", "fp64_plain", "speedup_fp32_batched_vs_fp64_plain", "ablation",
              "cpu_baseline", "error_vs_oracle"):
        if k in head:
            out[k] = head[k]
    wanted = [] if a.configs == "none" else (
        list(CONFIGS) if a.configs == "all" else [c.strip() for c in a.configs.split(",")])
    configs = {}
    for label in wanted:
        if label == HEADLINE:
            configs[label] = {"workload": cfg["workload"], "see": "the headline fields"}
            continue
        c = CONFIGS[label]
        s2, b2 = make_workload(c["workload"])
        steps = a.config_steps * (5 if b2.n_events == 1 else 1)
        r = measure(a, ct, torch, label, s2, b2, steps, 1, tune, launch, headline=False)
        configs[label] = r
    if configs:
        out["configs"] = configs
    print(json.dumps(out), flush=True)


def timed_runs(ct, torch, sensor, batch, steps, warmup, options, launch, label):
    """FP32 runs of the whole batch: warmup untimed (the first seeding tunes
    the launch under CT_OPT_AUTOTUNE), then `steps` timed; HIP events on the
    library's stream around the step kernel of each run."""
    sim = ct.Simulator(sensor, ct.CT_FP32, device=0, options=ct.CT_OPT_TIMING | options,
                       launch=launch)
    for _ in range(warmup):
        simulate(ct, sim, batch)
    torch.cuda.synchronize()
    pairs, kern_ms, launches, hsteps = 0, 0.0, 0, 0
    t0 = time.perf_counter()
    for _ in range(steps):
        r = simulate(ct, sim, batch)
        pairs += r["pairs"]
        hsteps += r["hole_steps"]
        kern_ms += r["stats"].field_kernel_ms
        launches += r["stats"].field_launches
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = r["stats"]
    sim.close()
    res = {"pairs_per_s": pairs / wall, "events_per_s": batch.n_events * steps / wall,
           "ms_per_run": 1e3 * wall / steps, "pairs_per_run": pairs // steps,
           "hole_steps_per_run": hsteps // steps, "kernel_ms_per_run": kern_ms / steps,
           "kernel_launches_per_run": launches / steps,
           "kernel_pairs_per_s": pairs / (kern_ms * 1e-3) if kern_ms > 0 else None,
           "newton_pairs": bool(st.newton_pairs),
           "launch": {"targets_per_thread": st.targets_per_thread, "block": st.block_size,
                      "chunk_len": st.chunk_len, "workgroups": st.workgroups}}
    log(f"{label}: {res['pairs_per_s']:.3e} pairs/s, {res['events_per_s']:.1f} events/s, step "
        f"kernel {res['kernel_ms_per_run']:.2f} ms per run; launch {res['launch']}")
    return res


def roofline(t, traffic_units=None, traffic_model=None, max_holes=None):
    """The step kernel against the published FP32 peak (20 flop per ordered
    pair, the N-body convention: a pair-equivalent rate) and against the VALU
    issue rate its compiled pair loop would need (one vector instruction per
    lane per clock), with what limits it."""
    kps = t["kernel_pairs_per_s"]
    newton = t["newton_pairs"]
    per_pair = NEWTON_INSTR_PER_PAIR if newton else ONE_SIDED_INSTR_PER_PAIR
    achieved = FLOP_PER_PAIR * kps
    executed = (NEWTON_EXECUTED_FLOP_PER_PAIR if newton else FLOP_PER_PAIR) * kps
    hps = t["hole_steps_per_run"] / max(t["kernel_launches_per_run"], 1)
    traffic, note = (None, "counters taken on the 8 keV batch only")
    if traffic_model:
        traffic, note = measured_traffic(traffic_model, hps, t["launch"]["chunk_len"], max_holes)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
            "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK,
            "frac_note": "pair-equivalent: 20 flop per ordered pair (N-body convention) against "
                         "the published FP32 peak, which counts packed FP32",
            "traffic": traffic, "traffic_note": note,
            "algorithmic_bytes_per_launch": ALG_BYTES_PER_HOLE_STEP * hps,
            "hole_steps_per_launch": hps,
            "kernel": "k_run_newton<256, false>" if newton else "k_run_f32",
            "pair_evaluation": "each unordered pair once, applied to both holes" if newton
                               else "every ordered pair",
            "avg_launch_ms": t["kernel_ms_per_run"] / max(t["kernel_launches_per_run"], 1),
            "flop_per_pair": FLOP_PER_PAIR,
            "executed_tflops": executed / 1e12, "executed_frac": executed / FP32_VECTOR_PEAK,
            "issue_bound": {"basis": "VALU issue, 256 CUs x 64 lanes x 2.4 GHz = 3.93e13 "
                                     "lane-instructions/s",
                            "lane_instr_per_pair": per_pair,
                            "pairs_per_s": VALU_ISSUE_PER_S / per_pair,
                            "frac": kps * per_pair / VALU_ISSUE_PER_S,
                            "note": "DPP moves and v_rsq_f32 partly co-issue with the FMAs, so "
                                    "a pair loop can issue above this basis (a standalone "
                                    "probe of the sweep: 66-69 lane-instructions per CU per clock "
                                    "against 64)",
                            "counted": counted_issue(kps) if newton and traffic_model == "pairs" else None},
            "limiter": "on the 8 keV batch the VALU issue rate and the per-step chain of "
                       "each event (its step's items, then the tile updates and the compaction "
                       "that publish the next step) together: the kernel issues about 69 "
                       "lane-instructions per CU per clock, the ceiling a standalone probe of "
                       "the pair sweep reaches, and fewer instructions per pair shorten both "
                       "(four targets per lane: 4-5% faster; a copy with half the pair-loop "
                       "instructions of an earlier version ran 11% faster, one with none no "
                       "faster than that)"}


def plain_rate(ct, torch, sensor, events, prec, max_steps=0):
    """One event at a time (the autotuner's launch for a single event); the
    first event of each hole count once untimed (the autotuner keys its
    launches by size, so every tuning happens there), then all timed."""
    sim = ct.Simulator(sensor, prec, device=0, options=ct.CT_OPT_AUTOTUNE)
    seen = set()
    for ev in events:
        n = (int(ev.n_carriers[0]), float(ev.energy_kev[0]))  # <= 0 holes: set by the energy
        if n not in seen:
            seen.add(n)
            simulate(ct, sim, ev, max_steps)
    torch.cuda.synchronize()
    pp, t1 = 0, time.perf_counter()
    for ev in events:
        pp += simulate(ct, sim, ev, max_steps)["pairs"]
    torch.cuda.synchronize()
    w = time.perf_counter() - t1
    sim.close()
    return pp / w, len(events) / w


def oracle_picks(cfg, batch):
    ev = cfg["oracle_events"]
    if ev == "per_energy":  # the events in turn by energy level
        levels = sorted(set(batch.energy_kev.tolist()))
        lists = [np.flatnonzero(batch.energy_kev == e).tolist() for e in levels]
        return [l[i] for i in range(max(map(len, lists))) for l in lists if i < len(l)]
    return list(range(batch.n_events)) if ev is None else ev


def measure(a, ct, torch, label, sensor, batch, steps, warmup, tune, launch, headline):
    cfg = CONFIGS[label]
    log(f"{label} {cfg['workload']}: {batch.n_events} events, "
        f"{int(batch.n_carriers.sum())} holes; warmup {warmup}, steps {steps}")
    res = {"workload": cfg["workload"], "events": batch.n_events,
           "holes": int(batch.n_carriers.sum())}
    t = timed_runs(ct, torch, sensor, batch, steps, warmup, tune, launch,
                   f"{label} fp32-batched" + (", autotuned" if tune else ""))
    res["fp32_batched"] = t
    res["roofline"] = roofline(t, traffic_model="pairs" if label == "cfg2" else None,
                               max_holes=int(batch.n_carriers.max()))
    if tune:
        d = timed_runs(ct, torch, sensor, batch, max(1, steps // 2), 1, 0, None,
                       f"{label} fp32-batched, default launch")
        res["default_launch"] = {"pairs_per_s": d["pairs_per_s"], "launch": d["launch"],
                                 "kernel_ms_per_run": d["kernel_ms_per_run"]}
    if not a.no_plain:
        # FP64-plain: the same events one at a time with the FP64 field; for
        # the tracks a prefix of each event (the rate is a rate)
        picks = oracle_picks(cfg, batch)[:cfg["plain"]] if cfg["oracle_events"] == "per_energy" \
            else list(range(min(cfg["plain"], batch.n_events)))
        evs = [batch.event(e) for e in picks]
        ms = 40 if cfg["workload"] == "track_200kev" else 0
        p64, e64 = plain_rate(ct, torch, sensor, evs, ct.CT_FP64, ms)
        res["fp64_plain"] = {"value": p64, "unit": "pair-interactions/s", "events": len(evs),
                             "events_per_s": e64 if not ms else None,
                             "sample": f"events {picks}" + (f", first {ms} steps" if ms else "")}
        res["speedup_fp32_batched_vs_fp64_plain"] = t["pairs_per_s"] / p64
        log(f"{label} fp64-plain {p64:.3e} pairs/s ({len(evs)} events"
            f"{', prefix' if ms else ''}); FP32-batched / FP64-plain {t['pairs_per_s'] / p64:.1f}")
        if headline:
            # the other two corners of precision x batching, and every ordered pair
            sim = ct.Simulator(sensor, ct.CT_FP64, device=0, options=tune)
            simulate(ct, sim, batch)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            b64 = simulate(ct, sim, batch)["pairs"] / (time.perf_counter() - t1)
            sim.close()
            p32, _ = plain_rate(ct, torch, sensor, evs, ct.CT_FP32)
            res["ablation"] = {"fp32_batched": t["pairs_per_s"], "fp64_batched": b64,
                               "fp32_plain": p32, "fp64_plain": p64, "unit": "pair-interactions/s",
                               "plain_events": len(evs)}
            if t["newton_pairs"]:
                o = timed_runs(ct, torch, sensor, batch, max(1, steps // 2), 1,
                               ct.CT_OPT_ONE_SIDED, None, f"{label} fp32-batched, every ordered pair")
                res["ablation"]["fp32_batched_one_sided"] = o["pairs_per_s"]
            log(f"{label} ablation: fp64-batched {b64:.3e}, fp32-plain {p32:.3e} pairs/s")
    if not a.no_cpu_baseline:
        oracle_leg(a, ct, sensor, batch, cfg, t, res, a.cpu_seconds * (1.0 if headline else 2 / 3))
    return res


def oracle_leg(a, ct, sensor, batch, cfg, t, res, seconds):
    """The FP64 oracle on a bounded sample of the workload's events (each
    alone, whole runs or a step prefix), timed on the host cores, and the GPU
    results of the same events against it: FP32 with the batch's launch (an
    event alone equals its slice of the batched run bit for bit under the same
    launch) and FP64."""
    import oracle
    oracle.build(force=False)
    steps = cfg["oracle_steps"]
    s_or = sensor.replace(max_steps=steps) if steps else sensor
    picks = oracle_picks(cfg, batch)
    launch = (t["launch"]["targets_per_thread"], t["launch"]["block"], t["launch"]["chunk_len"])
    cpairs, t2 = 0, time.perf_counter()
    runs = []
    for e in picks:
        if runs and time.perf_counter() - t2 >= seconds:
            break
        o = oracle.run(s_or, batch.event(e))
        cpairs += o["pairs"]
        runs.append((e, o))
    cwall = time.perf_counter() - t2
    n_done = len(runs)
    what = f"first {steps} steps of" if steps else "complete runs of"
    res["cpu_baseline"] = {"value": cpairs / cwall, "unit": "pair-interactions/s",
                           "cores": oracle.threads(), "kind": "oracle",
                           "sample": f"{what} events {[e for e, _ in runs]} of "
                                     f"{cfg['workload']}, each alone ({cpairs:.3e} pairs, "
                                     f"{cwall:.1f} s)",
                           "events_per_s": n_done / cwall if not steps else None}
    gpu = {}
    for lab, prec, lau in (("fp32_batched", ct.CT_FP32, launch), ("fp64_batched", ct.CT_FP64, None)):
        outs = []
        with ct.Simulator(s_or, prec, device=0, launch=lau) as sim:
            for e, _ in runs:
                r = sim.run(batch.event(e), 0)
                outs.append(r)
        gpu[lab] = outs
    res["error_vs_oracle"] = error_vs_oracle(gpu, [o for _, o in runs], full=not steps)
    e32, e64 = res["error_vs_oracle"]["fp32_batched"], res["error_vs_oracle"]["fp64_batched"]
    log(f"oracle {cpairs / cwall:.3e} pairs/s on {oracle.threads()} threads ({n_done} events); "
        f"vs oracle: FP32 endpoints max {e32['endpoint_um_max']:.2e} / p99 "
        f"{e32['endpoint_um_p99']:.2e} um, pixel fractions {e32.get('pixel_fraction_max_abs')}; "
        f"FP64 endpoints max {e64['endpoint_um_max']:.2e} um")


def error_vs_oracle(gpu_runs, oracle_runs, full=True):
    """Per precision: the (x, y) endpoint error of every carrier of the
    oracle's events (max, 99th percentile, mean, um; positions at the prefix's
    end when the runs are a step prefix), the largest pixel charge fraction
    error and the share of carriers with the oracle's collection step."""
    res = {"events": len(oracle_runs), "compared": "whole runs" if full else "after a step prefix"}
    for label, runs in gpu_runs.items():
        d, frac, same, ncar = [], 0.0, 0, 0
        for g, o in zip(runs, oracle_runs):
            d.append(np.hypot(*(g["xyz"][:, :2] - o["xyz"][:, :2]).T))
            n = max(int(o["pix"].sum()), 1)
            frac = max(frac, float(np.abs(g["pix"][0] - o["pix"][0]).max()) / n)
            same += int((g["cstep"] == o["cstep"]).sum())
            ncar += len(o["cstep"])
        d = np.concatenate(d) if d else np.zeros(1)
        res[label] = {"endpoint_um_max": float(d.max()), "endpoint_um_p99": float(np.percentile(d, 99)),
                      "endpoint_um_mean": float(d.mean()),
                      "pixel_fraction_max_abs": frac if full else None,
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
        off = gpu_run["offsets"]
        per_event = [{"xyz": gpu_run["xyz"][off[e]:off[e + 1]], "cstep": gpu_run["cstep"][off[e]:off[e + 1]],
                      "pix": gpu_run["pix"][e:e + 1]} for e in range(k)]
        out["error_vs_oracle"] = error_vs_oracle({"fp64": per_event}, oracle_runs)
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
