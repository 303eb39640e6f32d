// HIP kernels of the brute-force charge-transport Monte Carlo for gfx950
// (Xie et al., arXiv:2506.09712, Sec. 2.1 and Appendix A, Algorithm 1).
//
// Events never interact, so an event's step t + 1 needs only its own step t.
// A ct_step call is therefore one persistent kernel (k_run) fed by a device
// work queue, with no device-wide barrier between steps:
//   k_init     queues the first step of every event still drifting: one item
//              per (target tile, source chunk) of the event;
//   k_run      a resident grid of workgroups; each claims the next ticket of
//              the queue, computes the all-pairs repulsion field of Eq. 4 of
//              its target tile over its source chunk (source tiles staged in
//              LDS, one thread per KT targets), and writes the partial field.
//              The workgroup that completes the last chunk of a target tile
//              sums the partials in chunk order and applies the update of
//              Eqs. 3, 5 and 6 (drift field, mobility, diffusion, collection,
//              pixel count); the one that completes the event's last tile
//              compacts the event (holes still drifting, in carrier order),
//              recomputes its centroid, counts the step and queues the
//              event's next step;
//   k_summary  drifting holes and steps taken, for the host.
// The split of an event into tiles and chunks depends only on its own hole
// count, and partials are always summed in chunk order, so the result of an
// event does not depend on the rest of the batch or on scheduling.
#include <mutex>

#include "ct_device.hpp"

namespace ct {

namespace {

__device__ __forceinline__ void field_or_advance(const DevParams &dp, const DevBatch &bt, int b,
                                                 int slot, double ex, double ey, double ez,
                                                 int field_only, double *field_out)
{
    if (field_only) {
        const int carrier = bt.off[b] + bt.idx[slot];
        field_out[3 * (int64_t)carrier + 0] = ex;
        field_out[3 * (int64_t)carrier + 1] = ey;
        field_out[3 * (int64_t)carrier + 2] = ez;
        return;
    }
    advance(dp, bt, b, slot, ex, ey, ez, bt.ev_step[b], (uint32_t)(bt.first_event_id + b));
}


// ------------------------------------------------------------- pair loops

// Origin of the FP32 coordinates of a work item: the FP64 position of the
// first drifting carrier of its target tile at the step start (the same for
// every item of the tile, and a function of the event alone).  Tiles are runs
// of consecutive slots, and a multi-deposit event's slots run deposit by
// deposit, so a tile's carriers lie close to its first one: FP32 coordinates
// relative to it resolve close pairs far better than coordinates relative to
// the centroid of an event spread over a long track.
__device__ __forceinline__ void tile_origin(const DevBatch &bt, int slot, double &ox, double &oy,
                                            double &oz)
{
    ox = bt.cx[slot];
    oy = bt.cy[slot];
    oz = bt.cz[slot];
}

// FP32: targets and sources relative to the target tile's origin.  Sources
// past the end of a tile are parked at 1e18 um, where the pair term
// underflows to 0.
#ifndef CT_PAIR_UNROLL
#define CT_PAIR_UNROLL 8
#endif

template <int KT>
__device__ __forceinline__ void pairs_f32(const float4 *__restrict__ tile, int cnt, float s2,
                                          const float (&tx)[KT], const float (&ty)[KT],
                                          const float (&tz)[KT], float (&ax)[KT],
                                          float (&ay)[KT], float (&az)[KT])
{
    for (int j0 = 0; j0 < cnt; j0 += CT_PAIR_UNROLL) {
#pragma unroll
        for (int u = 0; u < CT_PAIR_UNROLL; ++u) {
            const float4 s = tile[j0 + u];
#pragma unroll
            for (int m = 0; m < KT; ++m) {
                const float dx = tx[m] - s.x;
                const float dy = ty[m] - s.y;
                const float dz = tz[m] - s.z;
                float r2 = fmaf(dx, dx, s2);
                r2 = fmaf(dy, dy, r2);
                r2 = fmaf(dz, dz, r2);
                const float inv = __builtin_amdgcn_rsqf(r2);
                const float inv3 = inv * inv * inv;
                ax[m] = fmaf(dx, inv3, ax[m]);
                ay[m] = fmaf(dy, inv3, ay[m]);
                az[m] = fmaf(dz, inv3, az[m]);
            }
        }
    }
}

struct alignas(32) D4 {
    double x, y, z, w;
};


template <int KT>
__device__ __forceinline__ void pair_f64(const D4 &s, double s2, const double (&tx)[KT],
                                         const double (&ty)[KT], const double (&tz)[KT],
                                         double (&ax)[KT], double (&ay)[KT], double (&az)[KT])
{
#pragma unroll
    for (int m = 0; m < KT; ++m) {
        const double dx = tx[m] - s.x;
        const double dy = ty[m] - s.y;
        const double dz = tz[m] - s.z;
        double r2 = fma(dx, dx, s2);
        r2 = fma(dy, dy, r2);
        r2 = fma(dz, dz, r2);
        const double inv3 = inv_r3_f64(r2);
        ax[m] = fma(dx, inv3, ax[m]);
        ay[m] = fma(dy, inv3, ay[m]);
        az[m] = fma(dz, inv3, az[m]);
    }
}


// ------------------------------------------------------------------ kernels

// Resident waves per SIMD the run kernels are compiled for: the pair loop
// needs few registers, the update and compaction many; capping registers so
// that 8 waves share each SIMD (FP32, one target per thread) measured 5-7%
// faster than the unconstrained allocation (5 waves).
#ifndef CT_F32_WAVES_PER_EU
#define CT_F32_WAVES_PER_EU 8
#endif
// The Newton-pair kernel at 7: at 8 the compiler keeps only 72 scalar
// registers (16 of the SIMD's share are held back for the trap handler) and
// spills the kernel's uniform values (parameters, pointers, the item's
// split) into vector lanes, about 1100 lane reads in the item set-up, the
// update and the compaction; at 7 it has 94 scalar and 72 vector registers,
// the lane reads halve, and whole runs are 2-5% faster although each SIMD
// holds one wave fewer.
#ifndef CT_NEWTON_WAVES_PER_EU
#define CT_NEWTON_WAVES_PER_EU 7
#endif
#ifndef CT_F64_WAVES_PER_EU
#define CT_F64_WAVES_PER_EU 4
#endif

// Longest time (seconds) a workgroup waits while no event step is queued and
// no event finishes anywhere before it gives up and reports an error; the
// longest legitimate gap is one step of the largest event (well under a
// second for a million holes).
constexpr double kIdleSeconds = 10.0;

struct RunArgs {
    int chunk;             // source chunk length
    int field_only;        // 1: write the field of every drifting hole, no update
    int64_t max_steps;     // steps per event in this call
    uint64_t idle_ticks;   // kIdleSeconds in wall-clock ticks
    double *field_out;     // [N][3] by carrier (field_only)
};

// Claim the next ticket and wait until its item is published.  Thread 0
// only.  Returns 1 with the item, or 0 when the run is over: the ticket lies
// past the queue, every event is finished (then no published ticket is left
// unclaimed), or another workgroup reported an error.  Liveness: a ticket is
// only ever held by a running workgroup and publishing never waits, so while
// some event is unfinished, some workgroup holds one of its items or is about
// to publish its next step.  The wait polls only the ticket's own sequence
// word, backing off, and looks at the shared counters every 16th poll; if
// neither an event step was queued nor an event finished for idle_ticks it
// sets the error flag instead of spinning on.
__device__ int claim(const DevQueue &dq, uint32_t n_events, uint64_t idle_ticks, QItem &out)
{
    Sched *sc = dq.sc;
    const uint32_t t = add_relaxed(&sc->head.v, 1u);
    if (t >= dq.cap) return 0;
    uint32_t seen_tail = 0, seen_done = 0;
    uint64_t since = wall_clock64();
    for (uint32_t it = 0;; ++it) {
        if (ld_relaxed(&dq.seq[t]) == dq.gen) break;
        if ((it & 15u) == 15u) {
            const uint32_t dn = ld_relaxed(&sc->done.v);
            if (dn >= n_events || ld_relaxed(&sc->error.v)) return 0;
            const uint32_t tl = ld_relaxed(&sc->tail.v);
            const uint64_t now = wall_clock64();
            if (tl != seen_tail || dn != seen_done) {
                seen_tail = tl;
                seen_done = dn;
                since = now;
            } else if (now - since > idle_ticks) {
                if (atomicCAS(&sc->error.v, 0u, 1u) == 0u) {  // first to give up: record why
                    st_relaxed(&sc->stall.pad[0], t);
                    st_relaxed(&sc->stall.pad[1], ld_relaxed(&sc->head.v));
                    st_relaxed(&sc->stall.pad[2], tl);
                    st_relaxed(&sc->stall.pad[3], dn);
                }
                return 0;
            }
        }
        if (it < 64) __builtin_amdgcn_s_sleep(2);
        else if (it < 1024) __builtin_amdgcn_s_sleep(16);
        else __builtin_amdgcn_s_sleep(127);
    }
    fence_acquire();
    const uint32_t *w = reinterpret_cast<const uint32_t *>(dq.q + t);
    out.e = (int32_t)ld_relaxed(w);
    out.tile = (int32_t)ld_relaxed(w + 1);
    out.chunk = (int32_t)ld_relaxed(w + 2);
    out.n = (int32_t)ld_relaxed(w + 3);
    out.nh = (int32_t)ld_relaxed(w + 4);
    return 1;
}

// Wave priority while a workgroup computes an item of an event whose drifting
// carriers have their centroid at height z_ref above the pixel plane.  Holes
// drift towards the pixels at similar speeds, so the deeper the centroid, the
// more steps the event has left, and the sooner its items should finish when
// workgroups share a SIMD: the four levels are the quarters of the sensor
// thickness.  (With electrons the centroid counts them too, which only blurs
// the ordering.)  Issue priority changes timing only, never results.
__device__ __forceinline__ void set_item_priority(double z_ref, double H)
{
    const int level = __builtin_amdgcn_readfirstlane(
        z_ref > 0.75 * H ? 3 : (z_ref > 0.5 * H ? 2 : (z_ref > 0.25 * H ? 1 : 0)));
    if (level == 3) __builtin_amdgcn_s_setprio(3);
    else if (level == 2) __builtin_amdgcn_s_setprio(2);
    else if (level == 1) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

template <int KT, int BS, bool F32>
__device__ void run_loop(const DevParams &dp_arg, const DevBatch &bt_arg, const DevQueue &dq_arg,
                         const RunArgs &ra_arg, void *lds)
{
    const DevParams &dp = dp_arg;
    const DevBatch &bt = bt_arg;
    const DevQueue &dq = dq_arg;
    constexpr int T = KT * BS;
    constexpr int W = BS / 64;
    __shared__ QItem s_item;
    __shared__ int s_go;
    __shared__ int s_wcount[kCompactChunks * W];
    __shared__ double s_wsum[3 * W];
    __shared__ int s_items, s_tiles, s_chunks, s_nh;
    __shared__ uint32_t s_t0;
    const int tid = threadIdx.x;
    Sched *sc = dq.sc;
    const uint32_t n_events = (uint32_t)bt.n_events;
    const bool repulsion = (dp.flags & 1u) != 0;

    for (;;) {
        const DevParams &dp = reload_arg(dp_arg);  // read again in every item
        const DevBatch &bt = reload_arg(bt_arg);
        const DevQueue &dq = reload_arg(dq_arg);
        const RunArgs &ra = reload_arg(ra_arg);
        __syncthreads();  // LDS of the previous item is free
        if (tid == 0) {
            QItem it{};
            s_go = claim(dq, n_events, ra.idle_ticks, it);
            s_item = it;
        }
        __syncthreads();
        if (!s_go) break;
        const QItem it = s_item;
        const int b = it.e;
        const int n = it.n;
        const int nh = it.nh;  // the first nh slots hold holes, the rest electrons
        const int base = bt.off[b];
        const int n0 = bt.off[b + 1] - base;
        set_item_priority(bt.ref[4 * b + 2], dp.H);
        int len = n, chunks = 1;
        if (repulsion) event_chunks(n, BS, ra.chunk, len, chunks);
        const int t0 = it.tile * T;
        const int sb = it.chunk * len;
        const int se = min(n, sb + len);
        const bool wave_has_targets = t0 + (tid & ~63) < n;

        double ex[KT], ey[KT], ez[KT];
#pragma unroll
        for (int m = 0; m < KT; ++m) ex[m] = ey[m] = ez[m] = 0.0;

        if (repulsion) {
            if constexpr (F32) {
                float4 *tile = static_cast<float4 *>(lds);
                double rx, ry, rz;
                tile_origin(bt, base + t0, rx, ry, rz);
                float tx[KT], ty[KT], tz[KT];
#pragma unroll
                for (int m = 0; m < KT; ++m) {
                    const int s = t0 + m * BS + tid;
                    if (s < n) {
                        tx[m] = (float)(bt.cx[base + s] - rx);
                        ty[m] = (float)(bt.cy[base + s] - ry);
                        tz[m] = (float)(bt.cz[base + s] - rz);
                    } else {
                        tx[m] = ty[m] = tz[m] = 0.0f;
                    }
                }
                // the chunk's holes add, its electrons subtract (q_j = +1 / -1)
                for (int seg = 0; seg < 2; ++seg) {
                    const int a0 = seg == 0 ? sb : max(sb, nh);
                    const int a1 = seg == 0 ? min(se, nh) : se;
                    const double sgn = seg == 0 ? 1.0 : -1.0;
                    // the next tile's source is loaded into registers while the
                    // current tile is computed
                    double px = 0.0, py = 0.0, pz = 0.0;
                    if (a0 + tid < a1) {
                        px = bt.cx[base + a0 + tid];
                        py = bt.cy[base + a0 + tid];
                        pz = bt.cz[base + a0 + tid];
                    }
                    for (int s0 = a0; s0 < a1; s0 += BS) {
                        __syncthreads();
                        const int j = s0 + tid;
                        float4 v = make_float4(1e18f, 1e18f, 1e18f, 0.0f);
                        if (j < a1) v = make_float4((float)(px - rx), (float)(py - ry), (float)(pz - rz), 0.0f);
                        tile[tid] = v;
                        __syncthreads();
                        const int jn = j + BS;
                        if (jn < a1) {
                            px = bt.cx[base + jn];
                            py = bt.cy[base + jn];
                            pz = bt.cz[base + jn];
                        }
                        if (!wave_has_targets) continue;
                        const int cnt = (min(BS, a1 - s0) + CT_PAIR_UNROLL - 1) / CT_PAIR_UNROLL * CT_PAIR_UNROLL;
                        float ax[KT], ay[KT], az[KT];
#pragma unroll
                        for (int m = 0; m < KT; ++m) ax[m] = ay[m] = az[m] = 0.0f;
                        pairs_f32<KT>(tile, cnt, dp.s2f, tx, ty, tz, ax, ay, az);
#pragma unroll
                        for (int m = 0; m < KT; ++m) {  // fold the tile's FP32 partial into FP64
                            ex[m] += sgn * (double)ax[m];
                            ey[m] += sgn * (double)ay[m];
                            ez[m] += sgn * (double)az[m];
                        }
                    }
                }
            } else {
                D4 *tile = static_cast<D4 *>(lds);
                double tx[KT], ty[KT], tz[KT];
#pragma unroll
                for (int m = 0; m < KT; ++m) {
                    const int s = t0 + m * BS + tid;
                    if (s < n) {
                        tx[m] = bt.cx[base + s];
                        ty[m] = bt.cy[base + s];
                        tz[m] = bt.cz[base + s];
                    } else {
                        tx[m] = ty[m] = tz[m] = 0.0;
                    }
                }
                const double s2 = dp.s2;
                // the chunk's holes add, its electrons subtract (q_j = +1 / -1)
                for (int seg = 0; seg < 2; ++seg) {
                    const int a0 = seg == 0 ? sb : max(sb, nh);
                    const int a1 = seg == 0 ? min(se, nh) : se;
                    const double sgn = seg == 0 ? 1.0 : -1.0;
                    double ax[KT], ay[KT], az[KT];
#pragma unroll
                    for (int m = 0; m < KT; ++m) ax[m] = ay[m] = az[m] = 0.0;
                    for (int s0 = a0; s0 < a1; s0 += BS) {
                        __syncthreads();
                        const int j = s0 + tid;
                        if (j < a1) tile[tid] = D4{bt.cx[base + j], bt.cy[base + j], bt.cz[base + j], 0.0};
                        __syncthreads();
                        if (!wave_has_targets) continue;
                        const int cnt = min(BS, a1 - s0);
                        const int cnt4 = cnt & ~3;
                        for (int j0 = 0; j0 < cnt4; j0 += 4) {
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                pair_f64<KT>(tile[j0 + u], s2, tx, ty, tz, ax, ay, az);
                        }
                        for (int jj = cnt4; jj < cnt; ++jj) pair_f64<KT>(tile[jj], s2, tx, ty, tz, ax, ay, az);
                    }
#pragma unroll
                    for (int m = 0; m < KT; ++m) {
                        ex[m] += sgn * ax[m];
                        ey[m] += sgn * ay[m];
                        ez[m] += sgn * az[m];
                    }
                }
            }
        }

        // the rest of the item (partials, update, compaction, publication)
        // holds up every later step of its event: top priority
        __builtin_amdgcn_s_setprio(3);
        if (chunks > 1) {
            // this chunk's partial field; the tile's last chunk sums them all
            const int64_t po = dq.part_off[b] + 3 * (int64_t)it.chunk * n0;
#pragma unroll
            for (int m = 0; m < KT; ++m) {
                const int s = t0 + m * BS + tid;
                if (s < n) {
                    st_dev(&dq.part[po + s], ex[m]);
                    st_dev(&dq.part[po + n0 + s], ey[m]);
                    st_dev(&dq.part[po + 2 * n0 + s], ez[m]);
                }
            }
            wait_own_stores();
            __syncthreads();
            if (tid == 0) s_go = dec_is_last(&dq.chunks_left[dq.tile_base[b] + it.tile]);
            __syncthreads();
            if (!s_go) continue;
#pragma unroll
            for (int m = 0; m < KT; ++m) {
                const int s = t0 + m * BS + tid;
                ex[m] = ey[m] = ez[m] = 0.0;
                if (s >= n) continue;
                for (int c = 0; c < chunks; ++c) {
                    const int64_t o = dq.part_off[b] + 3 * (int64_t)c * n0 + s;
                    ex[m] += dq.part[o];
                    ey[m] += dq.part[o + n0];
                    ez[m] += dq.part[o + 2 * n0];
                }
            }
        }
#pragma unroll
        for (int m = 0; m < KT; ++m) {
            const int s = t0 + m * BS + tid;
            if (s < n)
                field_or_advance(dp, bt, b, base + s, dp.K * ex[m], dp.K * ey[m], dp.K * ez[m],
                                 ra.field_only, ra.field_out);
        }
        wait_own_stores();
        __syncthreads();
        if (tid == 0) s_go = dec_is_last(&dq.tiles_left[b * kEventLine]);
        __syncthreads();
        if (!s_go) continue;

        // every tile of the event's step is updated
        if (ra.field_only) {
            if (tid == 0) add_relaxed(&sc->done.v, 1u);
            continue;
        }
        int holes_kept = 0;
        const int kept = compact_event<BS>(bt, b, n, nh, dp.H, 1, s_wcount, s_wsum, holes_kept);
        if (tid == 0) {
            int items = 0, tiles = 0, nchunk = 1;
            uint32_t t0q = 0;
            // the event ends with its last hole (electrons may still drift)
            if (holes_kept > 0 && bt.call_steps[b] < ra.max_steps) {
                tiles = (kept + T - 1) / T;
                int l2 = kept;
                if (repulsion) event_chunks(kept, BS, ra.chunk, l2, nchunk);
                items = tiles * nchunk;
                t0q = add_relaxed(&sc->tail.v, (uint32_t)items);
                if ((uint64_t)t0q + (uint64_t)items > (uint64_t)dq.cap) {
                    st_relaxed(&sc->exhausted.v, 1u);  // parked; the host runs again
                    items = 0;
                }
            }
            if (items == 0) add_relaxed(&sc->done.v, 1u);
            s_items = items;
            s_tiles = tiles;
            s_chunks = nchunk;
            s_nh = holes_kept;
            s_t0 = t0q;
        }
        __syncthreads();
        const int items = s_items;
        if (items > 0) {
            const int tiles = s_tiles, nchunk = s_chunks;
            const uint32_t t0q = s_t0;
            const int tb = dq.tile_base[b];
            for (int j = tid; j < tiles; j += BS) st_dev(&dq.chunks_left[tb + j], nchunk);
            if (tid == 0) st_dev(&dq.tiles_left[b * kEventLine], tiles);
            for (int i = tid; i < items; i += BS) {
                int32_t *w = reinterpret_cast<int32_t *>(dq.q + t0q + i);
                st_dev(w, b);
                st_dev(w + 1, i / nchunk);
                st_dev(w + 2, i % nchunk);
                st_dev(w + 3, kept);
                st_dev(w + 4, s_nh);
            }
            wait_own_stores();
            __syncthreads();
            if (tid == 0) fence_release();
            __syncthreads();  // the write-back has completed before any sequence word is set
            for (int i = tid; i < items; i += BS) st_relaxed(&dq.seq[t0q + i], dq.gen);
        }
    }
}

// ------------------------------------------------------ Newton pairs (FP32)

// Lane l receives the value of lane l + 1 (mod 64): DPP wave rotate.
__device__ __forceinline__ float lane_up(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x134,
                                                              0xF, 0xF, true));
}

// A wave's 64 targets against one block of 64 sources, staged twice in a row
// (x y z of entries 0..127).  With REACT, lane l meets source (l + s) mod 64
// at step s, so each (target, source) pair of the block is met once, and the
// lane carries that source's reaction (minus the pair term, Eq. 4
// antisymmetry) in b, which moves one lane down after each step: after 64
// steps every lane holds the reaction on its own source.  Without REACT all
// lanes meet source s at step s (broadcast reads) and b is untouched.
// With Q (holes and electrons), pq holds the sources' charges (+1 / -1) at
// the entries of p, and qi is the target's: the target receives q_j times the
// pair term, the source minus q_i times it.
template <bool REACT, bool Q, int STEPS = 64>
__device__ __forceinline__ void sweep64(const float *__restrict__ p, const float *__restrict__ pq,
                                        float s2, float tx, float ty, float tz, float qi,
                                        float &ax, float &ay, float &az, float &bx, float &by,
                                        float &bz)
{
    for (int s0 = 0; s0 < STEPS; s0 += CT_PAIR_UNROLL) {
#pragma unroll
        for (int u = 0; u < CT_PAIR_UNROLL; ++u) {
            const float *q = p + 3 * (s0 + u);
            const float dx = tx - q[0];
            const float dy = ty - q[1];
            const float dz = tz - q[2];
            float r2 = fmaf(dx, dx, s2);
            r2 = fmaf(dy, dy, r2);
            r2 = fmaf(dz, dz, r2);
            const float inv = __builtin_amdgcn_rsqf(r2);
            const float inv3 = inv * inv * inv;
            const float ti = Q ? inv3 * pq[s0 + u] : inv3;
            ax = fmaf(dx, ti, ax);
            ay = fmaf(dy, ti, ay);
            az = fmaf(dz, ti, az);
            if constexpr (REACT) {
                const float tj = Q ? inv3 * qi : inv3;
                bx = lane_up(fmaf(-dx, tj, bx));
                by = lane_up(fmaf(-dy, tj, by));
                bz = lane_up(fmaf(-dz, tj, bz));
            }
        }
    }
}

// Two targets per lane (t0, t1: the same lane of two target blocks) against
// one block of 64 sources, laid out and rotated as in sweep64<true>: every
// source read and every rotation of the reaction registers serves two pair
// evaluations.  The charged kernel's partner sweep: the targets receive q_j
// times the pair term, the source minus q_i0 and q_i1 times theirs (four
// targets per lane, as in the holes-only kernel, spill registers there).
template <bool Q>
__device__ __forceinline__ void sweep64x2(const float *__restrict__ p, const float *__restrict__ pq,
                                          float s2, float t0x, float t0y, float t0z, float t1x,
                                          float t1y, float t1z, float qi0, float qi1, float &a0x,
                                          float &a0y, float &a0z, float &a1x, float &a1y,
                                          float &a1z, float &bx, float &by, float &bz)
{
    for (int s0 = 0; s0 < 64; s0 += CT_PAIR_UNROLL) {
#pragma unroll
        for (int u = 0; u < CT_PAIR_UNROLL; ++u) {
            const float *q = p + 3 * (s0 + u);
            const float qx = q[0], qy = q[1], qz = q[2];
            const float dx0 = t0x - qx, dy0 = t0y - qy, dz0 = t0z - qz;
            const float dx1 = t1x - qx, dy1 = t1y - qy, dz1 = t1z - qz;
            float r0 = fmaf(dx0, dx0, s2);
            float r1 = fmaf(dx1, dx1, s2);
            r0 = fmaf(dy0, dy0, r0);
            r1 = fmaf(dy1, dy1, r1);
            r0 = fmaf(dz0, dz0, r0);
            r1 = fmaf(dz1, dz1, r1);
            const float i0 = __builtin_amdgcn_rsqf(r0);
            const float i1 = __builtin_amdgcn_rsqf(r1);
            const float c0 = i0 * i0 * i0;
            const float c1 = i1 * i1 * i1;
            const float qs = Q ? pq[s0 + u] : 1.0f;
            const float g0 = Q ? c0 * qs : c0, g1 = Q ? c1 * qs : c1;  // target sides
            const float h0 = Q ? c0 * qi0 : c0, h1 = Q ? c1 * qi1 : c1;  // source side
            a0x = fmaf(dx0, g0, a0x);
            a0y = fmaf(dy0, g0, a0y);
            a0z = fmaf(dz0, g0, a0z);
            a1x = fmaf(dx1, g1, a1x);
            a1y = fmaf(dy1, g1, a1y);
            a1z = fmaf(dz1, g1, a1z);
            bx = lane_up(fmaf(-dx1, h1, fmaf(-dx0, h0, bx)));
            by = lane_up(fmaf(-dy1, h1, fmaf(-dy0, h0, by)));
            bz = lane_up(fmaf(-dz1, h1, fmaf(-dz0, h0, bz)));
        }
    }
}

// Four targets per lane (lane l of each of the tile's four target blocks)
// against one block of 64 sources, laid out and rotated as in sweep64<true>:
// every source read and every rotation of the reaction registers serves four
// pair evaluations, 63 VALU instructions per four pairs (holes only).  With
// Q the charges enter as in sweep64.  Only the first NT target blocks hold
// holes (a ragged tile); the others are skipped.
template <bool Q, int NT>
__device__ __forceinline__ void sweep64x4(const float *__restrict__ p, const float *__restrict__ pq,
                                          float s2, const float (&t)[4][3], const float (&qt)[4],
                                          float (&acc)[4][3], float &bx, float &by, float &bz)
{
    // 4 steps (16 evaluations) per iteration: at 8 the loop spills a register
    for (int s0 = 0; s0 < 64; s0 += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float *q = p + 3 * (s0 + u);
            const float qx = q[0], qy = q[1], qz = q[2];
            const float qs = Q ? pq[s0 + u] : 1.0f;
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                const float dx = t[k][0] - qx, dy = t[k][1] - qy, dz = t[k][2] - qz;
                float r2 = fmaf(dx, dx, s2);
                r2 = fmaf(dy, dy, r2);
                r2 = fmaf(dz, dz, r2);
                const float i1 = __builtin_amdgcn_rsqf(r2);
                const float c = i1 * i1 * i1;
                const float g = Q ? c * qs : c;     // target side
                const float h = Q ? c * qt[k] : c;  // source side
                acc[k][0] = fmaf(dx, g, acc[k][0]);
                acc[k][1] = fmaf(dy, g, acc[k][1]);
                acc[k][2] = fmaf(dz, g, acc[k][2]);
                bx = fmaf(-dx, h, bx);
                by = fmaf(-dy, h, by);
                bz = fmaf(-dz, h, bz);
            }
            bx = lane_up(bx);
            by = lane_up(by);
            bz = lane_up(bz);
        }
    }
}

// A wave's 64 targets against the other 63 holes of their own block: lane l
// meets hole l + s (mod 64) at the offsets s = 1..32, read from p = the
// block's doubled entries + lane + 1, so that each pair of the block is met
// once (offset 32 pairs l with l + 32 twice; only lanes below 32 count it).
// After the 32 rotations lane l holds the reaction on hole (l + 33) mod 64.
template <bool Q>
__device__ __forceinline__ void sweep_self(const float *__restrict__ p, const float *__restrict__ pq,
                                           float s2, float tx, float ty, float tz, float qi, int lane,
                                           float &ax, float &ay, float &az, float &bx, float &by,
                                           float &bz)
{
#pragma unroll
    for (int u = 0; u < 32; ++u) {
        const float *q = p + 3 * u;
        const float dx = tx - q[0];
        const float dy = ty - q[1];
        const float dz = tz - q[2];
        float r2 = fmaf(dx, dx, s2);
        r2 = fmaf(dy, dy, r2);
        r2 = fmaf(dz, dz, r2);
        const float inv = __builtin_amdgcn_rsqf(r2);
        float inv3 = inv * inv * inv;
        if (u == 31 && lane >= 32) inv3 = 0.0f;
        const float ti = Q ? inv3 * pq[u] : inv3;
        const float tj = Q ? inv3 * qi : inv3;
        ax = fmaf(dx, ti, ax);
        ay = fmaf(dy, ti, ay);
        az = fmaf(dz, ti, az);
        bx = lane_up(fmaf(-dx, tj, bx));
        by = lane_up(fmaf(-dy, tj, by));
        bz = lane_up(fmaf(-dz, tj, bz));
    }
}

// Most tiles one item contributes to: its own and one partner per offset.
constexpr int kMaxTouch = kSymMaxC + 1;

// The persistent loop with the Newton-pair split of the field (FP32, one
// target per thread, tiles of kSymTile; the split is described with
// sym_split; with Q the events hold holes and electrons, whose charges are
// staged beside the sources).  An item stages each partner tile in LDS as
// four doubled blocks of 64.  Against itself the tile is swept one target
// per lane, 128 steps per wave; against a partner tile waves w and w ^ 1
// each sweep two of the four source blocks with two targets per lane
// (blocks w and w ^ 1).  The reactions on a source are summed over the
// waves that met it, in wave order (FP64), into the partner's partial slot;
// the target side folds each partner tile's FP32 sums into FP64 and goes to
// the item's own slot (slots hold FP32).  Each item then counts down the
// tiles it contributed to; the workgroup that completes a tile sums its
// slots in slot order and updates it, and the one that completes the
// event's last tile compacts the event and queues its next step, as in
// run_loop.
template <int BS, bool Q>
__device__ void run_loop_newton(const DevParams &dp_arg, const DevBatch &bt_arg,
                                const DevQueue &dq_arg, const RunArgs &ra_arg, float *src,
                                float *react, float *sq)
{
    const DevBatch &bt = bt_arg;
    const DevQueue &dq = dq_arg;
    const RunArgs &ra = ra_arg;
    static_assert(BS == kSymTile, "one target per thread over tiles of kSymTile");
    constexpr int W = BS / 64;
    __shared__ QItem s_item;
    __shared__ int s_go;
    __shared__ int s_wcount[kCompactChunks * W];
    __shared__ double s_wsum[3 * W];
    __shared__ int s_items, s_kept, s_nh;
    __shared__ uint32_t s_t0;
    __shared__ int s_fin[kMaxTouch];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    Sched *sc = dq.sc;
    const uint32_t n_events = (uint32_t)bt.n_events;
    const int ctiles = ra.chunk / BS;

    for (;;) {
        // the arguments are read again in every item (about 480 fewer lane
        // reads of spilled scalars in the kernel; whole runs 0.6-1.4% faster)
        const DevParams &dp = reload_arg(dp_arg);
        const DevBatch &bt = reload_arg(bt_arg);
        const DevQueue &dq = reload_arg(dq_arg);
        const RunArgs &ra = reload_arg(ra_arg);
        __syncthreads();  // LDS of the previous item is free
        if (tid == 0) {
            QItem it{};
            s_go = claim(dq, n_events, ra.idle_ticks, it);
            s_item = it;
        }
        __syncthreads();
        if (!s_go) break;
        const QItem it = s_item;
        const int b = it.e, n = it.n, a = it.tile, r = it.chunk;
        const int nh = Q ? it.nh : n;  // the first nh slots hold holes, the rest electrons
        const int base = bt.off[b];
        const int n0 = bt.off[b + 1] - base;
        set_item_priority(bt.ref[4 * b + 2], dp.H);
        const SymSplit sp = sym_split(n, ctiles);
        const int64_t po = dq.part_off[b];
        // partial fields of Newton items are kept in FP32 (the slot array
        // read as floats, same indices): each is one FP32 rounding of an
        // FP64 sum of FP32 partials, and the tile adds its slots in FP64
        float *const pf = reinterpret_cast<float *>(dq.part);
        double rx, ry, rz;
        tile_origin(bt, base + a * BS, rx, ry, rz);
        // targets past the end are parked far away, where every pair term
        // with them underflows to 0 (they also act as sources here)
        const int si = a * BS + tid;
        float tx = 1e18f, ty = 1e18f, tz = 1e18f;
        const float qi = si < nh ? 1.0f : (si < n ? -1.0f : 0.0f);
        if (si < n) {
            tx = (float)(bt.cx[base + si] - rx);
            ty = (float)(bt.cy[base + si] - ry);
            tz = (float)(bt.cz[base + si] - rz);
        }
        const bool wave_has_targets = a * BS + w * 64 < n;
        // Partner tiles are swept four targets per lane: every wave holds
        // lane `lane` of the four target blocks, and wave w sweeps source
        // block w of the partner tile.  (The charged kernel sweeps two per
        // lane: waves w and w ^ 1 hold blocks w and w ^ 1 and split the
        // source blocks, w even taking 0 and 1; its second target is lane
        // `lane` of block w ^ 1.)
        const int si1 = a * BS + (w ^ 1) * 64 + lane;
        float ux = 1e18f, uy = 1e18f, uz = 1e18f;
        const float qi1 = si1 < nh ? 1.0f : (si1 < n ? -1.0f : 0.0f);
        if (Q && si1 < n) {
            ux = (float)(bt.cx[base + si1] - rx);
            uy = (float)(bt.cy[base + si1] - ry);
            uz = (float)(bt.cz[base + si1] - rz);
        }
        const bool pair_has_targets = a * BS + (w & ~1) * 64 < n;
        float t4[4][3], q4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int sk = a * BS + k * 64 + lane;
            q4[k] = sk < nh ? 1.0f : (sk < n ? -1.0f : 0.0f);
            t4[k][0] = t4[k][1] = t4[k][2] = 1e18f;
            if (!Q && sk < n) {
                t4[k][0] = (float)(bt.cx[base + sk] - rx);
                t4[k][1] = (float)(bt.cy[base + sk] - ry);
                t4[k][2] = (float)(bt.cz[base + sk] - rz);
            }
        }
        const int o0 = r * sp.C;
        const int o1 = min(o0 + sp.C, sp.newton ? sym_partners(sp.T, a) : sp.T);
        double ex = 0.0, ey = 0.0, ez = 0.0;
        // the next partner tile's source is loaded into registers while the
        // current one is computed
        double px = 0.0, py = 0.0, pz = 0.0;
        {
            const int sj = (sp.newton ? (a + o0) % sp.T : o0) * BS + tid;
            if (o0 < o1 && sj < n) {
                px = bt.cx[base + sj];
                py = bt.cy[base + sj];
                pz = bt.cz[base + sj];
            }
        }
        for (int o = o0; o < o1; ++o) {
            const int pt = sp.newton ? (a + o) % sp.T : o;  // partner tile
            const bool reacts = sp.newton && o > 0;
            const int sj = pt * BS + tid;
            float fx = 1e18f, fy = 1e18f, fz = 1e18f;
            if (sj < n) {
                fx = (float)(px - rx);
                fy = (float)(py - ry);
                fz = (float)(pz - rz);
            }
            __syncthreads();  // the previous partner's sources and reactions are consumed
            float *d = src + 3 * (w * 128 + lane);
            d[0] = fx;
            d[1] = fy;
            d[2] = fz;
            d[192] = fx;
            d[193] = fy;
            d[194] = fz;
            if constexpr (Q) {
                const float qs = sj < nh ? 1.0f : (sj < n ? -1.0f : 0.0f);
                sq[w * 128 + lane] = qs;
                sq[w * 128 + 64 + lane] = qs;
            }
            __syncthreads();
            if (o + 1 < o1) {
                const int sn = (sp.newton ? (a + o + 1) % sp.T : o + 1) * BS + tid;
                if (sn < n) {
                    px = bt.cx[base + sn];
                    py = bt.cy[base + sn];
                    pz = bt.cz[base + sn];
                }
            }
            const int nblk = min(W, (n - pt * BS + 63) / 64);  // blocks holding holes
            float ax = 0.0f, ay = 0.0f, az = 0.0f;
            if (sp.newton && o == 0) {
                // the tile with itself, 128 steps per wave: block w with
                // itself (offsets 1 to 32), block pair (w, w + 1), and half
                // of (w, w + 2): waves 0 and 1 take its offsets 0 to 31 from
                // block w's side, waves 2 and 3 the rest from the other
                // side (offsets 1 to 32 of (w, w - 2)); the reactions land on
                // this tile's own holes
                static_assert(W == 4, "four blocks per tile");
                {
                    float bx = 0.0f, by = 0.0f, bz = 0.0f;
                    if (wave_has_targets)
                        sweep_self<Q>(src + 3 * (w * 128 + lane + 1), sq + w * 128 + lane + 1, dp.s2f,
                                      tx, ty, tz, qi, lane, ax, ay, az, bx, by, bz);
                    float *q = react + 3 * (w * BS + w * 64 + ((lane + 33) & 63));
                    q[0] = bx;
                    q[1] = by;
                    q[2] = bz;
                }
                {
                    const int v = (w + 1) & (W - 1);
                    float bx = 0.0f, by = 0.0f, bz = 0.0f;
                    if (wave_has_targets && v < nblk)
                        sweep64<true, Q>(src + 3 * (v * 128 + lane), sq + v * 128 + lane, dp.s2f, tx,
                                         ty, tz, qi, ax, ay, az, bx, by, bz);
                    float *q = react + 3 * (w * BS + v * 64 + lane);
                    q[0] = bx;
                    q[1] = by;
                    q[2] = bz;
                }
                {
                    const int v = (w + 2) & (W - 1);
                    const int off = w < 2 ? 0 : 1;  // first offset of this wave's half
                    float bx = 0.0f, by = 0.0f, bz = 0.0f;
                    if (wave_has_targets && v < nblk)
                        sweep64<true, Q, 32>(src + 3 * (v * 128 + lane + off), sq + v * 128 + lane + off,
                                             dp.s2f, tx, ty, tz, qi, ax, ay, az, bx, by, bz);
                    // after 32 rotations lane l holds source l + off + 32
                    float *q = react + 3 * (w * BS + v * 64 + ((lane + off + 32) & 63));
                    q[0] = bx;
                    q[1] = by;
                    q[2] = bz;
                }
                {
                    float *q = react + 3 * (w * BS + ((w + 3) & (W - 1)) * 64 + lane);
                    q[0] = 0.0f;
                    q[1] = 0.0f;
                    q[2] = 0.0f;
                }
                __syncthreads();
                if (si < n) {
#pragma unroll
                    for (int w2 = 0; w2 < W; ++w2) {
                        const float *q = react + 3 * (w2 * BS + tid);
                        ex += (double)q[0];
                        ey += (double)q[1];
                        ez += (double)q[2];
                    }
                }
            } else if (!Q && reacts) {
                // source block w against all four target blocks; this lane
                // ends with the reaction on source w * 64 + lane, which is
                // this thread's sj, and the target sums go to their threads
                // through the reaction rows
                static_assert(W == 4, "four blocks per tile");
                float acc[4][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f},
                                   {0.0f, 0.0f, 0.0f}};
                float bx = 0.0f, by = 0.0f, bz = 0.0f;
                if (w < nblk) {
                    const float *ps = src + 3 * (w * 128 + lane);
                    const float *pq = sq + w * 128 + lane;
                    const int ntb = min(W, (n - a * BS + 63) / 64);  // target blocks with holes
                    if (ntb == 4)
                        sweep64x4<Q, 4>(ps, pq, dp.s2f, t4, q4, acc, bx, by, bz);
                    else if (ntb == 3)
                        sweep64x4<Q, 3>(ps, pq, dp.s2f, t4, q4, acc, bx, by, bz);
                    else if (ntb == 2)
                        sweep64x4<Q, 2>(ps, pq, dp.s2f, t4, q4, acc, bx, by, bz);
                    else
                        sweep64x4<Q, 1>(ps, pq, dp.s2f, t4, q4, acc, bx, by, bz);
                }
                if (sj < n) {
                    const int64_t o2 = po + 3 * (int64_t)(sp.R + o - 1) * n0 + sj;
                    st_dev(&pf[o2], bx);
                    st_dev(&pf[o2 + n0], by);
                    st_dev(&pf[o2 + 2 * n0], bz);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    float *q = react + 3 * (w * BS + k * 64 + lane);
                    q[0] = acc[k][0];
                    q[1] = acc[k][1];
                    q[2] = acc[k][2];
                }
                __syncthreads();
#pragma unroll
                for (int w2 = 0; w2 < W; ++w2) {
                    const float *q = react + 3 * (w2 * BS + tid);
                    ex += (double)q[0];
                    ey += (double)q[1];
                    ez += (double)q[2];
                }
            } else if (reacts) {
                // blocks v = 2 (w & 1) and v + 1 against targets w and w ^ 1;
                // the sums of target w ^ 1 go to wave w ^ 1 through the two
                // blocks of this wave's reaction rows it does not use
                static_assert(W == 4, "four blocks per tile");
                float cx = 0.0f, cy = 0.0f, cz = 0.0f;
                for (int k = 0; k < 2; ++k) {
                    const int v = 2 * (w & 1) + k;
                    float bx = 0.0f, by = 0.0f, bz = 0.0f;
                    if (pair_has_targets && v < nblk)
                        sweep64x2<Q>(src + 3 * (v * 128 + lane), sq + v * 128 + lane, dp.s2f, tx, ty,
                                     tz, ux, uy, uz, qi, qi1, ax, ay, az, cx, cy, cz, bx, by, bz);
                    float *q = react + 3 * (w * BS + v * 64 + lane);
                    q[0] = bx;
                    q[1] = by;
                    q[2] = bz;
                }
                {
                    float *q = react + 3 * (w * BS + (2 - 2 * (w & 1)) * 64 + lane);
                    q[0] = cx;
                    q[1] = cy;
                    q[2] = cz;
                }
                __syncthreads();
                if (sj < n) {
                    // source block v = tid / 64 was swept by waves v / 2 and
                    // v / 2 + 2
                    const int wa = (tid >> 6) >> 1;
                    const float *q0 = react + 3 * (wa * BS + tid);
                    const float *q1 = react + 3 * ((wa + 2) * BS + tid);
                    const double qx = (double)q0[0] + (double)q1[0];
                    const double qy = (double)q0[1] + (double)q1[1];
                    const double qz = (double)q0[2] + (double)q1[2];
                    const int64_t o2 = po + 3 * (int64_t)(sp.R + o - 1) * n0 + sj;
                    st_dev(&pf[o2], (float)qx);
                    st_dev(&pf[o2 + n0], (float)qy);
                    st_dev(&pf[o2 + 2 * n0], (float)qz);
                }
                {
                    // target block w over the other two source blocks, from
                    // wave w ^ 1
                    const int wp = w ^ 1;
                    const float *q = react + 3 * (wp * BS + (2 - 2 * (wp & 1)) * 64 + lane);
                    ex += (double)q[0];
                    ey += (double)q[1];
                    ez += (double)q[2];
                }
            } else if (wave_has_targets) {
                float bx = 0.0f, by = 0.0f, bz = 0.0f;
                for (int v = 0; v < nblk; ++v)
                    sweep64<false, Q>(src + 3 * v * 128, sq + v * 128, dp.s2f, tx, ty, tz, qi, ax, ay,
                                      az, bx, by, bz);
            }
            ex += (double)ax;
            ey += (double)ay;
            ez += (double)az;
        }

        // the rest of the item holds up every later step of its event
        __builtin_amdgcn_s_setprio(3);
        const bool split = sym_partials(sp);
        const int oa = max(o0, 1);
        const int ntouch = split ? 1 + (sp.newton ? max(0, o1 - oa) : 0) : 1;
        if (split) {
            if (si < n) {
                const int64_t o2 = po + 3 * (int64_t)r * n0 + si;
                st_dev(&pf[o2], (float)ex);
                st_dev(&pf[o2 + n0], (float)ey);
                st_dev(&pf[o2 + 2 * n0], (float)ez);
            }
            wait_own_stores();
            __syncthreads();
            if (tid < ntouch) {
                const int u = tid == 0 ? a : (a + oa + tid - 1) % sp.T;
                s_fin[tid] = dec_is_last(&dq.chunks_left[dq.tile_base[b] + u]) ? u : -1;
            }
        } else if (tid == 0) {
            s_fin[0] = a;
        }
        __syncthreads();
        // The tiles this item completed (often several: its own and partners
        // whose last reaction it delivered) are updated in one pass, without a
        // barrier between them, and counted off the event with one atomic, so
        // that the end of an event's step waits for one store round trip and
        // one release instead of one of each per tile.  (Loading a hole's
        // state or several partial slots ahead of the sums was slower: the
        // extra registers spill at this occupancy.)
        int done_tiles = 0;
        for (int k = 0; k < ntouch; ++k) {
            const int u = s_fin[k];
            if (u < 0) continue;
            ++done_tiles;
            const int s = u * BS + tid;
            if (s < n) {
                double fx = ex, fy = ey, fz = ez;
                if (split) {
                    // own slots in item order, then reactions by offset
                    const int nslot = sym_expected(sp, u);
                    fx = fy = fz = 0.0;
                    for (int k2 = 0; k2 < nslot; ++k2) {
                        const int64_t o2 = po + 3 * (int64_t)k2 * n0 + s;
                        fx += (double)pf[o2];
                        fy += (double)pf[o2 + n0];
                        fz += (double)pf[o2 + 2 * n0];
                    }
                }
                field_or_advance(dp, bt, b, base + s, dp.K * fx, dp.K * fy, dp.K * fz,
                                 ra.field_only, ra.field_out);
            }
        }
        if (done_tiles > 0) {
            wait_own_stores();
            __syncthreads();
            if (tid == 0) s_go = dec_is_last(&dq.tiles_left[b * kEventLine], done_tiles);
            __syncthreads();
        }
        if (done_tiles > 0 && s_go) {
            // every tile of the event's step is updated
            if (ra.field_only) {
                if (tid == 0) add_relaxed(&sc->done.v, 1u);
                continue;
            }
            int holes_kept = 0;
            const int kept = compact_event<BS>(bt, b, n, nh, dp.H, 1, s_wcount, s_wsum, holes_kept);
            if (tid == 0) {
                int items = 0;
                uint32_t t0q = 0;
                if (holes_kept > 0 && bt.call_steps[b] < ra.max_steps) {
                    const SymSplit s2 = sym_split(kept, ctiles);
                    items = s2.T * s2.R;
                    t0q = add_relaxed(&sc->tail.v, (uint32_t)items);
                    if ((uint64_t)t0q + (uint64_t)items > (uint64_t)dq.cap) {
                        st_relaxed(&sc->exhausted.v, 1u);  // parked; the host runs again
                        items = 0;
                    }
                }
                if (items == 0) add_relaxed(&sc->done.v, 1u);
                s_items = items;
                s_kept = kept;
                s_nh = holes_kept;
                s_t0 = t0q;
            }
            __syncthreads();
            const int items = s_items;
            if (items > 0) {
                const SymSplit s2 = sym_split(s_kept, ctiles);
                const uint32_t t0q = s_t0;
                const int tb = dq.tile_base[b];
                for (int j = tid; j < s2.T; j += BS) st_dev(&dq.chunks_left[tb + j], sym_expected(s2, j));
                if (tid == 0) st_dev(&dq.tiles_left[b * kEventLine], s2.T);
                for (int i = tid; i < items; i += BS) {
                    int32_t *q = reinterpret_cast<int32_t *>(dq.q + t0q + i);
                    st_dev(q, b);
                    st_dev(q + 1, i / s2.R);
                    st_dev(q + 2, i % s2.R);
                    st_dev(q + 3, s_kept);
                    st_dev(q + 4, s_nh);
                }
                wait_own_stores();
                __syncthreads();
                if (tid == 0) fence_release();
                __syncthreads();  // the write-back has completed before any sequence word is set
                for (int i = tid; i < items; i += BS) st_relaxed(&dq.seq[t0q + i], dq.gen);
            }
        }
    }
}

// (With charges the LDS of 8 workgroups would not fit a CU either.)
template <int BS, bool Q>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(CT_NEWTON_WAVES_PER_EU)))
void k_run_newton(DevParams dp, DevBatch bt, DevQueue dq, RunArgs ra)
{
    __shared__ float src[3 * 2 * BS];             // four blocks of 64 sources, each twice
    __shared__ float react[3 * BS * (BS / 64)];   // reactions per wave and source
    __shared__ float sq[Q ? 2 * BS : 1];          // the sources' charges (holes and electrons)
    run_loop_newton<BS, Q>(dp, bt, dq, ra, src, react, sq);
}

template <int KT, int BS>
__global__ __launch_bounds__(BS)
__attribute__((amdgpu_waves_per_eu(KT == 1 ? CT_F32_WAVES_PER_EU : (KT == 2 ? 5 : 4))))
void k_run_f32(DevParams dp, DevBatch bt, DevQueue dq, RunArgs ra)
{
    __shared__ float4 lds[BS];
    run_loop<KT, BS, true>(dp, bt, dq, ra, lds);
}

template <int KT, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(CT_F64_WAVES_PER_EU)))
void k_run_f64(DevParams dp, DevBatch bt, DevQueue dq, RunArgs ra)
{
    __shared__ D4 lds[BS];
    run_loop<KT, BS, false>(dp, bt, dq, ra, lds);
}

// First step of every event still drifting (and, for a field evaluation,
// with no step cap): its items, tickets in event order, and its completion
// counters; resets the run's control block.  One workgroup of 1024; events
// in blocks of 1024, each wave emitting the items of every 16th event.
__global__ __launch_bounds__(1024) void k_init(DevBatch bt, DevQueue dq, int T, int bs, int chunk,
                                               int64_t max_steps, int field_only, int repulsion,
                                               int newton)
{
    __shared__ int wtot[16];
    __shared__ uint32_t s_base[1024];
    __shared__ int s_nitems[1024], s_nchunk[1024];
    __shared__ uint32_t carry, n_done;
    __shared__ int overflow;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int B = bt.n_events;
    if (tid == 0) {
        carry = 0;
        n_done = 0;
        overflow = 0;
    }
    __syncthreads();
    for (int e0 = 0; e0 < B; e0 += 1024) {
        const int e = e0 + tid;
        int items = 0, nchunk = 1;
        if (e < B) {
            const int n = bt.n_act[e];
            if (bt.n_hole[e] > 0 && (field_only || bt.call_steps[e] < max_steps)) {
                if (newton) {
                    const SymSplit sp = sym_split(n, chunk / kSymTile);
                    nchunk = sp.R;
                    items = sp.T * sp.R;
                    dq.tiles_left[e * kEventLine] = sp.T;
                    for (int j = 0; j < sp.T; ++j) dq.chunks_left[dq.tile_base[e] + j] = sym_expected(sp, j);
                } else {
                    const int tiles = (n + T - 1) / T;
                    int len = n;
                    if (repulsion) event_chunks(n, bs, chunk, len, nchunk);
                    items = tiles * nchunk;
                    dq.tiles_left[e * kEventLine] = tiles;
                    for (int j = 0; j < tiles; ++j) dq.chunks_left[dq.tile_base[e] + j] = nchunk;
                }
            } else {
                atomicAdd(&n_done, 1u);
            }
        }
        int v = items;  // inclusive scan within the wave
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(v, o);
            if (lane >= o) v += t;
        }
        if (lane == 63) wtot[wave] = v;
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            before += q < wave ? wtot[q] : 0;
            total += wtot[q];
        }
        s_base[tid] = carry + (uint32_t)(before + v - items);
        s_nitems[tid] = items;
        s_nchunk[tid] = nchunk;
        __syncthreads();
        for (int k = wave; k < 1024 && e0 + k < B; k += 16) {
            const int ni = s_nitems[k], nc = s_nchunk[k];
            const uint32_t b0 = s_base[k];
            if ((uint64_t)b0 + (uint64_t)ni > (uint64_t)dq.cap) {
                if (lane == 0) overflow = 1;
                continue;
            }
            for (int i = lane; i < ni; i += 64) {
                dq.q[b0 + i] = QItem{e0 + k, i / nc, i % nc, bt.n_act[e0 + k], bt.n_hole[e0 + k], {0, 0, 0}};
                dq.seq[b0 + i] = dq.gen;
            }
        }
        __syncthreads();
        if (tid == 0) carry += (uint32_t)total;
        __syncthreads();
    }
    if (tid == 0) {
        Sched *sc = dq.sc;
        sc->head.v = 0;
        sc->tail.v = carry;
        sc->done.v = overflow ? (uint32_t)B : n_done;
        sc->error.v = overflow ? 2u : 0u;
        sc->stall.pad[0] = sc->stall.pad[1] = sc->stall.pad[2] = sc->stall.pad[3] = 0;
        sc->exhausted.v = 0;
    }
}


// Drifting holes and the most steps any event took in this call.
__global__ __launch_bounds__(1024) void k_summary(DevBatch bt, Sched *sc)
{
    __shared__ int64_t ssum[16], smax[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int64_t sum = 0, mx = 0;
    for (int e = tid; e < bt.n_events; e += 1024) {
        sum += bt.n_hole[e];
        mx = max(mx, bt.call_steps[e]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        sum += __shfl_down(sum, o);
        mx = max(mx, (int64_t)__shfl_down(mx, o));
    }
    if (lane == 0) {
        ssum[wave] = sum;
        smax[wave] = mx;
    }
    __syncthreads();
    if (tid == 0) {
        int64_t S = 0, M = 0;
        for (int q = 0; q < 16; ++q) {
            S += ssum[q];
            M = max(M, smax[q]);
        }
        sc->active = S;
        sc->max_steps = M;
    }
}

// Compaction of every event at seeding (holes already at z <= 0 are out),
// which also sets the FP32 reference points.  One workgroup per event.
__global__ __launch_bounds__(256) void k_compact(DevParams dp, DevBatch bt)
{
    __shared__ int wcount[kCompactChunks * 4];
    __shared__ double wsum[12];
    int holes = 0;
    compact_event<256>(bt, blockIdx.x, bt.n_act[blockIdx.x], bt.nh0[blockIdx.x], dp.H, 0, wcount,
                       wsum, holes);
}

// Initial clouds (Algorithm 1, initialisation; Eq. 2 width).  One thread per
// slot; the event is found by binary search over the slot offsets.  Slots
// hold an event's holes, then its electrons; within each species the slots
// of a multi-deposit event run deposit-major (deposit_major).  Outputs are
// indexed by carrier.
__global__ __launch_bounds__(256) void k_seed(DevParams dp, DevBatch bt)
{
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= bt.n_total) return;
    int lo = 0, hi = bt.n_events;  // off[lo] <= g < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bt.off[mid] <= g) lo = mid;
        else hi = mid;
    }
    const int b = lo;
    const int s = g - bt.off[b];
    const int nh = bt.nh0[b], n = bt.off[b + 1] - bt.off[b];
    const int d0 = bt.dep_off[b], nd = bt.dep_off[b + 1] - d0;
    const int k = s < nh ? deposit_major(s, nh, nd) : nh + deposit_major(s - nh, n - nh, nd);
    const int carrier = bt.off[b] + k;
    const bool electron = k >= nh;
    double x, y, z;
    if (nd > 0) {
        // electron k of a cloud event starts where hole k starts: same draw
        const int kh = electron ? k - bt.nh0[b] : k;
        const double *d = bt.deposits + 3 * (int64_t)(d0 + kh % nd);
        double n3[3];
        normals3(dp, Ctr{(uint32_t)bt.rngid[bt.off[b] + kh], 0u, (uint32_t)(bt.first_event_id + b),
                         kDomainCloud},
                 n3);
        const double sg = bt.sigma[b];
        x = d[0] + sg * n3[0];
        y = d[1] + sg * n3[1];
        z = d[2] + sg * n3[2];
    } else {
        const double *p = bt.xyz_in + 3 * (int64_t)(bt.x_off[b] + k);
        x = p[0];
        y = p[1];
        z = p[2];
    }
    const bool done = boundary(dp, electron, z);
    bt.nidx[g] = k;
    bt.nx[g] = x;
    bt.ny[g] = y;
    bt.nz[g] = z;
    bt.out_cstep[carrier] = -1;
    if (done) collect(dp, bt, b, carrier, electron, x, y, z, bt.start[b]);
}

// Current positions of drifting carriers into the carrier-ordered output.
__global__ __launch_bounds__(256) void k_scatter_alive(DevBatch bt)
{
    const int b = blockIdx.y;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= bt.n_act[b]) return;
    const int slot = bt.off[b] + s;
    const int64_t carrier = bt.off[b] + bt.idx[slot];
    bt.out_xyz[3 * carrier + 0] = bt.cx[slot];
    bt.out_xyz[3 * carrier + 1] = bt.cy[slot];
    bt.out_xyz[3 * carrier + 2] = bt.cz[slot];
}

__global__ __launch_bounds__(256) void k_philox(DevParams dp, const uint32_t *ctr, int64_t n,
                                                uint32_t *words, double *normals)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const Ctr c{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
    if (words) {
        const Ctr w = philox10(c, dp.key0, dp.key1);
        words[4 * i + 0] = w.c0;
        words[4 * i + 1] = w.c1;
        words[4 * i + 2] = w.c2;
        words[4 * i + 3] = w.c3;
    }
    if (normals) {
        double g[3];
        normals3(dp, c, g);
        normals[3 * i + 0] = g[0];
        normals[3 * i + 1] = g[1];
        normals[3 * i + 2] = g[2];
    }
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

template <int KT, int BS>
hipError_t launch_run_t(const DevParams &dp, const DevBatch &bt, const DevQueue &dq,
                        const RunArgs &ra, int fp32, int grid, hipStream_t s)
{
    if (fp32)
        hipLaunchKernelGGL((k_run_f32<KT, BS>), dim3(grid), dim3(BS), 0, s, dp, bt, dq, ra);
    else
        hipLaunchKernelGGL((k_run_f64<KT, BS>), dim3(grid), dim3(BS), 0, s, dp, bt, dq, ra);
    return hipGetLastError();
}

int occupancy_newton(bool charged)
{
    int nb = 0;
    const void *k = charged ? reinterpret_cast<const void *>(&k_run_newton<kSymTile, true>)
                            : reinterpret_cast<const void *>(&k_run_newton<kSymTile, false>);
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kSymTile, 0);
    return e == hipSuccess ? nb : -1;
}

template <int KT, int BS>
int occupancy_t(int fp32)
{
    int nb = 0;
    hipError_t e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &nb, reinterpret_cast<const void *>(&k_run_f32<KT, BS>), BS, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &nb, reinterpret_cast<const void *>(&k_run_f64<KT, BS>), BS, 0);
    return e == hipSuccess ? nb : -1;
}

uint64_t idle_ticks()
{
    static uint64_t ticks = 0;
    if (!ticks) {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
            khz <= 0)
            khz = 100000;  // 100 MHz
        ticks = (uint64_t)(kIdleSeconds * 1e3 * khz);
    }
    return ticks;
}

}  // namespace

// ---------------------------------------- memory for callers that cannot allocate

// Work queue, partial fields and counters of contexts seeded with
// ct_seed_events_noalloc: one array per GPU, held from the library's load
// until the process ends, shared by every such context on that GPU.  In host
// code its name is only a stand-in: the device address comes from
// hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t scratch_memory(int device, void **ptr, size_t *bytes)
{
    *ptr = nullptr;
    *bytes = 0;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        // with that device current (the caller has set it)
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    *bytes = kScratchBytes;
    return hipSuccess;
}

uint64_t run_idle_ticks() { return idle_ticks(); }

hipError_t launch_seed(const DevParams &dp, const DevBatch &bt, hipStream_t s)
{
    if (bt.n_total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seed, dim3((bt.n_total + 255) / 256), dim3(256), 0, s, dp, bt);
    return hipGetLastError();
}

hipError_t launch_compact(const DevParams &dp, const DevBatch &bt, hipStream_t s)
{
    if (bt.n_events <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact, dim3(bt.n_events), dim3(256), 0, s, dp, bt);
    return hipGetLastError();
}

hipError_t launch_init(const DevBatch &bt, const DevQueue &dq, const LaunchCfg &cfg,
                       int64_t max_steps, int field_only, int repulsion, hipStream_t s)
{
    hipLaunchKernelGGL(k_init, dim3(1), dim3(1024), 0, s, bt, dq, cfg.bs * cfg.kt, cfg.bs,
                       cfg.chunk, max_steps, field_only, repulsion, cfg.newton);
    return hipGetLastError();
}

#define CT_LAUNCH_CASES(X) \
    X(1, 64) X(2, 64) X(4, 64) X(1, 128) X(2, 128) X(4, 128) X(1, 256) X(2, 256) X(4, 256)

// The persistent run over the queue k_init filled; field_out receives the
// field ([N][3], carrier order) when field_only is set.
hipError_t launch_run(const DevParams &dp, const DevBatch &bt, const DevQueue &dq,
                      const LaunchCfg &cfg, int fp32, int grid, int64_t max_steps, int field_only,
                      double *field_out, hipStream_t s)
{
    if (bt.n_events <= 0 || grid <= 0) return hipSuccess;
    RunArgs ra{cfg.chunk, field_only, max_steps, idle_ticks(), field_out};
    if (cfg.newton) {
        if (!fp32 || cfg.kt != 1 || cfg.bs != kSymTile || cfg.chunk % kSymTile != 0 ||
            cfg.chunk / kSymTile > kSymMaxC)
            return hipErrorInvalidValue;
        if (cfg.newton == 2)
            hipLaunchKernelGGL((k_run_newton<kSymTile, true>), dim3(grid), dim3(kSymTile), 0, s, dp,
                               bt, dq, ra);
        else
            hipLaunchKernelGGL((k_run_newton<kSymTile, false>), dim3(grid), dim3(kSymTile), 0, s, dp,
                               bt, dq, ra);
        return hipGetLastError();
    }
#define CT_RUN_CASE(KT_, BS_) \
    if (cfg.kt == KT_ && cfg.bs == BS_) return launch_run_t<KT_, BS_>(dp, bt, dq, ra, fp32, grid, s);
    CT_LAUNCH_CASES(CT_RUN_CASE)
#undef CT_RUN_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_summary(const DevBatch &bt, Sched *sc, hipStream_t s)
{
    hipLaunchKernelGGL(k_summary, dim3(1), dim3(1024), 0, s, bt, sc);
    return hipGetLastError();
}

// Resident workgroups per compute unit of the run kernel for a configuration.
int run_occupancy(const LaunchCfg &cfg, int fp32)
{
    if (cfg.newton) return fp32 ? occupancy_newton(cfg.newton == 2) : -1;
#define CT_OCC_CASE(KT_, BS_) \
    if (cfg.kt == KT_ && cfg.bs == BS_) return occupancy_t<KT_, BS_>(fp32);
    CT_LAUNCH_CASES(CT_OCC_CASE)
#undef CT_OCC_CASE
    return -1;
}

bool launch_supported(int kt, int bs)
{
    return (kt == 1 || kt == 2 || kt == 4) && (bs == 64 || bs == 128 || bs == 256);
}

hipError_t launch_scatter_alive(const DevBatch &bt, int n_max, hipStream_t s)
{
    if (bt.n_events <= 0 || n_max <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_alive, dim3((n_max + 255) / 256, bt.n_events), dim3(256), 0, s, bt);
    return hipGetLastError();
}

hipError_t launch_philox(const DevParams &dp, const uint32_t *ctr, int64_t n, uint32_t *words,
                         double *normals, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dp, ctr, n,
                       words, normals);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace ct
