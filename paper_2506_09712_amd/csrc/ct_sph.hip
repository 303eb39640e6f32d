// Simplified spherical model of arXiv:2506.09712 (Sec. 2.2, Eq. 7) for gfx950:
// the repulsion field of the holes strictly closer to the event's centre,
// with the carrier update and compaction of the brute-force path.
#include "ct_device.hpp"
#include "ct_sph_layout.hpp"

namespace ct {

namespace {

// ------------------------------------------------ simplified spherical model

// Eq. 7: the field at hole i is K Q_i (r_i - c) / (|r_i - c|^2 + s^2)^(3/2),
// with c the mean position of the event's drifting holes and Q_i the number
// of them strictly closer to c than i.  Q_i comes from a counting sort of the
// squared distances (keys): kSphBins counters over [0, largest key], a bin
// being a monotone function of the key, so Q_i = (keys in lower bins) + (keys
// of its own bin below its own).  The update and the compaction (which also
// yields the next centre) are those of the brute-force path.  A workgroup
// takes an event through all its steps of a call, alone or, for a large
// event, with the other workgroups of its group (see sph_group).

// Squared distance from the centre, summed left to right without fused
// multiply-adds: enclosed counts are decided by comparing these values.
__device__ __forceinline__ double sq_dist(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    return dx * dx + dy * dy + dz * dz;
}

// Bin of a key in [0, largest key] (scale = kSphBins / largest key): bins of
// equal width in the key.  Non-decreasing in the key (any such binning gives
// exact counts), always in [0, kSphBins) (a key that is not finite goes to
// the last bin).
__device__ __forceinline__ int sph_bin(double key, double scale)
{
    const double v = key * scale;  // in [0, kSphBins (1 + eps)] for finite keys
    return v < (double)(kSphBins - 1) ? (int)v : kSphBins - 1;
}

// The same with bins of equal width in distance, sqrt(key) (inv_max = 1 /
// largest key), for events shared by several workgroups: line-like clouds
// (tracks), whose keys crowd near 0, then spread over the bins as evenly as
// round ones.
__device__ __forceinline__ int sph_bin_dist(double key, double inv_max)
{
    const double v = sqrt(key * inv_max) * (double)kSphBins;  // in [0, kSphBins (1 + eps)]
    return v < (double)(kSphBins - 1) ? (int)v : kSphBins - 1;
}

// Largest v over the workgroup, in every thread.  Contains a workgroup
// barrier, so the workgroup's earlier LDS and memory writes are visible to
// all of it afterwards.
template <int BS>
__device__ double block_max(double v, double *red)
{
    constexpr int W = BS / 64;
    for (int o = 1; o < 64; o <<= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = red[0];
#pragma unroll
    for (int q = 1; q < W; ++q) m = fmax(m, red[q]);
    return m;
}

// Inclusive prefix sum of the kSphBins LDS counters h, in place; each thread
// owns kSphBins / BS consecutive counters.  Ends with a barrier.
template <int BS>
__device__ void scan_bins(int *h, int *wtot)
{
    constexpr int R = kSphBins / BS;
    constexpr int W = BS / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int v[R];
    int run = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        run += h[tid * R + r];
        v[r] = run;
    }
    int inc = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    int before = inc - run;
#pragma unroll
    for (int q = 0; q < W; ++q) before += q < wave ? wtot[q] : 0;
#pragma unroll
    for (int r = 0; r < R; ++r) h[tid * R + r] = before + v[r];
    __syncthreads();
}

struct SphArgs {
    double *key;        // [N] by slot: squared distance of the hole from its event's centre
    double *sorted;     // [N] by slot: the event's keys grouped by bin
    int field_only;     // 1: write the field of every drifting hole, no update
    int64_t max_steps;  // steps per event in this call
    double *field_out;  // [N][3] by carrier (field_only)
    const int32_t *single;  // events run by one workgroup each (k_sph_single)
};

// What the run over shared events needs besides (kept apart so that the
// single-workgroup kernel's arguments stay few).
struct SphGroupArgs {
    DevQueue dq;        // control block, tickets and group state
    uint64_t idle_ticks;
};

// Holes per thread whose keys stay in registers while an event's keys are
// ranked; events of at most kSphRegs * kSphBlock drifting holes keep their
// grouped keys in LDS, larger ones in the scratch arrays.
constexpr int kSphRegs = 5;
constexpr int kSphLdsKeys = kSphRegs * kSphBlock;

// Enclosed count of a hole from its key: start of its bin plus the keys of
// its bin below its own (grouped: the event's keys grouped by bin).
__device__ __forceinline__ int sph_inside(const int *hist, const double *grouped, int n,
                                          double key, int bin)
{
    const int lo = hist[bin];
    const int hi = bin + 1 < kSphBins ? hist[bin + 1] : n;
    int inside = lo;
    for (int j = lo; j < hi; ++j) inside += grouped[j] < key ? 1 : 0;
    return inside;
}

// Ranking of an event of n <= kSphLdsKeys holes: thread t keeps the keys of
// slots t + p BS in registers; the grouped keys go to LDS.  Returns the bin
// scale; hist[q] = start of bin q afterwards (ends with a barrier).
template <int BS>
__device__ double sph_rank_small(const DevBatch &bt, int base, int n, double cx, double cy,
                                 double cz, int *hist, double *lkeys, int *wtot, double *red)
{
    constexpr int P = kSphRegs;
    const int tid = threadIdx.x;
    double key[P];
    double mx = 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int s = tid + p * BS;
        key[p] = 0.0;
        if (s < n) {
            key[p] = sq_dist(bt.cx[base + s] - cx, bt.cy[base + s] - cy, bt.cz[base + s] - cz);
            mx = fmax(mx, key[p]);
        }
    }
    for (int i = tid; i < kSphBins; i += BS) hist[i] = 0;
    mx = block_max<BS>(mx, red);
    const double scale = mx > 1e-300 ? (double)kSphBins / mx : 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p)
        if (tid + p * BS < n) atomicAdd(&hist[sph_bin(key[p], scale)], 1);
    __syncthreads();
    scan_bins<BS>(hist, wtot);  // hist[q] = end of bin q
#pragma unroll
    for (int p = 0; p < P; ++p)
        if (tid + p * BS < n) lkeys[atomicSub(&hist[sph_bin(key[p], scale)], 1) - 1] = key[p];
    __syncthreads();
    return scale;
}

// The same for a larger event, through the scratch arrays.
template <int BS>
__device__ double sph_rank_large(const DevBatch &bt, const SphArgs &sa, int base, int n, double cx,
                                 double cy, double cz, int *hist, int *wtot, double *red)
{
    const int tid = threadIdx.x;
    double *key = sa.key + base;
    double *grouped = sa.sorted + base;
    double mx = 0.0;
    for (int s = tid; s < n; s += BS) {
        const double k = sq_dist(bt.cx[base + s] - cx, bt.cy[base + s] - cy, bt.cz[base + s] - cz);
        key[s] = k;
        mx = fmax(mx, k);
    }
    for (int i = tid; i < kSphBins; i += BS) hist[i] = 0;
    mx = block_max<BS>(mx, red);
    const double scale = mx > 1e-300 ? (double)kSphBins / mx : 0.0;
    for (int s = tid; s < n; s += BS) atomicAdd(&hist[sph_bin(key[s], scale)], 1);
    __syncthreads();
    scan_bins<BS>(hist, wtot);  // hist[q] = end of bin q
    for (int s = tid; s < n; s += BS) {
        const double k = key[s];
        grouped[atomicSub(&hist[sph_bin(k, scale)], 1) - 1] = k;
    }
    __syncthreads();
    return scale;
}

// LDS of a workgroup of the spherical kernel.
struct SphShared {
    int *hist;       // [kSphBins]
    double *lkeys;   // [kSphLdsKeys] (one workgroup per event only)
    int *wtot;       // [W]
    double *red;     // [W]
    int *wcount;     // [kCompactChunks * W] (one workgroup per event), [W] (shared events)
    double *wsum;    // [4 * W]
    int *range_base; // [kSphMaxGroup]
    int *flag;
};

// Barrier of the workgroups of one event.  Every thread's stores have
// completed; thread 0 adds one to the event's counter with release order and
// waits until it reaches `target` (all G workgroups, k-th barrier), then
// acquires, and the workgroup barrier orders its threads' later loads.
// Returns false if the wait outlived the liveness guard or another workgroup
// gave up (the control block's error flag is then set).
__device__ bool group_barrier(uint32_t *bar, uint32_t target, const SphGroupArgs &ga, int *flag)
{
    wait_own_stores();
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t t0 = wall_clock64();
        for (uint32_t it = 0; ld_relaxed(bar) < target; ++it) {
            if ((it & 63u) == 63u) {
                if (ld_relaxed(&ga.dq.sc->error.v)) {
                    ok = 0;
                    break;
                }
                if (wall_clock64() - t0 > ga.idle_ticks) {
                    atomicCAS(&ga.dq.sc->error.v, 0u, 3u);
                    ok = 0;
                    break;
                }
            }
            __builtin_amdgcn_s_sleep(1);
        }
        fence_acquire();
        *flag = ok;
    }
    __syncthreads();
    return *flag != 0;
}

// Exclusive prefix sum of v[0, len) in LDS, in place (len <= kSphBins);
// returns the total.  Starts reading without a barrier, ends with one.
template <int BS>
__device__ int scan_excl(int *v, int len, int *wtot)
{
    constexpr int W = BS / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (len + BS - 1) / BS;
    const int a = min(len, tid * per), e = min(len, a + per);
    int run = 0;
    for (int i = a; i < e; ++i) run += v[i];
    int inc = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    int before = inc - run, total = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        before += q < wave ? wtot[q] : 0;
        total += wtot[q];
    }
    for (int i = a; i < e; ++i) {
        const int x = v[i];
        v[i] = before;
        before += x;
    }
    __syncthreads();
    return total;
}

// Workgroup g of G owns bins [kSphBins g / G, kSphBins (g + 1) / G); the owner
// of bin q.
__device__ __forceinline__ int bin_owner(int q, int G)
{
    return ((q + 1) * G + kSphBins - 1) / kSphBins - 1;
}

// Sums of v[0..3] over the workgroup, in every thread (neighbouring lanes
// first, then the waves in order): the same order on every call.  red holds
// 4 W doubles.  Contains barriers.
template <int BS>
__device__ void block_sum4(double (&v)[4], double *red)
{
    constexpr int W = BS / 64;
#pragma unroll
    for (int c = 0; c < 4; ++c)
        for (int o = 1; o < 64; o <<= 1) v[c] += __shfl_xor(v[c], o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int c = 0; c < 4; ++c) red[4 * (threadIdx.x >> 6) + c] = v[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < W; ++q) t += red[4 * q + c];
        v[c] = t;
    }
}

// Workgroup g of the G that share event b.  Each step the drifting holes
// (packed, carrier order) are split into G contiguous slices, slice g
// [n g / G, n (g + 1) / G) being this workgroup's:
//  1. keys of the slice; the event's largest key from every slice's  (barrier)
//  2. the slice's bin histogram                                       (barrier)
//  3. for the bins this workgroup owns: each slice's first position within
//     the bin (prefix over slices), the bin totals' exclusive scan within
//     the owned range, and the range total                            (barrier)
//  4. the slice's keys scattered to their bins' positions              (barrier)
//  5. enclosed counts, field and update of the slice;
//  6. the slice's survivors and coordinate sums                       (barrier)
//     then every workgroup forms the same new count and centre (sums in
//     slice order) and copies its survivors to their packed slots        (barrier)
// All workgroups of the event run the same number of steps and barriers.
__device__ void sph_event_group(const DevParams &dp_arg, const DevBatch &bt_arg,
                                const SphArgs &sa_arg, const SphGroupArgs &ga_arg, int b, int g,
                                int G, const SphShared &sh)
{
    const DevParams &dp = dp_arg;
    const DevBatch &bt = bt_arg;
    const SphArgs &sa = sa_arg;
    const SphGroupArgs &ga = ga_arg;
    constexpr int BS = kSphSharedBlock, W = BS / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int base = bt.off[b];
    const uint32_t eid = (uint32_t)(bt.first_event_id + b);
    const bool repulsion = (dp.flags & 1u) != 0;
    const SphGroupView gv = sph_group_view(ga.dq.grp + ga.dq.grp_off[b], G);
    double *key = sa.key + base;
    double *grouped = sa.sorted + base;
    const int q0 = kSphBins * g / G, q1 = kSphBins * (g + 1) / G;
    uint32_t nbar = 0;
    int n = bt.n_act[b];
    int64_t step = bt.ev_step[b];
    int64_t taken = bt.call_steps[b];
    double cx = bt.ref[4 * b + 0], cy = bt.ref[4 * b + 1], cz = bt.ref[4 * b + 2];
    while (n > 0 && (sa.field_only || taken < sa.max_steps)) {
        const DevParams &dp = reload_arg(dp_arg);  // read again in every step
        const DevBatch &bt = reload_arg(bt_arg);
        const SphArgs &sa = reload_arg(sa_arg);
        const SphGroupArgs &ga = reload_arg(ga_arg);
        const int lo = (int)((int64_t)n * g / G), hi = (int)((int64_t)n * (g + 1) / G);
        double scale = 0.0;
        if (repulsion) {
            double mx = 0.0;
            for (int s = lo + tid; s < hi; s += BS) {
                const double k = sq_dist(bt.cx[base + s] - cx, bt.cy[base + s] - cy, bt.cz[base + s] - cz);
                key[s] = k;
                mx = fmax(mx, k);
            }
            for (int i = tid; i < kSphBins; i += BS) sh.hist[i] = 0;
            mx = block_max<BS>(mx, sh.red);
            if (tid == 0) st_dev(&gv.gmax[g], mx);
            if (!group_barrier(gv.bar, (uint32_t)G * ++nbar, ga, sh.flag)) return;
            double M = 0.0;
            for (int r = 0; r < G; ++r) M = fmax(M, gv.gmax[r]);
            scale = M > 1e-300 ? 1.0 / M : 0.0;
            for (int s = lo + tid; s < hi; s += BS) atomicAdd(&sh.hist[sph_bin_dist(key[s], scale)], 1);
            __syncthreads();
            for (int q = tid; q < kSphBins; q += BS) st_dev(&gv.ghist[g * kSphBins + q], sh.hist[q]);
            if (!group_barrier(gv.bar, (uint32_t)G * ++nbar, ga, sh.flag)) return;
            for (int q = q0 + tid; q < q1; q += BS) {
                // eight slices' counts at a time (independent loads), then their prefix
                int run = 0;
                for (int r0 = 0; r0 < G; r0 += 8) {
                    int v[8];
#pragma unroll
                    for (int r = 0; r < 8; ++r) v[r] = r0 + r < G ? gv.ghist[(r0 + r) * kSphBins + q] : 0;
#pragma unroll
                    for (int r = 0; r < 8; ++r) {
                        if (r0 + r < G) st_dev(&gv.ghist[(r0 + r) * kSphBins + q], run);
                        run += v[r];
                    }
                }
                sh.hist[q] = run;
            }
            __syncthreads();
            const int range_tot = scan_excl<BS>(sh.hist + q0, q1 - q0, sh.wtot);
            for (int q = q0 + tid; q < q1; q += BS) st_dev(&gv.colscan[q], sh.hist[q]);
            if (tid == 0) st_dev(&gv.range_tot[g], range_tot);
            if (!group_barrier(gv.bar, (uint32_t)G * ++nbar, ga, sh.flag)) return;
            if (tid == 0) {
                int run = 0;
                for (int r = 0; r < G; ++r) {
                    sh.range_base[r] = run;
                    run += gv.range_tot[r];
                }
            }
            __syncthreads();
#pragma unroll 8
            for (int q = tid; q < kSphBins; q += BS)
                sh.hist[q] = sh.range_base[bin_owner(q, G)] + gv.colscan[q] + gv.ghist[g * kSphBins + q];
            __syncthreads();
            for (int s = lo + tid; s < hi; s += BS) {
                const double k = key[s];
                st_dev(&grouped[atomicAdd(&sh.hist[sph_bin_dist(k, scale)], 1)], k);
            }
            if (!group_barrier(gv.bar, (uint32_t)G * ++nbar, ga, sh.flag)) return;
        }
#pragma unroll 1
        for (int s = lo + tid; s < hi; s += BS) {
            const double x = bt.cx[base + s], y = bt.cy[base + s], z = bt.cz[base + s];
            const int k = bt.idx[base + s];
            double ex = 0.0, ey = 0.0, ez = 0.0;
            if (repulsion) {
                const double dx = x - cx, dy = y - cy, dz = z - cz;
                const double kk = sq_dist(dx, dy, dz);
                const int bin = sph_bin_dist(kk, scale);
                // the bin's keys are grouped[start, end) (clamped to the n keys)
                const int start = min(n, sh.range_base[bin_owner(bin, G)] + gv.colscan[bin]);
                const int end = bin + 1 < kSphBins
                                    ? min(n, sh.range_base[bin_owner(bin + 1, G)] + gv.colscan[bin + 1])
                                    : n;
                int inside = start;
                for (int j = start; j < end; ++j) inside += grouped[j] < kk ? 1 : 0;
                if (inside > 0) {
                    const double f = dp.K * (double)inside * inv_r3_f64(kk + dp.s2);
                    ex = f * dx;
                    ey = f * dy;
                    ez = f * dz;
                }
            }
            if (sa.field_only) {
                const int64_t carrier = base + k;
                sa.field_out[3 * carrier + 0] = ex;
                sa.field_out[3 * carrier + 1] = ey;
                sa.field_out[3 * carrier + 2] = ez;
            } else {
                advance_at<true>(dp, bt, b, base + s, x, y, z, k, bt.rngid[base + k], ex, ey, ez,
                                 step, eid);
            }
        }
        if (sa.field_only) return;
        __syncthreads();
        // survivors of the slice (holes with z > 0 after the step) and their sums
        double acc[4] = {0.0, 0.0, 0.0, 0.0};  // x, y, z sums and the count
        for (int s = lo + tid; s < hi; s += BS) {
            const double z = bt.nz[base + s];
            if (z > 0.0) {
                acc[0] += bt.nx[base + s];
                acc[1] += bt.ny[base + s];
                acc[2] += z;
                acc[3] += 1.0;
            }
        }
        block_sum4<BS>(acc, sh.wsum);
        if (tid == 0) {
            st_dev(&gv.kept[g], (int)acc[3]);
            st_dev(&gv.sums[3 * g + 0], acc[0]);
            st_dev(&gv.sums[3 * g + 1], acc[1]);
            st_dev(&gv.sums[3 * g + 2], acc[2]);
        }
        if (!group_barrier(gv.bar, (uint32_t)G * ++nbar, ga, sh.flag)) return;
        int off = 0, total = 0;
        double X = 0.0, Y = 0.0, Z = 0.0;
        for (int r = 0; r < G; ++r) {
            const int kr = gv.kept[r];
            off += r < g ? kr : 0;
            total += kr;
            X += gv.sums[3 * r + 0];
            Y += gv.sums[3 * r + 1];
            Z += gv.sums[3 * r + 2];
        }
        for (int w0 = lo; w0 < hi; w0 += BS) {
            const int s = w0 + tid;
            const int sl = base + min(s, hi - 1);  // loads independent of the ballot
            const double px = bt.nx[sl], py = bt.ny[sl], pz = bt.nz[sl];
            const int pk = bt.nidx[sl];
            const bool a = s < hi && pz > 0.0;
            const uint64_t mask = __ballot(a);
            const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            if (lane == 0) sh.wcount[wave] = __popcll(mask);
            __syncthreads();
            int before = 0, wtotal = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int v = sh.wcount[q];
                before += q < wave ? v : 0;
                wtotal += v;
            }
            if (a) {
                const int d = base + off + before + rank;
                st_dev(&bt.cx[d], px);
                st_dev(&bt.cy[d], py);
                st_dev(&bt.cz[d], pz);
                st_dev(&bt.idx[d], pk);
            }
            off += wtotal;
            __syncthreads();  // the wave counts are read before the next window overwrites them
        }
        if (total > 0) {
            cx = X / total;
            cy = Y / total;
            cz = Z / total;
        }
        if (g == 0 && tid == 0) {
            st_dev(&bt.n_hole[b], total);
            if (total > 0) {
                st_dev(&bt.ref[4 * b + 0], cx);
                st_dev(&bt.ref[4 * b + 1], cy);
                st_dev(&bt.ref[4 * b + 2], cz);
            }
            st_dev(&bt.n_act[b], total);
            bt.pairs[b] += (uint64_t)n * (uint64_t)(n - 1);
            bt.hsteps[b] += (uint64_t)n;
            st_dev(&bt.ev_step[b], step + 1);
            st_dev(&bt.ev_taken[b], bt.ev_taken[b] + 1);
            st_dev(&bt.call_steps[b], taken + 1);
        }
        if (!group_barrier(gv.bar, (uint32_t)G * ++nbar, ga, sh.flag)) return;
        n = total;
        ++step;
        ++taken;
    }
}

// Registers capped at 128 so that two workgroups share a CU: 5 keys per thread
// in registers fit without spilling, and the capped build measured faster
// than the uncapped one on mixed batches.  Two kernels, so that each path
// gets its own register allocation: k_sph_single takes every event of the
// batch that one workgroup runs (one workgroup per such event, from the list
// sa.single), k_sph_shared the events shared by several.
__global__ __launch_bounds__(kSphBlock) __attribute__((amdgpu_waves_per_eu(4)))
void k_sph_single(DevParams dp_arg, DevBatch bt_arg, SphArgs sa_arg)
{
    const DevParams &dp = dp_arg;
    const DevBatch &bt = bt_arg;
    const SphArgs &sa = sa_arg;
    constexpr int BS = kSphBlock, W = BS / 64;
    static_assert(kSphBins % BS == 0, "bins per thread");
    __shared__ int hist[kSphBins];
    __shared__ double lkeys[kSphLdsKeys];
    __shared__ int wtot[W];
    __shared__ double red[W];
    __shared__ int s_wcount[kCompactChunks * W];
    __shared__ double s_wsum[3 * W];
    const int b = sa.single[blockIdx.x];
    const int tid = threadIdx.x;
    const int base = bt.off[b];
    const uint32_t eid = (uint32_t)(bt.first_event_id + b);
    const bool repulsion = (dp.flags & 1u) != 0;
    int n = bt.n_act[b];  // drifting holes (the model has no electrons)
    int64_t step = bt.ev_step[b];
    int64_t taken = bt.call_steps[b];
    while (n > 0 && (sa.field_only || taken < sa.max_steps)) {
        const DevParams &dp = reload_arg(dp_arg);  // read again in every step
        const DevBatch &bt = reload_arg(bt_arg);
        const SphArgs &sa = reload_arg(sa_arg);
        const double cx = bt.ref[4 * b + 0], cy = bt.ref[4 * b + 1], cz = bt.ref[4 * b + 2];
        const bool small = n <= kSphLdsKeys;
        double scale = 0.0;
        if (repulsion)
            scale = small ? sph_rank_small<BS>(bt, base, n, cx, cy, cz, hist, lkeys, wtot, red)
                          : sph_rank_large<BS>(bt, sa, base, n, cx, cy, cz, hist, wtot, red);
        // the field and update of every hole; its key is recomputed from the
        // position exactly as the ranking computed it
#pragma unroll 1
        for (int s = tid; s < n; s += BS) {
            const double x = bt.cx[base + s], y = bt.cy[base + s], z = bt.cz[base + s];
            const int k = bt.idx[base + s];
            double ex = 0.0, ey = 0.0, ez = 0.0;
            if (repulsion) {
                const double dx = x - cx, dy = y - cy, dz = z - cz;
                const double key = sq_dist(dx, dy, dz);
                const int bin = sph_bin(key, scale);
                const int inside = small ? sph_inside(hist, lkeys, n, key, bin)
                                         : sph_inside(hist, sa.sorted + base, n, key, bin);
                if (inside > 0) {
                    const double f = dp.K * (double)inside * inv_r3_f64(key + dp.s2);
                    ex = f * dx;
                    ey = f * dy;
                    ez = f * dz;
                }
            }
            if (sa.field_only) {
                const int64_t carrier = base + k;
                sa.field_out[3 * carrier + 0] = ex;
                sa.field_out[3 * carrier + 1] = ey;
                sa.field_out[3 * carrier + 2] = ez;
            } else {
                advance_at<true>(dp, bt, b, base + s, x, y, z, k, bt.rngid[base + k], ex, ey, ez,
                                 step, eid);
            }
        }
        if (sa.field_only) break;
        __syncthreads();  // every update is written before the compaction reads it
        int holes_kept = 0;
        n = compact_event<BS>(bt, b, n, n, dp.H, 1, s_wcount, s_wsum, holes_kept);
        ++step;
        ++taken;
    }
}

// A persistent grid of resident workgroups claims tickets in order: G
// consecutive ones for an event shared by G workgroups (tickets of
// single-workgroup events are skipped).  Claimed tickets are always a prefix,
// so every shared event but the last claimed one has all its workgroups
// running; as long as the grid holds at least G workgroups, the missing ones
// of the last event are claimed as soon as others finish.
// 1024 threads per workgroup (16 waves per CU) measured 14-20% faster than 512
// on shared events, whose steps alternate short phases with barriers.
__global__ __launch_bounds__(kSphSharedBlock) __attribute__((amdgpu_waves_per_eu(4)))
void k_sph_shared(DevParams dp, DevBatch bt, SphArgs sa, SphGroupArgs ga)
{
    constexpr int W = kSphSharedBlock / 64;
    static_assert(kSphBins % kSphSharedBlock == 0, "bins per thread");
    __shared__ int hist[kSphBins];
    __shared__ int wtot[W];
    __shared__ double red[W];
    __shared__ int s_wcount[W];
    __shared__ double s_wsum[4 * W];
    __shared__ int s_range_base[kSphMaxGroup];
    __shared__ int s_flag, s_ticket;
    const SphShared sh{hist, nullptr, wtot, red, s_wcount, s_wsum, s_range_base, &s_flag};
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0)
            s_ticket = ld_relaxed(&ga.dq.sc->error.v) ? ga.dq.n_tickets
                                                      : (int)add_relaxed(&ga.dq.sc->head.v, 1u);
        __syncthreads();
        const int t = s_ticket;
        if (t >= ga.dq.n_tickets) break;
        int lo = 0, hi = bt.n_events;  // tk_off[lo] <= t < tk_off[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (ga.dq.tk_off[mid] <= t) lo = mid;
            else hi = mid;
        }
        const int G = ga.dq.tk_off[lo + 1] - ga.dq.tk_off[lo];
        if (G > 1) sph_event_group(dp, bt, sa, ga, lo, t - ga.dq.tk_off[lo], G, sh);
    }
}

// Ticket counter, error flag and the barrier counters of shared events,
// cleared before a run.
__global__ __launch_bounds__(256) void k_sph_init(DevBatch bt, DevQueue dq)
{
    const int tid = blockIdx.x * 256 + threadIdx.x;
    if (tid == 0) {
        dq.sc->head.v = 0;
        dq.sc->error.v = 0;
    }
    if (tid < bt.n_events && dq.tk_off[tid + 1] - dq.tk_off[tid] > 1)
        *reinterpret_cast<uint32_t *>(dq.grp + dq.grp_off[tid]) = 0u;
}

}  // namespace

// Simplified spherical model: every event with drifting holes to completion
// or max_steps (or, field_only, its field): the grid_single events of the
// list dq.single, one workgroup each, then the shared ones on grid_shared
// resident workgroups.
hipError_t launch_sph(const DevParams &dp, const DevBatch &bt, const DevQueue &dq, double *scratch,
                      int grid_single, int grid_shared, int64_t max_steps, int field_only,
                      double *field_out, hipStream_t s)
{
    if (bt.n_events <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sph_init, dim3((bt.n_events + 255) / 256), dim3(256), 0, s, bt, dq);
    const SphArgs sa{scratch, scratch + bt.n_total, field_only, max_steps, field_out, dq.single};
    if (grid_single > 0)
        hipLaunchKernelGGL(k_sph_single, dim3(grid_single), dim3(kSphBlock), 0, s, dp, bt, sa);
    if (grid_shared > 0)
        hipLaunchKernelGGL(k_sph_shared, dim3(grid_shared), dim3(kSphSharedBlock), 0, s, dp, bt, sa,
                           SphGroupArgs{dq, run_idle_ticks()});
    return hipGetLastError();
}

// Resident workgroups per CU of the shared-event kernel.
int sph_occupancy()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&k_sph_shared),
                                                     kSphSharedBlock, 0) != hipSuccess)
        return -1;
    return nb;
}

}  // namespace ct
