// Simplified spherical model of arXiv:2506.09712 (Sec. 2.2, Eq. 7) for gfx950:
// the repulsion field of the holes strictly closer to the event's centre,
// with the carrier update and compaction of the brute-force path.
#include "ct_device.hpp"

namespace ct {

namespace {

// ------------------------------------------------ simplified spherical model

// Eq. 7: the field at hole i is K Q_i (r_i - c) / (|r_i - c|^2 + s^2)^(3/2),
// with c the mean position of the event's drifting holes and Q_i the number
// of them strictly closer to c than i.  One workgroup takes one event through
// all its steps of a call (no other workgroup touches the event).  Q_i comes
// from a counting sort of the squared distances (keys): kSphBins LDS
// counters over [0, largest key], a bin being a monotone function of the key,
// so Q_i = (keys in lower bins) + (keys of its own bin below its own).  The
// update and the compaction (which also yields the next centre) are those of
// the brute-force path.
constexpr int kSphBlock = 512;
constexpr int kSphBins = 8192;

// Squared distance from the centre, summed left to right without fused
// multiply-adds: enclosed counts are decided by comparing these values.
__device__ __forceinline__ double sq_dist(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    return dx * dx + dy * dy + dz * dz;
}

// Bin of a key in [0, largest key]: non-decreasing in the key, always in
// [0, kSphBins) (a key that is not finite goes to the last bin).
__device__ __forceinline__ int sph_bin(double key, double scale)
{
    const double v = key * scale;  // in [0, kSphBins (1 + eps)] for finite keys
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

// Registers capped at 128 so that two workgroups share a CU: 5 keys per thread
// in registers fit without spilling, and the capped build measured faster
// than the uncapped one on mixed batches.
__global__ __launch_bounds__(kSphBlock) __attribute__((amdgpu_waves_per_eu(4)))
void k_sph(DevParams dp, DevBatch bt, SphArgs sa)
{
    constexpr int BS = kSphBlock, W = BS / 64;
    static_assert(kSphBins % BS == 0, "bins per thread");
    __shared__ int hist[kSphBins];
    __shared__ double lkeys[kSphLdsKeys];
    __shared__ int wtot[W];
    __shared__ double red[W];
    __shared__ int s_wcount[kCompactChunks * W];
    __shared__ double s_wsum[3 * W];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    const int base = bt.off[b];
    const uint32_t eid = (uint32_t)(bt.first_event_id + b);
    const bool repulsion = (dp.flags & 1u) != 0;
    int n = bt.n_act[b];  // drifting holes (the model has no electrons)
    int64_t step = bt.ev_step[b];
    int64_t taken = bt.call_steps[b];
    while (n > 0 && (sa.field_only || taken < sa.max_steps)) {
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

}  // namespace

// Simplified spherical model: every event with drifting holes to completion
// or max_steps (or, field_only, its field), one workgroup per event.
hipError_t launch_sph(const DevParams &dp, const DevBatch &bt, double *scratch, int64_t max_steps,
                      int field_only, double *field_out, hipStream_t s)
{
    if (bt.n_events <= 0) return hipSuccess;
    SphArgs sa{scratch, scratch + bt.n_total, field_only, max_steps, field_out};
    hipLaunchKernelGGL(k_sph, dim3(bt.n_events), dim3(kSphBlock), 0, s, dp, bt, sa);
    return hipGetLastError();
}

int sph_block() { return kSphBlock; }

}  // namespace ct
