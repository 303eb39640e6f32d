// HIP kernels of the brute-force charge-transport Monte Carlo for gfx950
// (Xie et al., arXiv:2506.09712, Sec. 2.1 and Appendix A, Algorithm 1).
//
// One time step of a batch is three launches on one stream:
//   k_step     per (event, target tile, source chunk) workgroup: the all-pairs
//              repulsion field of Eq. 4 over the event's drifting holes, with
//              source tiles staged in LDS and one thread per KT targets; for
//              unsplit events the update of Eqs. 3, 5 and 6 (drift field,
//              mobility, diffusion, collection, pixel count) runs in the same
//              kernel;
//   k_update   for events whose sources were split over several workgroups:
//              sums the partial fields in chunk order and applies the update;
//   k_compact  one workgroup per event: keeps the holes still drifting, in
//              carrier order (wave ballot + mbcnt prefix, workgroup scan),
//              recomputes the event centroid and counts the step.
#include <math.h>

#include "ct_internal.hpp"

namespace ct {

namespace {

constexpr uint32_t kDomainDiffusion = 0u;
constexpr uint32_t kDomainCloud = 1u;
constexpr int kCompactThreads = 1024;

// ------------------------------------------------------------------ Philox

struct Ctr {
    uint32_t c0, c1, c2, c3;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products, Weyl-sequence round keys.
__device__ __forceinline__ Ctr philox10(Ctr c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.c0, hi0 = __umulhi(0xD2511F53u, c.c0);
        const uint32_t lo1 = 0xCD9E8D57u * c.c2, hi1 = __umulhi(0xCD9E8D57u, c.c2);
        c = Ctr{hi1 ^ c.c1 ^ k0, lo1, hi0 ^ c.c3 ^ k1, lo0};
    }
    return c;
}

__device__ __forceinline__ double to_unit(uint32_t w)
{
    return ((double)w + 0.5) * (1.0 / 4294967296.0);  // in (0, 1)
}

// Three standard normals from one Philox block (Box-Muller on (u0,u1), (u2,u3)).
__device__ void normals3(const DevParams &dp, Ctr ctr, double n[3])
{
    const Ctr w = philox10(ctr, dp.key0, dp.key1);
    const double u0 = to_unit(w.c0), u1 = to_unit(w.c1);
    const double u2 = to_unit(w.c2), u3 = to_unit(w.c3);
    const double ra = sqrt(-2.0 * log(u0));
    const double rb = sqrt(-2.0 * log(u2));
    double s1, c1;
    sincospi(2.0 * u1, &s1, &c1);  // sin, cos of 2 pi u1 without a general range reduction
    n[0] = ra * c1;
    n[1] = ra * s1;
    n[2] = rb * cospi(2.0 * u3);
}

// ------------------------------------------------------------------ physics

__device__ __forceinline__ double mobility(const DevParams &dp, double e_mag)
{
    if (dp.mobility == 1) return dp.mu0;
    return dp.mu0 / pow(1.0 + pow(e_mag / dp.ec, dp.beta), dp.inv_beta);
}

__device__ __forceinline__ int pixel_bin(const DevParams &dp, double x, double y)
{
    const int G = dp.grid_n;
    const double fx = floor((x + dp.half_width) / dp.pitch);
    const double fy = floor((y + dp.half_width) / dp.pitch);
    if (fx >= 0.0 && fx < (double)G && fy >= 0.0 && fy < (double)G) return (int)fy * G + (int)fx;
    return G * G;
}

__device__ void collect(const DevParams &dp, const DevBatch &bt, int b, int carrier, double x,
                        double y, double z, int64_t step)
{
    bt.out_xyz[3 * (int64_t)carrier + 0] = x;
    bt.out_xyz[3 * (int64_t)carrier + 1] = y;
    bt.out_xyz[3 * (int64_t)carrier + 2] = z;
    bt.out_cstep[carrier] = (int32_t)step;
    const int g1 = dp.grid_n * dp.grid_n + 1;
    atomicAdd(&bt.pix[(int64_t)b * g1 + pixel_bin(dp, x, y)], 1);
}

// Update of one drifting hole (Eqs. 3, 5, 6 and Algorithm 1): E_rep is the
// repulsion field at the step-start snapshot, already scaled by K.
__device__ void advance(const DevParams &dp, const DevBatch &bt, int b, int slot, double ex,
                        double ey, double ez_rep, int64_t step, uint32_t eid)
{
    const double x = bt.cx[slot], y = bt.cy[slot], z = bt.cz[slot];
    const int k = bt.idx[slot];
    const int carrier = bt.off[b] + k;
    double ez = ez_rep;
    if (dp.flags & 2u) ez += -(dp.e0 - dp.e1 * z);
    const double e_mag = sqrt(ex * ex + ey * ey + ez * ez);
    const double mu = mobility(dp, e_mag);
    double g[3] = {0.0, 0.0, 0.0};
    double hop = 0.0;
    if (dp.flags & 4u) {
        hop = sqrt(2.0 * (mu * dp.kT) * dp.dt);
        normals3(dp, Ctr{(uint32_t)bt.rngid[carrier], (uint32_t)step, eid, kDomainDiffusion}, g);
    }
    const double x1 = x + mu * ex * dp.dt + hop * g[0];
    const double y1 = y + mu * ey * dp.dt + hop * g[1];
    double z1 = z + mu * ez * dp.dt + hop * g[2];
    if (z1 > dp.H) z1 = 2.0 * dp.H - z1;  // mirror at the entrance side
    bt.nx[slot] = x1;
    bt.ny[slot] = y1;
    bt.nz[slot] = z1;
    if (z1 <= 0.0) collect(dp, bt, b, carrier, x1, y1, z1, step + 1);
}

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

// FP32: targets and sources relative to the event centroid.  Sources past the
// end of a tile are parked at 1e18 um, where the pair term underflows to 0.
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

// FP64 reciprocal cube of sqrt(r2): hardware estimate refined by one
// third-order Newton step, y <- y (1 + e/2 + 3 e^2/8), e = 1 - r2 y^2.
__device__ __forceinline__ double inv_r3_f64(double r2)
{
    double y = __builtin_amdgcn_rsq(r2);
    const double e = fma(-r2, y * y, 1.0);
    y = fma(y * e, fma(e, 0.375, 0.5), y);
    return y * y * y;
}

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

// Sources of an event split into nsplit chunks: equal lengths rounded up to
// whole LDS tiles, so every chunk boundary is also a tile boundary.
__device__ __forceinline__ int chunk_length(int n, int nsplit, int bs)
{
    if (nsplit <= 1) return n;
    const int per = (n + nsplit - 1) / nsplit;
    return (per + bs - 1) / bs * bs;
}

// Pair work of one item.  Thread t owns targets tile*BS*KT + m*BS + t
// (m < KT); the workgroup stages the sources in LDS tiles of BS.  Waves whose
// targets all lie past the event's end only help staging.  For unsplit events
// the update follows in the same kernel; otherwise the raw partial sum is
// stored for k_update.
template <int KT, int BS, bool F32>
__device__ void run_item(const DevParams &dp, const DevBatch &bt, const Item it, int chunk,
                         int field_only, double *field_out, void *lds)
{
    const int b = it.b;
    const int n = bt.n_act[b];
    const int t0 = it.tile * (BS * KT);
    const int clen = chunk_length(n, it.nsplit, BS);
    const int sb = it.c * clen;
    const int se = min(n, sb + clen);
    const int base = bt.off[b];
    const int tid = threadIdx.x;
    const bool wave_has_targets = t0 + (tid & ~63) < n;

    double ex[KT], ey[KT], ez[KT];
#pragma unroll
    for (int m = 0; m < KT; ++m) ex[m] = ey[m] = ez[m] = 0.0;

    if (dp.flags & 1u) {
        if constexpr (F32) {
            float4 *tile = static_cast<float4 *>(lds);
            const double rx = bt.ref[4 * b + 0], ry = bt.ref[4 * b + 1], rz = bt.ref[4 * b + 2];
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
            for (int s0 = sb; s0 < se; s0 += BS) {
                __syncthreads();
                const int j = s0 + tid;
                float4 v = make_float4(1e18f, 1e18f, 1e18f, 0.0f);
                if (j < se)
                    v = make_float4((float)(bt.cx[base + j] - rx), (float)(bt.cy[base + j] - ry),
                                    (float)(bt.cz[base + j] - rz), 0.0f);
                tile[tid] = v;
                __syncthreads();
                if (!wave_has_targets) continue;
                const int cnt = (min(BS, se - s0) + CT_PAIR_UNROLL - 1) / CT_PAIR_UNROLL * CT_PAIR_UNROLL;
                float ax[KT], ay[KT], az[KT];
#pragma unroll
                for (int m = 0; m < KT; ++m) ax[m] = ay[m] = az[m] = 0.0f;
                pairs_f32<KT>(tile, cnt, dp.s2f, tx, ty, tz, ax, ay, az);
#pragma unroll
                for (int m = 0; m < KT; ++m) {  // fold the tile's FP32 partial into FP64
                    ex[m] += (double)ax[m];
                    ey[m] += (double)ay[m];
                    ez[m] += (double)az[m];
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
            for (int s0 = sb; s0 < se; s0 += BS) {
                __syncthreads();
                const int j = s0 + tid;
                if (j < se) tile[tid] = D4{bt.cx[base + j], bt.cy[base + j], bt.cz[base + j], 0.0};
                __syncthreads();
                if (!wave_has_targets) continue;
                const int cnt = min(BS, se - s0);
                const int cnt4 = cnt & ~3;
                for (int j0 = 0; j0 < cnt4; j0 += 4) {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        pair_f64<KT>(tile[j0 + u], s2, tx, ty, tz, ex, ey, ez);
                }
                for (int jj = cnt4; jj < cnt; ++jj) pair_f64<KT>(tile[jj], s2, tx, ty, tz, ex, ey, ez);
            }
        }
    }
#pragma unroll
    for (int m = 0; m < KT; ++m) {
        const int s = t0 + m * BS + tid;
        if (s >= n) continue;
        if (it.nsplit == 1) {
            field_or_advance(dp, bt, b, base + s, dp.K * ex[m], dp.K * ey[m], dp.K * ez[m],
                             field_only, field_out);
        } else {
            const int64_t N = bt.n_total;
            bt.part[(3 * (int64_t)it.c + 0) * N + base + s] = ex[m];
            bt.part[(3 * (int64_t)it.c + 1) * N + base + s] = ey[m];
            bt.part[(3 * (int64_t)it.c + 2) * N + base + s] = ez[m];
        }
    }
}

// Persistent step kernel: a fixed grid sized to the resident capacity of the
// device; each workgroup takes the next item of the step's work list with one
// atomic until the list is exhausted, so every workgroup exits.
// Resident waves per SIMD the pair kernels are compiled for: the pair loop
// needs few registers, the update epilogue many; capping registers so that 8
// waves share each SIMD (FP32) measured 5-7% faster than the unconstrained
// allocation (84 registers, 5 waves).
#ifndef CT_F32_WAVES_PER_EU
#define CT_F32_WAVES_PER_EU 8
#endif
#ifndef CT_F64_WAVES_PER_EU
#define CT_F64_WAVES_PER_EU 4
#endif

// Persistent step kernel: a fixed grid sized to the resident capacity of the
// device; each workgroup takes the next item of the step's work list with one
// atomic until the list is exhausted, so every workgroup exits.
template <int KT, int BS, bool F32>
__device__ __forceinline__ void step_loop(const DevParams &dp, const DevBatch &bt, int chunk,
                                          int field_only, double *field_out, void *lds)
{
    __shared__ int s_item;
    const int n_items = *bt.n_items;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(bt.counter, 1u);
        __syncthreads();
        const int i = s_item;
        if (i >= n_items) break;
        run_item<KT, BS, F32>(dp, bt, bt.work[i], chunk, field_only, field_out, lds);
    }
}

template <int KT, int BS>
__global__ __launch_bounds__(BS)
__attribute__((amdgpu_waves_per_eu(KT == 1 ? CT_F32_WAVES_PER_EU : 5)))
void k_step_f32(DevParams dp, DevBatch bt, int chunk, int field_only, double *field_out)
{
    __shared__ float4 lds[BS];
    step_loop<KT, BS, true>(dp, bt, chunk, field_only, field_out, lds);
}

template <int KT, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(CT_F64_WAVES_PER_EU)))
void k_step_f64(DevParams dp, DevBatch bt, int chunk, int field_only, double *field_out)
{
    __shared__ D4 lds[BS];
    step_loop<KT, BS, false>(dp, bt, chunk, field_only, field_out, lds);
}

// Work list of one step (one workgroup of 1024): per event ceil(n/T) target
// tiles times ceil(n/chunk) source chunks, events in order, items of an event
// contiguous.  Also resets the item counter and the drifting-hole total.
// Up to kPlanLds events keep their item offsets in LDS and every thread emits
// items located by binary search; larger batches emit one event per wave.
constexpr int kPlanLds = 4096;

__global__ __launch_bounds__(1024) void k_plan(DevBatch bt, int T, int chunk)
{
    __shared__ int wtot[16];
    __shared__ int carry;
    __shared__ int s_base[kPlanLds + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int B = bt.n_events;
    const bool in_lds = B <= kPlanLds;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int e0 = 0; e0 < B; e0 += 1024) {
        const int e = e0 + tid;
        int items = 0;
        if (e < B) {
            const int n = bt.n_act[e];
            if (n > 0) items = ((n + T - 1) / T) * (chunk > 0 ? (n + chunk - 1) / chunk : 1);
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
        if (e < B) {
            const int base = carry + before + v - items;
            if (in_lds) s_base[e] = base;
            else bt.item_base[e] = base;
        }
        __syncthreads();
        if (tid == 0) carry += total;
        __syncthreads();
    }
    const int total = min(carry, bt.work_cap);
    if (in_lds) {
        if (tid == 0) s_base[B] = carry;
        __syncthreads();
        for (int i = tid; i < total; i += 1024) {
            int lo = 0, hi = B;  // s_base[lo] <= i < s_base[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_base[mid] <= i) lo = mid;
                else hi = mid;
            }
            const int n = bt.n_act[lo];
            const int ns = chunk > 0 ? (n + chunk - 1) / chunk : 1;
            const int k = i - s_base[lo];
            bt.work[i] = Item{lo, k / ns, k % ns, ns};
        }
    } else {
        for (int e = wave; e < B; e += 16) {
            const int n = bt.n_act[e];
            if (n <= 0) continue;
            const int ns = chunk > 0 ? (n + chunk - 1) / chunk : 1;
            const int items = ((n + T - 1) / T) * ns;
            const int base = bt.item_base[e];
            for (int i = lane; i < items; i += 64)
                if (base + i < bt.work_cap) bt.work[base + i] = Item{e, i / ns, i % ns, ns};
        }
    }
    if (tid == 0) {
        *bt.n_items = total;
        *bt.counter = 0u;
        bt.active[0] = 0;
    }
}

// Events split over several source chunks: sum the partial fields in chunk
// order, then update.  Grid: (slot tiles of 256, events).
__global__ __launch_bounds__(256) void k_update(DevParams dp, DevBatch bt, int chunk,
                                                int field_only, double *field_out)
{
    const int b = blockIdx.y;
    const int n = bt.n_act[b];
    const int nsplit = chunk > 0 ? (n + chunk - 1) / chunk : 1;
    if (nsplit <= 1) return;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const int slot = bt.off[b] + s;
    const int64_t N = bt.n_total;
    double ex = 0.0, ey = 0.0, ez = 0.0;
    for (int c = 0; c < nsplit; ++c) {
        ex += bt.part[(3 * (int64_t)c + 0) * N + slot];
        ey += bt.part[(3 * (int64_t)c + 1) * N + slot];
        ez += bt.part[(3 * (int64_t)c + 2) * N + slot];
    }
    field_or_advance(dp, bt, b, slot, dp.K * ex, dp.K * ey, dp.K * ez, field_only, field_out);
}

// One workgroup per event.  Holes with z > 0 after the step survive; they
// are packed to the front of the event's slots in carrier order.  Each wave
// ranks its survivors with a 64-bit ballot and mbcnt, the workgroup adds the
// wave totals; carrier indices are compacted in place (every read of a chunk
// precedes the barrier, every write follows it and lands at or below it).
__global__ __launch_bounds__(kCompactThreads) void k_compact(DevParams dp, DevBatch bt,
                                                             int count_step)
{
    (void)dp;
    constexpr int W = kCompactThreads / 64;
    __shared__ int wcount[W];
    __shared__ double wsum[3][W];
    const int b = blockIdx.x;
    const int n = bt.n_act[b];
    const int base = bt.off[b];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    int kept = 0;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int c0 = 0; c0 < n; c0 += kCompactThreads) {
        const int i = c0 + tid;
        bool alive = false;
        double x = 0.0, y = 0.0, z = 0.0;
        int k = 0;
        if (i < n) {
            z = bt.nz[base + i];
            alive = z > 0.0;
            if (alive) {
                x = bt.nx[base + i];
                y = bt.ny[base + i];
                k = bt.idx[base + i];
            }
        }
        const uint64_t mask = __ballot(alive);
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        if (lane == 0) wcount[wave] = __popcll(mask);
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const int v = wcount[q];
            before += q < wave ? v : 0;
            total += v;
        }
        if (alive) {
            const int d = base + kept + before + rank;
            bt.cx[d] = x;
            bt.cy[d] = y;
            bt.cz[d] = z;
            bt.idx[d] = k;
            sx += x;
            sy += y;
            sz += z;
        }
        kept += total;
        __syncthreads();
    }
    // fixed-order reduction of the survivors' coordinate sums (deterministic)
    for (int o = 32; o > 0; o >>= 1) {
        sx += __shfl_down(sx, o);
        sy += __shfl_down(sy, o);
        sz += __shfl_down(sz, o);
    }
    if (lane == 0) {
        wsum[0][wave] = sx;
        wsum[1][wave] = sy;
        wsum[2][wave] = sz;
    }
    __syncthreads();
    if (tid == 0) {
        double X = 0.0, Y = 0.0, Z = 0.0;
        for (int q = 0; q < W; ++q) {
            X += wsum[0][q];
            Y += wsum[1][q];
            Z += wsum[2][q];
        }
        if (kept > 0) {
            bt.ref[4 * b + 0] = X / kept;
            bt.ref[4 * b + 1] = Y / kept;
            bt.ref[4 * b + 2] = Z / kept;
        }
        bt.n_act[b] = kept;
        if (count_step && n > 0) {
            bt.pairs[b] += (uint64_t)n * (uint64_t)(n - 1);
            bt.hsteps[b] += (uint64_t)n;
            bt.ev_step[b] += 1;
            bt.ev_taken[b] += 1;
        }
        if (kept > 0) atomicAdd((unsigned long long *)bt.active, (unsigned long long)kept);
    }
}

// Initial clouds (Algorithm 1, initialisation; Eq. 2 width).  One thread per
// carrier; the event is found by binary search over the slot offsets.
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
    const int k = g - bt.off[b];
    double x, y, z;
    const int d0 = bt.dep_off[b], nd = bt.dep_off[b + 1] - d0;
    if (nd > 0) {
        const double *d = bt.deposits + 3 * (int64_t)(d0 + k % nd);
        double n3[3];
        normals3(dp, Ctr{(uint32_t)bt.rngid[g], 0u, (uint32_t)(bt.first_event_id + b), kDomainCloud},
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
    if (z > dp.H) z = 2.0 * dp.H - z;
    bt.idx[g] = k;
    bt.nx[g] = x;
    bt.ny[g] = y;
    bt.nz[g] = z;
    bt.out_cstep[g] = -1;
    if (z <= 0.0) collect(dp, bt, b, g, x, y, z, bt.start[b]);
}

// Current positions of drifting holes into the carrier-ordered output.
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
hipError_t launch_step_t(const DevParams &dp, const DevBatch &bt, const LaunchCfg &cfg, int fp32,
                         int grid, int field_only, double *field_out, hipStream_t s)
{
    if (fp32)
        hipLaunchKernelGGL((k_step_f32<KT, BS>), dim3(grid), dim3(BS), 0, s, dp, bt, cfg.chunk,
                           field_only, field_out);
    else
        hipLaunchKernelGGL((k_step_f64<KT, BS>), dim3(grid), dim3(BS), 0, s, dp, bt, cfg.chunk,
                           field_only, field_out);
    return hipGetLastError();
}

template <int KT, int BS>
int occupancy_t(int fp32)
{
    int nb = 0;
    hipError_t e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &nb, reinterpret_cast<const void *>(&k_step_f32<KT, BS>), BS, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &nb, reinterpret_cast<const void *>(&k_step_f64<KT, BS>), BS, 0);
    return e == hipSuccess ? nb : -1;
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_seed(const DevParams &dp, const DevBatch &bt, hipStream_t s)
{
    if (bt.n_total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seed, dim3((bt.n_total + 255) / 256), dim3(256), 0, s, dp, bt);
    return hipGetLastError();
}

hipError_t launch_compact(const DevParams &dp, const DevBatch &bt, int count_step, hipStream_t s)
{
    if (bt.n_events <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact, dim3(bt.n_events), dim3(kCompactThreads), 0, s, dp, bt,
                       count_step);
    return hipGetLastError();
}

hipError_t launch_plan(const DevBatch &bt, const LaunchCfg &cfg, hipStream_t s)
{
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, s, bt, cfg.bs * cfg.kt, cfg.chunk);
    return hipGetLastError();
}

#define CT_LAUNCH_CASES(X) \
    X(1, 64) X(2, 64) X(4, 64) X(1, 128) X(2, 128) X(4, 128) X(1, 256) X(2, 256) X(4, 256)

// Persistent step launch over the work list built by launch_plan; field_out
// receives the field ([N][3], carrier order) when field_only is set.
hipError_t launch_step(const DevParams &dp, const DevBatch &bt, const LaunchCfg &cfg, int fp32,
                       int grid, int field_only, double *field_out, hipStream_t s)
{
    if (bt.n_events <= 0 || grid <= 0) return hipSuccess;
#define CT_STEP_CASE(KT_, BS_) \
    if (cfg.kt == KT_ && cfg.bs == BS_) \
        return launch_step_t<KT_, BS_>(dp, bt, cfg, fp32, grid, field_only, field_out, s);
    CT_LAUNCH_CASES(CT_STEP_CASE)
#undef CT_STEP_CASE
    return hipErrorInvalidValue;
}

// Resident workgroups per compute unit of the step kernel for a configuration.
int step_occupancy(const LaunchCfg &cfg, int fp32)
{
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

hipError_t launch_update(const DevParams &dp, const DevBatch &bt, const LaunchCfg &cfg, int n_max,
                         int field_only, double *field_out, hipStream_t s)
{
    if (bt.n_events <= 0 || n_max <= 0 || cfg.chunk <= 0 || n_max <= cfg.chunk) return hipSuccess;
    const dim3 grid((n_max + 255) / 256, bt.n_events);
    hipLaunchKernelGGL(k_update, grid, dim3(256), 0, s, dp, bt, cfg.chunk, field_only, field_out);
    return hipGetLastError();
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
