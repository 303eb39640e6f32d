// Device code shared by the kernels of the library (ct_kernels.hip: the
// brute-force method; ct_sph.hip: the simplified spherical model): the
// counter-based RNG, the memory-order helpers, the physics of one carrier
// update (Eqs. 3, 5, 6 of arXiv:2506.09712 and Algorithm 1) and the per-event
// compaction.  Each translation unit that includes it gets its own copy.
#pragma once

#include <math.h>

#include "ct_internal.hpp"

namespace ct {

namespace {

constexpr uint32_t kDomainDiffusion = 0u;           // holes
constexpr uint32_t kDomainDiffusionElectron = 4u;
constexpr uint32_t kDomainCloud = 1u;

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
        // low and high halves as two independent products (a single 64-bit
        // product measured slower: it lengthens the dependent chain)
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
__device__ inline void normals3(uint32_t key0, uint32_t key1, Ctr ctr, double n[3])
{
    const Ctr w = philox10(ctr, key0, key1);
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

__device__ __forceinline__ void normals3(const DevParams &dp, Ctr ctr, double n[3])
{
    normals3(dp.key0, dp.key1, ctr, n);
}

// ------------------------------------------------------------ memory order

// Publication between workgroups of one run.  Data that other workgroups
// read later in the same run is stored with agent-scope relaxed atomic
// stores, which go to device-coherent memory instead of staying dirty in the
// L2 of this XCD.  Every thread then waits for its own stores to complete
// (vmcnt 0, no cache maintenance), the workgroup meets at a barrier, and
// thread 0 alone publishes with a release operation on a completion counter
// or flag: one L2 write-back per workgroup, with almost nothing left to write
// back.  (A release fence in every thread costs one write-back per wave,
// several times more under load.)  The observing thread reads the flag,
// executes an acquire fence (invalidating stale cache lines), and a
// workgroup barrier orders the rest of its workgroup's loads after it.
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// s_waitcnt vmcnt(0): this thread's vector memory operations have completed.
__device__ __forceinline__ void wait_own_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// The same kernel argument, read through an index the compiler cannot see is
// 0.  Called at the top of a persistent loop's body, it makes the compiler
// load the argument's fields (scalar loads from the argument segment) where
// the body uses them, instead of keeping all of them in scalar registers from
// kernel entry on: the run kernels take more uniform values than fit, and the
// compiler would spill the rest into vector lanes and read each back with one
// VALU instruction.
template <class T>
__device__ __forceinline__ const T &reload_arg(const T &arg)
{
    int zero = 0;
    asm volatile("" : "+s"(zero));
    return (&arg)[zero];
}

__device__ __forceinline__ void st_dev(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_dev(float *p, float v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_dev(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_dev(int64_t *p, int64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_relaxed(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t add_relaxed(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decrement of a completion counter by `by` (thread 0, after a workgroup
// barrier): releases the workgroup's results; the caller that takes the
// counter to zero also acquires everyone else's.
__device__ __forceinline__ bool dec_is_last(int32_t *p, int32_t by = 1)
{
    const int32_t left = __hip_atomic_fetch_add(p, -by, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (left != by) return false;
    fence_acquire();
    return true;
}

// ------------------------------------------------------------------ physics

// mu0 / (1 + (E/Ec)^beta)^(1/beta) through base-2 logarithms, with no
// division: (E/Ec)^beta = 2^(beta log2(E/Ec)) and the mobility is
// mu0 2^(-log2(1 + that) / beta).  E = 0 gives 2^-inf = 0, so mu = mu0.
__device__ __forceinline__ double mobility(const DevParams &dp, bool electron, double e_mag)
{
    const double mu0 = electron ? dp.mu0_e : dp.mu0;
    if (dp.mobility == 1) return mu0;
    const double inv_ec = electron ? dp.inv_ec_e : dp.inv_ec;
    const double beta = electron ? dp.beta_e : dp.beta;
    const double inv_beta = electron ? dp.inv_beta_e : dp.inv_beta;
    const double t = exp2(beta * log2(e_mag * inv_ec));
    return mu0 * exp2(-inv_beta * log2(1.0 + t));
}

// Boundaries after a move: holes are mirrored at the entrance side and
// collected at the pixel plane; electrons are mirrored at the pixel plane and
// collected at the entrance side.  Returns true when collected.
__device__ __forceinline__ bool boundary(const DevParams &dp, bool electron, double &z)
{
    if (!electron) {
        if (z > dp.H) z = 2.0 * dp.H - z;
        return z <= 0.0;
    }
    if (z < 0.0) z = -z;
    return z >= dp.H;
}

__device__ __forceinline__ int pixel_bin(const DevParams &dp, double x, double y)
{
    const int G = dp.grid_n;
    const double fx = floor((x + dp.half_width) / dp.pitch);
    const double fy = floor((y + dp.half_width) / dp.pitch);
    if (fx >= 0.0 && fx < (double)G && fy >= 0.0 && fy < (double)G) return (int)fy * G + (int)fx;
    return G * G;
}

// A carrier reaches an electrode: endpoint and step by carrier; holes are
// counted in the pixel grid (with an overflow bin), electrons are not.
__device__ inline void collect(const DevParams &dp, const DevBatch &bt, int b, int carrier, bool electron,
                        double x, double y, double z, int64_t step)
{
    bt.out_xyz[3 * (int64_t)carrier + 0] = x;
    bt.out_xyz[3 * (int64_t)carrier + 1] = y;
    bt.out_xyz[3 * (int64_t)carrier + 2] = z;
    bt.out_cstep[carrier] = (int32_t)step;
    if (electron) return;
    const int g1 = dp.grid_n * dp.grid_n + 1;
    atomicAdd(&bt.pix[(int64_t)b * g1 + pixel_bin(dp, x, y)], 1);
}

// Update of one drifting carrier (Eqs. 3, 5, 6 and Algorithm 1): (ex, ey,
// ez_rep) is the field of the other carriers at the step-start snapshot,
// already scaled by K.  A hole moves along the total field, an electron
// against it, each with its own mobility at the total field's magnitude.
// HolesOnly: the batch has no electrons (the test is compiled out).  The
// carrier's position, index k within its event and RNG id are given.
template <bool HolesOnly = false>
__device__ void advance_at(const DevParams &dp, const DevBatch &bt, int b, int slot, double x,
                           double y, double z, int k, int rng_id, double ex, double ey,
                           double ez_rep, int64_t step, uint32_t eid)
{
    const int carrier = bt.off[b] + k;
    const bool electron = !HolesOnly && k >= bt.nh0[b];
    double ez = ez_rep;
    if (dp.flags & 2u) ez += -(dp.e0 - dp.e1 * z);
    const double e_mag = sqrt(ex * ex + ey * ey + ez * ez);
    const double mu = mobility(dp, electron, e_mag);
    const double sm = electron ? -mu : mu;  // signed mobility
    double g[3] = {0.0, 0.0, 0.0};
    double hop = 0.0;
    if (dp.flags & 4u) {
        hop = sqrt(2.0 * (mu * dp.kT) * dp.dt);
        normals3(dp, Ctr{(uint32_t)rng_id, (uint32_t)step, eid,
                         electron ? kDomainDiffusionElectron : kDomainDiffusion}, g);
    }
    const double x1 = x + sm * ex * dp.dt + hop * g[0];
    const double y1 = y + sm * ey * dp.dt + hop * g[1];
    double z1 = z + sm * ez * dp.dt + hop * g[2];
    const bool done = boundary(dp, electron, z1);
    st_dev(&bt.nx[slot], x1);
    st_dev(&bt.ny[slot], y1);
    st_dev(&bt.nz[slot], z1);
    st_dev(&bt.nidx[slot], k);
    if (done) collect(dp, bt, b, carrier, electron, x1, y1, z1, step + 1);
}

// The same, loading the carrier of slot `slot` itself.
template <bool HolesOnly = false>
__device__ void advance(const DevParams &dp, const DevBatch &bt, int b, int slot, double ex,
                        double ey, double ez_rep, int64_t step, uint32_t eid)
{
    const int k = bt.idx[slot];
    advance_at<HolesOnly>(dp, bt, b, slot, bt.cx[slot], bt.cy[slot], bt.cz[slot], k,
                          bt.rngid[bt.off[b] + k], ex, ey, ez_rep, step, eid);
}

// FP64 reciprocal cube of sqrt(r2): hardware estimate refined by one
// third-order Newton step, y <- y (1 + e/2 + 3 e^2/8), e = 1 - r2 y^2.
__device__ __forceinline__ double inv_r3_f64(double r2)
{
    double y = __builtin_amdgcn_rsq(r2);
    const double e = fma(-r2, y * y, 1.0);
    y = fma(y * e, fma(e, 0.375, 0.5), y);
    return y * y * y;
}


// ------------------------------------------------------------ compaction

// Carriers of event b still drifting after the step (holes: z > 0, the
// first nh of the n slots; electrons: z < H) are packed to the front of the
// event's slots in carrier order by the NT threads of one workgroup, from the
// post-step arrays (nx, ny, nz, nidx) into the current ones (cx, cy, cz,
// idx); surviving holes therefore stay ahead of surviving electrons.  Windows
// of kCompactChunks chunks of NT slots:
// every z of a window is loaded at once, each wave ranks its survivors with
// a 64-bit ballot and mbcnt per chunk, one barrier publishes the wave totals,
// and the survivors are copied with independent loads and stores, so about
// two memory latencies are exposed per window.  n is the event's count
// before the step.  Thread 0 stores the new counts (all, holes) and the
// centroid (summed in a fixed order; within a wave, neighbouring lanes
// first, so that partners at adjacent slots of a point-symmetric cloud cancel
// exactly) and, for a step, counts it.  Returns the
// survivors (in every thread) and, in thread 0, the surviving holes; ends
// with a barrier.
constexpr int kCompactChunks = 8;

template <int NT>
__device__ int compact_event(const DevBatch &bt, int b, int n, int nh, double H, int count_step,
                             int *wcount, double *wsum, int &holes_kept)
{
    constexpr int W = NT / 64;
    constexpr int K = kCompactChunks;
    const int base = bt.off[b];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    int kept = 0, my_holes = 0;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int w0 = 0; w0 < n; w0 += K * NT) {
        double z[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int i = w0 + j * NT + tid;
            z[j] = i < n ? bt.nz[base + i] : 0.0;
        }
        uint32_t alive = 0;  // bit j: this thread's slot of chunk j survives
        int rank[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int i = w0 + j * NT + tid;
            const bool a = i < nh ? z[j] > 0.0 : (i < n && z[j] < H);
            my_holes += (a && i < nh) ? 1 : 0;
            const uint64_t mask = __ballot(a);
            rank[j] = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            if (lane == 0) wcount[j * W + wave] = __popcll(mask);
            alive |= (a ? 1u : 0u) << j;
        }
        __syncthreads();
        int before = kept;  // survivors ahead of this thread's slot in the current chunk
#pragma unroll
        for (int j = 0; j < K; ++j) {
            int mine = 0, total = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int v = wcount[j * W + q];
                mine += q < wave ? v : 0;
                total += v;
            }
            if (alive & (1u << j)) {
                const int i = w0 + j * NT + tid;
                const int d = base + before + mine + rank[j];
                const double x = bt.nx[base + i], y = bt.ny[base + i];
                const int k = bt.nidx[base + i];
                st_dev(&bt.cx[d], x);
                st_dev(&bt.cy[d], y);
                st_dev(&bt.cz[d], z[j]);
                st_dev(&bt.idx[d], k);
                sx += x;
                sy += y;
                sz += z[j];
            }
            before += total;
        }
        kept = before;
        __syncthreads();  // wave totals of this window are read before the next overwrites them
    }
    for (int o = 1; o < 64; o <<= 1) {
        sx += __shfl_xor(sx, o);
        sy += __shfl_xor(sy, o);
        sz += __shfl_xor(sz, o);
        my_holes += __shfl_xor(my_holes, o);
    }
    if (lane == 0) {
        wsum[0 * W + wave] = sx;
        wsum[1 * W + wave] = sy;
        wsum[2 * W + wave] = sz;
        wcount[wave] = my_holes;
    }
    __syncthreads();
    if (tid == 0) {
        double X = 0.0, Y = 0.0, Z = 0.0;
        int holes = 0;
        for (int q = 0; q < W; ++q) {
            X += wsum[0 * W + q];
            Y += wsum[1 * W + q];
            Z += wsum[2 * W + q];
            holes += wcount[q];
        }
        holes_kept = holes;
        st_dev(&bt.n_hole[b], holes);
        if (kept > 0) {
            st_dev(&bt.ref[4 * b + 0], X / kept);
            st_dev(&bt.ref[4 * b + 1], Y / kept);
            st_dev(&bt.ref[4 * b + 2], Z / kept);
        }
        st_dev(&bt.n_act[b], kept);
        if (count_step && n > 0) {
            bt.pairs[b] += (uint64_t)n * (uint64_t)(n - 1);
            bt.hsteps[b] += (uint64_t)n;
            st_dev(&bt.ev_step[b], bt.ev_step[b] + 1);
            st_dev(&bt.ev_taken[b], bt.ev_taken[b] + 1);
            st_dev(&bt.call_steps[b], bt.call_steps[b] + 1);
        }
    }
    __syncthreads();
    return kept;
}

}  // namespace

}  // namespace ct
