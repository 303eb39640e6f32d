// Internal types shared by the host side (ct_capi.cpp) and the kernels
// (ct_kernels.hip) of the library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ct {

// Physics constants of one context, precomputed on the host (all FP64).
struct DevParams {
    double H;          // thickness (um)
    double e0, e1;     // drift field magnitude e0 - e1 z (V/um), Eq. 6 on this z axis
    double dt;         // time step (ns)
    double K;          // e / (4 pi eps0 eps_r) (V um)
    double kT;         // k T / e (V)
    double s2;         // softening^2 (um^2), never below a tiny floor
    double mu0, ec, beta, inv_beta, inv_ec;           // holes
    double mu0_e, ec_e, beta_e, inv_beta_e, inv_ec_e; // electrons
    double pitch, half_width;  // pixel pitch, grid_n * pitch / 2
    float s2f;
    int32_t grid_n;
    int32_t mobility;  // 0 Caughey-Thomas (Jacoboni-Canali), 1 constant
    uint32_t flags;    // repulsion 1, drift 2, diffusion 4, electrons 8, spherical model 16
    uint32_t key0, key1;
};

// Most source chunks an event is split into; larger events get longer chunks.
constexpr int kMaxChunks = 256;

// One work item: target tile `tile` of event `e` (bs * kt targets) against
// source chunk `chunk` of the same event, for the event's current step, in
// which the event has `n` drifting carriers, the first `nh` of them holes
// (the item's split into tiles and chunks follows from n alone).
struct QItem {
    int32_t e, tile, chunk, n, nh, pad[3];
};

// Control block of one run of the persistent step kernel.  Tickets index the
// work queue; a ticket's item is valid once its sequence word equals the
// run's generation.  Each counter that workgroups update or poll has a
// 256-byte line of its own: atomics on one shared line serialise device-wide.
struct alignas(256) Line {
    uint32_t v;
    uint32_t pad[63];
};

struct Sched {
    Line head;       // next ticket to claim
    Line tail;       // next ticket to reserve
    Line done;       // events finished for this run (drained, at the step cap, or parked)
    Line error;      // 1: the liveness guard expired; 2: the first step did not fit the queue
    Line exhausted;  // 1: some event was parked because the queue was full
    Line stall;      // when the guard expires: ticket waited for, head, tail, done
    int64_t active;      // drifting holes (summary kernel)
    int64_t max_steps;   // most steps any event took in this call (summary kernel)
};

// Completion counter of an event's step: one 64-byte line per event.
constexpr int kEventLine = 16;  // int32 words

// Device view of a batch.  Slots [off[b], off[b] + n_act[b]) of the position
// arrays hold the drifting carriers of event b, compacted in their seeded
// slot order: its n_hole[b] drifting holes first, then its drifting
// electrons (carrier indices below nh0[b] are holes), each species in
// carrier order, or deposit by deposit for an event of several deposits
// (deposit_major).  Slots [off[b], off[b + 1]) belong to event b for the
// whole run.
struct DevBatch {
    int32_t n_events;
    int32_t n_total;
    uint64_t first_event_id;
    const int32_t *off;     // [B + 1] first slot of each event
    int32_t *n_act;         // [B] drifting carriers
    int32_t *n_hole;        // [B] drifting holes (the first n_hole of the n_act slots)
    const int32_t *nh0;     // [B] holes of the event (carrier indices below are holes)
    int64_t *ev_step;       // [B] absolute step of the event
    int64_t *ev_taken;      // [B] steps taken since seeding
    int64_t *call_steps;    // [B] steps taken in the current ct_step call
    double *ref;            // [B][4] centroid of the drifting carriers (the spherical
                            //        model's centre; wave priorities)
    double *cx, *cy, *cz;   // [N] current positions (compacted)
    double *nx, *ny, *nz;   // [N] positions after the step (same slots)
    int32_t *idx;           // [N] carrier index within its event, per slot (compacted)
    int32_t *nidx;          // [N] the same after the step (same slots as nx)
    const int32_t *rngid;   // [N] RNG carrier id by carrier (event offset + index)
    double *out_xyz;        // [N][3] by carrier
    int32_t *out_cstep;     // [N] by carrier
    int32_t *pix;           // [B][grid_n^2 + 1]
    uint64_t *pairs;        // [B] sum over steps of N_a (N_a - 1)
    uint64_t *hsteps;       // [B] sum over steps of N_a
    // seeding inputs
    const double *sigma;    // [B]
    const int32_t *dep_off; // [B + 1]
    const double *deposits; // [n_dep][3]
    const int32_t *x_off;   // [B + 1] offsets into explicit positions
    const double *xyz_in;   // [n_explicit][3]
    const int64_t *start;   // [B]
};

// Work queue and per-event scheduling state of the persistent step kernel,
// sized for a batch and a launch configuration.
struct DevQueue {
    Sched *sc;
    QItem *q;               // [cap]
    uint32_t *seq;          // [cap]
    uint32_t cap;
    uint32_t gen;           // generation of the current run (never 0)
    int32_t *tiles_left;    // [B * kEventLine] target tiles of the event's step not yet updated
    int32_t *chunks_left;   // [sum of tiles] source chunks of a target tile not yet summed
    const int32_t *tile_base;  // [B + 1] prefix of the most target tiles of each event
    double *part;           // partial fields of split events
    const int64_t *part_off;   // [B + 1] prefix of 3 * n0 * most chunks of each event
    // spherical model: tickets (event, workgroup of the event) and the shared
    // state of events taken by several workgroups
    const int32_t *tk_off;     // [B + 1] first ticket of each event
    const int64_t *grp_off;    // [B + 1] byte offset of each event's group state in grp
    char *grp;
    int32_t n_tickets;
    const int32_t *single;     // the events run by one workgroup, in batch order
};

struct LaunchCfg {
    int kt;        // targets per thread
    int bs;        // block size = sources per LDS tile
    int chunk;     // source chunk length (a multiple of bs; events longer than this are split)
    int newton;    // FP32 pair kernel that takes each unordered pair once (kt 1, bs 256):
                   // 1 holes only, 2 holes and electrons; 0 every ordered pair
};

// Parameters of the event generator (Sec. 4.2), precomputed on the host.
struct GenDev {
    double H;                    // thickness (um)
    double e_entrance, e_pixels; // drift field magnitude at the entrance side and the pixels (V/um)
    double k;                    // its slope along the drift (V/um^2), Eq. 6
    double inv_mu0, inv_ec;      // hole Jacoboni-Canali parameters (Eq. 9)
    double atten, keep;          // absorption length (um), 1 - exp(-H / atten)
    double mean_n, sd_n;         // E / w and sqrt(F E / w)
    double w_kev, noise, pitch;  // pair energy (keV), pixel noise sigma (keV), pixel pitch (um)
    double pa[4], pb[5];         // Eqs. 10 and 11
    int32_t grid_n;
    uint32_t key0, key1;
    uint64_t first_event_id;
};

// Kernel launchers (ct_kernels.hip).  All return the launch status.
hipError_t launch_seed(const DevParams &dp, const DevBatch &bt, hipStream_t s);
hipError_t launch_compact(const DevParams &dp, const DevBatch &bt, hipStream_t s);
hipError_t launch_init(const DevBatch &bt, const DevQueue &dq, const LaunchCfg &cfg,
                       int64_t max_steps, int field_only, int repulsion, hipStream_t s);
hipError_t launch_run(const DevParams &dp, const DevBatch &bt, const DevQueue &dq,
                      const LaunchCfg &cfg, int fp32, int grid, int64_t max_steps, int field_only,
                      double *field_out, hipStream_t s);
hipError_t launch_summary(const DevBatch &bt, Sched *sc, hipStream_t s);
// Simplified spherical model (Eq. 7): one workgroup per event of the list
// dq.single (grid_single of them), then grid_shared resident workgroups
// claiming the tickets of the shared events (one per workgroup of an event);
// scratch holds 2 * n_total doubles.  sph_occupancy: resident workgroups per
// CU of the shared-event kernel.
hipError_t launch_sph(const DevParams &dp, const DevBatch &bt, const DevQueue &dq, double *scratch,
                      int grid_single, int grid_shared, int64_t max_steps, int field_only,
                      double *field_out, hipStream_t s);
int sph_occupancy();
// Wall-clock ticks of the liveness guard of the persistent kernels.
uint64_t run_idle_ticks();
// Event generator (ct_gen.hip): n_events events, one wave each; outputs
// (device, nullable) energy [n][G^2], counts [n][G^2 + 1], info [n][5].
hipError_t launch_gen(const GenDev &g, int64_t n_events, double *energy, int32_t *counts,
                      double *info, hipStream_t s);
int run_occupancy(const LaunchCfg &cfg, int fp32);
// The device address and size of the library's static scratch array on a
// device (for contexts seeded with ct_seed_events_noalloc); the device must
// be current.  Looked up once per device.
hipError_t scratch_memory(int device, void **ptr, size_t *bytes);
bool launch_supported(int kt, int bs);
hipError_t launch_scatter_alive(const DevBatch &bt, int n_max, hipStream_t s);
hipError_t launch_philox(const DevParams &dp, const uint32_t *ctr, int64_t n, uint32_t *words,
                         double *normals, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);

// Newton-pair split of the FP32 field (Eq. 4 is antisymmetric: the term of
// pair (i, j) is minus that of (j, i), so one evaluation serves both holes).
// An event of n holes has T tiles of kSymTile.  Tile a meets the tiles
// a + o (mod T) for the offsets o in [0, P_a): offset 0 is the tile with
// itself (every ordered pair evaluated), the others are Newton pairs whose
// reaction goes to the partner tile.  With P_a = (T - 1) / 2 + 1, plus one
// for a < T / 2 when T is even, every unordered pair of tiles is met exactly
// once.  An item takes C consecutive offsets of one tile (R items per tile).
// Events of more than kSymMaxTiles tiles (whose reaction partials would need
// too much memory) evaluate every ordered pair: item r of a tile takes the
// tiles [r C, r C + C) as sources, C lengthened so that R <= kMaxChunks.
// Partial fields: slot r holds the target side of item r of each tile, slot
// R + o - 1 the reaction a tile receives through offset o.  Everything
// depends on n and C alone.
constexpr int kSymTile = 256;
constexpr int kSymMaxTiles = 512;
constexpr int kSymMaxC = 15;  // longest chunk, in tiles

struct SymSplit {
    int T;        // tiles
    int C;        // offsets (partner tiles) per item
    int R;        // items per tile
    int P;        // largest partner count (Newton pairs), or T
    int newton;   // 1: Newton pairs
};

__host__ __device__ inline SymSplit sym_split(int n, int chunk_tiles)
{
    SymSplit s;
    s.T = (n + kSymTile - 1) / kSymTile;
    s.newton = s.T <= kSymMaxTiles;
    if (s.newton) {
        s.P = s.T / 2 + 1;
        s.C = chunk_tiles;
    } else {
        s.P = s.T;
        const int c_min = (s.T + kMaxChunks - 1) / kMaxChunks;
        s.C = chunk_tiles > c_min ? chunk_tiles : c_min;
    }
    s.R = s.T > 0 ? (s.P + s.C - 1) / s.C : 0;
    return s;
}

// Partner offsets of tile a: [0, sym_partners(T, a)).
__host__ __device__ inline int sym_partners(int T, int a)
{
    return (T - 1) / 2 + 1 + ((T % 2 == 0 && a < T / 2) ? 1 : 0);
}

// Reactions tile b receives: through the offsets [1, sym_received(T, b)].
__host__ __device__ inline int sym_received(int T, int b)
{
    return T % 2 == 1 ? (T - 1) / 2 : T / 2 - 1 + (b >= T / 2 ? 1 : 0);
}

// Contributions a tile waits for, and whether partial fields are used at all.
__host__ __device__ inline int sym_expected(const SymSplit &s, int b)
{
    return s.R + (s.newton ? sym_received(s.T, b) : 0);
}
__host__ __device__ inline bool sym_partials(const SymSplit &s)
{
    return s.newton ? s.T > 1 : s.R > 1;
}
__host__ __device__ inline int sym_slots(const SymSplit &s)
{
    return sym_partials(s) ? (s.newton ? s.R + s.P - 1 : s.R) : 0;
}

// Source chunk length and count of an event of n drifting holes: chunks of
// `chunk` sources (a multiple of bs), lengthened to whole tiles so that no
// event has more than kMaxChunks of them.  Depends on n and the launch only,
// so the grouping of the field sum is a function of the event alone.
__host__ __device__ inline void event_chunks(int n, int bs, int chunk, int &len, int &count)
{
    const int min_len = ((n + kMaxChunks - 1) / kMaxChunks + bs - 1) / bs * bs;
    len = chunk > min_len ? chunk : min_len;
    if (len < bs) len = bs;
    count = n > 0 ? (n + len - 1) / len : 0;
}

// Carrier of slot s among the n carriers of one species spread over nd
// deposits (carrier k sits on deposit k mod nd): slots run deposit by
// deposit, each deposit's carriers in increasing order, so that every tile
// of consecutive slots is spatially compact (FP32 coordinates are formed
// relative to a tile's first carrier).  A bijection of [0, n).
__host__ __device__ inline int deposit_major(int s, int n, int nd)
{
    if (nd <= 1) return s;
    const int q = n / nd, r = n % nd;  // deposits below r hold q + 1 carriers
    int d, m;
    if (s < r * (q + 1)) {
        d = s / (q + 1);
        m = s - d * (q + 1);
    } else {
        const int t = s - r * (q + 1);
        d = r + t / q;
        m = t - (d - r) * q;
    }
    return d + m * nd;
}

}  // namespace ct
