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
    double mu0, ec, beta, inv_beta;
    double pitch, half_width;  // pixel pitch, grid_n * pitch / 2
    float s2f;
    int32_t grid_n;
    int32_t mobility;  // 0 Caughey-Thomas (Jacoboni-Canali), 1 constant
    uint32_t flags;    // repulsion 1, drift 2, diffusion 4
    uint32_t key0, key1;
};

// Device view of one batch.  Slots [off[b], off[b] + n_act[b]) of the
// position arrays hold the drifting holes of event b, compacted and in
// carrier order.
// One work item of the step kernel: the target tile `tile` of event b
// against its source chunk c of nsplit.
struct Item {
    int32_t b, tile, c, nsplit;
};

struct DevBatch {
    int32_t n_events;
    int32_t n_total;
    uint64_t first_event_id;
    const int32_t *off;     // [B + 1] first slot of each event
    int32_t *n_act;         // [B] drifting holes
    int64_t *ev_step;       // [B] absolute step of the event
    int64_t *ev_taken;      // [B] steps taken since seeding
    double *ref;            // [B][4] reference point (centroid) for FP32 coordinates
    double *cx, *cy, *cz;   // [N] current positions (compacted)
    double *nx, *ny, *nz;   // [N] positions after the step (same slots)
    int32_t *idx;           // [N] carrier index within its event, per slot (compacted)
    const int32_t *rngid;   // [N] RNG carrier id by carrier (event offset + index)
    double *out_xyz;        // [N][3] by carrier
    int32_t *out_cstep;     // [N] by carrier
    int32_t *pix;           // [B][grid_n^2 + 1]
    uint64_t *pairs;        // [B] sum over steps of N_a (N_a - 1)
    uint64_t *hsteps;       // [B] sum over steps of N_a
    int64_t *active;        // [1] drifting holes after the last compaction
    double *part;           // [nsplit][3][N] partial fields of split events
    int32_t part_chunks;    // chunks the partial buffer holds
    Item *work;             // [work_cap] work list of the current step
    int32_t work_cap;
    int32_t *item_base;     // [B] first item of each event
    int32_t *n_items;       // [1]
    uint32_t *counter;      // [1] next item to take
    // seeding inputs
    const double *sigma;    // [B]
    const int32_t *dep_off; // [B + 1]
    const double *deposits; // [n_dep][3]
    const int32_t *x_off;   // [B + 1] offsets into explicit positions (-1 rows: none)
    const double *xyz_in;   // [n_explicit][3]
    const int64_t *start;   // [B]
};

struct LaunchCfg {
    int kt;        // targets per thread
    int bs;        // block size
    int chunk;     // longest source chunk of one work item; an event with n holes is
                   // split into ceil(n / chunk) chunks of equal length (0: no split)
};

// Kernel launchers (ct_kernels.hip).  All return the launch status.
hipError_t launch_seed(const DevParams &dp, const DevBatch &bt, hipStream_t s);
hipError_t launch_compact(const DevParams &dp, const DevBatch &bt, int count_step, hipStream_t s);
hipError_t launch_plan(const DevBatch &bt, const LaunchCfg &cfg, hipStream_t s);
hipError_t launch_step(const DevParams &dp, const DevBatch &bt, const LaunchCfg &cfg, int fp32,
                       int grid, int field_only, double *field_out, hipStream_t s);
int step_occupancy(const LaunchCfg &cfg, int fp32);
bool launch_supported(int kt, int bs);
hipError_t launch_update(const DevParams &dp, const DevBatch &bt, const LaunchCfg &cfg, int n_max,
                         int field_only, double *field_out, hipStream_t s);
hipError_t launch_scatter_alive(const DevBatch &bt, int n_max, hipStream_t s);
hipError_t launch_philox(const DevParams &dp, const uint32_t *ctr, int64_t n, uint32_t *words,
                         double *normals, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);

}  // namespace ct
