/*
 * ct.h - C ABI of the MI355X (gfx950) brute-force charge-transport Monte Carlo.
 *
 * The library simulates the holes of many independent X-ray / electron events
 * in a planar p-on-n silicon sensor with the comprehensive time-stepping method
 * of Xie et al., arXiv:2506.09712, Sec. 2.1 (Eqs. 2-6) and Appendix A
 * (Algorithm 1).  Each step evaluates, for every alive hole i of an event,
 *
 *     E_rep,i = K * sum_{j != i, j alive in the same event}
 *               (r_i - r_j) / (|r_i - r_j|^2 + s^2)^(3/2),   K = e/(4 pi eps0 eps_r)
 *
 * (Eq. 4 for holes, with an optional Plummer softening s), adds the linear
 * drift field of Eq. 6, evaluates the Caughey-Thomas / Jacoboni-Canali
 * mobility at |E_drift + E_rep|, and moves the hole by mu E dt plus a
 * Gaussian diffusion step of variance 2 D dt per axis, D = mu k T / e
 * (Eqs. 3 and 5).  Holes whose update leaves them at z <= 0 are collected
 * on the pixel plane and counted in a grid_n x grid_n pixel array.
 *
 * With CT_ELECTRONS the electrons are simulated too (Sec. 2.1: both species
 * as individual carriers, including electron-hole attraction).  Each source
 * enters the sum with its sign (+1 hole, -1 electron); a hole moves along
 * the total field, an electron against it with the Jacoboni-Canali electron
 * mobility.  Electrons are collected at the entrance side (z >= H), mirrored
 * at the pixel plane, and not counted in pixels.  An event ends when its
 * last hole is collected; its electrons then keep their current position.
 *
 * Units: micrometre, nanosecond, volt, kelvin.  z is the distance from the
 * pixel (collecting) plane; the paper's z (from the entrance side) is H - z.
 *
 * Conventions shared by every call:
 *  - Every call returns ct_status; no exception or abort crosses the ABI.
 *    ct_last_error() returns a thread-local message for the last failure.
 *  - Host arrays passed in are owned by the caller and only read during the
 *    call.  Device memory belongs to the context, or to the caller when it
 *    binds a workspace (ct_bind_workspace); a bound workspace must outlive
 *    the context.
 *  - A context is used by one host thread at a time.  Separate contexts are
 *    independent.  Work is issued on the context's HIP stream; every call
 *    that returns results synchronises that stream before returning.
 *  - CT_EINVAL / CT_ESTATE leave the context unchanged.  CT_EDEVICE means a
 *    HIP call failed; the context must then only be destroyed.
 *    CT_EMAXSTEPS keeps the state so it can be collected or continued.
 */
#ifndef CT_H
#define CT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CT_ABI_VERSION 3u

typedef struct ct_ctx ct_ctx; /* opaque, owned by the library */

typedef enum {
    CT_OK = 0,
    CT_EINVAL = -1,     /* bad argument or parameter */
    CT_ESTATE = -2,     /* call out of order (e.g. ct_step before ct_seed_events) */
    CT_ENOMEM = -3,     /* device allocation failed or bound workspace too small */
    CT_EDEVICE = -4,    /* no gfx950 device, or a HIP runtime call failed */
    CT_EMAXSTEPS = -5,  /* step cap reached with holes still drifting */
    CT_ENONFINITE = -6  /* an explicit position is NaN or infinite */
} ct_status;

/* Arithmetic of the pairwise field.  Positions and the time integration are
 * FP64 in both modes.  CT_FP32: the pair terms are summed in FP32 on
 * coordinates relative to the FP64 position of the first carrier of the
 * target's tile (256 consecutive slots; multi-deposit events occupy their
 * slots deposit by deposit, so a tile is spatially compact) over each LDS
 * tile of sources, and the tile sums are added in FP64; CT_FP64: everything
 * in FP64 on absolute coordinates.  An event's sources are split into chunks whose
 * length depends only on the event's own hole count and the launch
 * configuration (ct_set_launch), and the chunk sums are added in chunk
 * order, so an event's result does not depend on the rest of the batch. */
typedef enum { CT_FP64 = 0, CT_FP32 = 1 } ct_precision;

/* Mobility model.  CT_MOB_JACOBONI: mu = mu0 / (1 + (E/Ec)^beta)^(1/beta),
 * with the Jacoboni-Canali laws at T unless overridden, mu0 = vm/Ec:
 *   holes:     vm = 1.62e8 T^-0.52 cm/s, Ec = 1.24 T^1.68 V/cm, beta = 0.46 T^0.17;
 *   electrons: vm = 1.53e9 T^-0.87 cm/s, Ec = 1.01 T^1.55 V/cm, beta = 2.57e-2 T^0.66.
 * CT_MOB_CONSTANT: mu = mu0 of the species. */
typedef enum { CT_MOB_JACOBONI = 0, CT_MOB_CONSTANT = 1 } ct_mobility;

/* physics_flags bits: repulsion, drift and diffusion are the paper's method;
 * CT_ELECTRONS adds the electrons of every pair (two species).
 * CT_SPHERICAL replaces the pairwise repulsion field (Eq. 4) by the
 * simplified spherical model of Sec. 2.2, Eq. 7: the field at hole i is
 *     K Q_i (r_i - c) / (|r_i - c|^2 + s^2)^(3/2),
 * c being the mean position of the event's drifting holes at the step start
 * and Q_i the number of them strictly closer to c than i (Q_i = 0: no
 * field).  Holes only (with CT_ELECTRONS: CT_EINVAL).  It is evaluated in
 * FP64 whatever the precision, and the launch configuration (ct_set_launch)
 * has no effect.  One workgroup runs all of an event's steps of a ct_step
 * call; an event of more than 8192 holes at seeding is shared by
 * ceil(n / 5120) workgroups (at most 32), a number fixed by the event alone,
 * so results do not depend on the batch.  The enclosed counts come from a
 * counting sort over 8192 bins per event and step; a bin holding many holes
 * at nearly the same distance costs time quadratic in its size.  A shared
 * event whose workgroups fail to meet for 10 s ends the call with
 * CT_EDEVICE. */
enum { CT_REPULSION = 1u, CT_DRIFT = 2u, CT_DIFFUSION = 4u, CT_ELECTRONS = 8u, CT_SPHERICAL = 16u };

/* options bits */
enum {
    CT_OPT_TIMING = 1u,   /* time every run of the step kernel with HIP events (ct_run_stats) */
    CT_OPT_AUTOTUNE = 4u, /* on seeding, time candidate launch configurations on the first
                             steps of the seeded batch (environment variable CT_TUNE_STEPS, by
                             default as many as make about 6e11 pair evaluations, 2 to 1000; each
                             from the freshly seeded state, the persistent kernel alone) and
                             keep the fastest if it beats the current launch by 1% or more
                             (3% when those steps do not finish the batch); candidates keep
                             Newton pairs
                             where the context uses them.  The choice is cached per device
                             architecture, compute units, precision, physics switches,
                             CT_OPT_ONE_SIDED and batch shape (events, largest event, total
                             carriers, in powers of two), in memory and in the file
                             CT_TUNE_CACHE (default $XDG_CACHE_HOME or ~/.cache
                             /ct_launch_cache.txt), so later processes reuse it.  The batch is
                             left as seeded.  The chosen configuration sets the grouping of the
                             field sum (see ct_set_launch) */
    CT_OPT_ONE_SIDED = 8u /* CT_FP32: evaluate every ordered pair (i, j) on its own.  By default
                             an FP32 run with one target per thread and blocks of 256
                             evaluates each unordered pair once and applies it to both carriers
                             (Eq. 4 is antisymmetric), in events of up to 131072 drifting carriers;
                             the two differ only in FP32 rounding */
};

typedef struct {
    uint32_t abi_version;      /* CT_ABI_VERSION */
    double thickness_um;       /* H > 0 (Algorithm 1 input) */
    double v_bias;             /* V_bias (Algorithm 1 input) */
    double v_dep;              /* V_depletion, 0 <= v_dep < v_bias when CT_DRIFT is set (Eq. 6) */
    double temperature_k;      /* T > 0 (Algorithm 1 input) */
    double pitch_um;           /* pixel pitch > 0 */
    int32_t grid_n;            /* pixels per side, 1..64; grid centred on (0, 0) */
    double dt_ns;              /* time step > 0 */
    double softening_um;       /* s >= 0 (0 = Eq. 4 exactly) */
    double eps_r;              /* relative permittivity > 0 (11.7 for silicon) */
    double pair_energy_ev;     /* energy per electron-hole pair > 0 (3.62 eV in the paper) */
    int32_t mobility;          /* ct_mobility */
    double mu0_override;       /* holes: um^2/(V ns); NaN = model value */
    double ec_override;        /* holes: V/um; NaN = model value */
    double beta_override;      /* holes: NaN = model value */
    uint32_t physics_flags;    /* CT_REPULSION | CT_DRIFT | CT_DIFFUSION
                                  [| CT_ELECTRONS or CT_SPHERICAL] */
    int32_t precision;         /* ct_precision */
    uint64_t seed;             /* Philox4x32-10 key = (low 32 bits, high 32 bits) */
    int64_t max_steps;         /* default step cap for ct_step (> 0) */
    void *hip_stream;          /* hipStream_t to issue work on (e.g. torch's); NULL = own stream */
    int32_t device;            /* HIP device ordinal; -1 = the current device */
    uint32_t options;          /* CT_OPT_* bits */
    double mu0_e_override;     /* electrons (CT_ELECTRONS): um^2/(V ns); NaN = model value */
    double ec_e_override;      /* electrons: V/um; NaN = model value */
    double beta_e_override;    /* electrons: NaN = model value */
} ct_sensor_params;

/* One event.  Its carriers are its holes, then (with CT_ELECTRONS) its
 * electrons.  Hole k is placed at deposit (k mod n_deposits) plus sigma
 * times three standard normals drawn from Philox counter (id_k, 0, event id,
 * 1); electron k of a cloud event starts at hole k's position.  With
 * n_deposits == 0 the carriers are placed at xyz (holes, then electrons).
 * Holes above the entrance side (z > H) are mirrored to 2H - z and holes at
 * z <= 0 are collected at step start_step; electrons below the pixel plane
 * are mirrored to -z and electrons at z >= H are collected at start_step.
 * Diffusion draws use counter (id, step, event id, 0) for holes and
 * (id, step, event id, 4) for electrons.
 *
 * Tracks (seg_len_um > 0; the paper has no track model, this extends the
 * deposit-based seeding of Algorithm 1 to an extended track): deposits holds
 * one point, the track's start, and the library places the event's
 * n_deposits deposits itself, on the device, at the midpoints of a walk of
 * n_deposits straight segments of length seg_len_um from that start.
 * Segment 0 points along -z; segment k >= 1 along the isotropic unit vector
 * of the Philox block at counter (k, 0, event id, 3), with
 * cos(theta) = 1 - 2 u0 and phi = 2 pi u1 (u = (w + 0.5) 2^-32).  Walk points
 * and midpoints are folded back into [0, H] (mirrored at either face).  The
 * carriers then sit on the deposits as for any multi-deposit event. */
typedef struct {
    double energy_kev;         /* used when n_carriers <= 0 or sigma_um < 0 */
    int32_t n_carriers;        /* > 0, or <= 0 for round(1000 E / pair_energy_ev) (Algorithm 1) */
    int32_t n_deposits;        /* >= 1: Gaussian cloud(s); 0: explicit positions */
    double sigma_um;           /* per-axis width >= 0, or < 0 for 0.0044 E^1.75 (Eq. 2) */
    const double *deposits;    /* host [n_deposits][3], x y z in um */
    const double *xyz;         /* host [n_carriers][3] when n_deposits == 0 */
    const int32_t *ids;        /* host [carriers] RNG carrier ids (holes, then electrons), or
                                  NULL for 0..n-1 within each species */
    int64_t start_step;        /* absolute step of the given state (0 for a new event) */
    int32_t n_electrons;       /* with CT_ELECTRONS: < 0 one per hole (cloud events; explicit
                                  events then list n_carriers electrons), >= 0 that many; without
                                  CT_ELECTRONS it must be <= 0 */
    double seg_len_um;         /* > 0: a track of n_deposits (>= 1) segments of this length
                                  whose start is deposits[0..2]; 0: deposits as given.
                                  Negative or not finite: CT_EINVAL */
} ct_event_desc;

typedef struct {
    int64_t steps;             /* sum over ct_step calls of the most steps any event took */
    uint64_t pairs;            /* sum over steps and events of N_a (N_a - 1) */
    int64_t n_total;           /* carriers in the batch (both species) */
    int64_t n_active;          /* holes still drifting */
    int64_t field_launches;    /* runs of the step kernel timed (CT_OPT_TIMING); one per
                                  ct_step call unless its work queue filled up */
    double field_kernel_ms;    /* their summed duration, HIP events on the context's stream */
    double step_wall_ms;       /* host wall time spent inside ct_step */
    int32_t targets_per_thread;/* launch configuration in use */
    int32_t block_size;
    int32_t chunk_len;         /* source chunk length (ct_set_launch) */
    int32_t workgroups;        /* workgroups of the step kernel (spherical model: one per
                                  single-workgroup event plus those taking shared events) */
    uint64_t hole_steps;       /* sum over steps and events of N_a (carrier updates performed,
                                  both species) */
    int32_t newton_pairs;      /* 1: the FP32 field evaluates each unordered pair once and applies
                                  it to both holes (CT_OPT_ONE_SIDED not set; see there) */
    int32_t reserved;
} ct_run_stats;

/* Create a context for one sensor configuration on one gfx950 device.
 * Validates every parameter (CT_EINVAL), requires a gfx950 device
 * (CT_EDEVICE otherwise, also on a host without a GPU). */
ct_status ct_init_sensor(const ct_sensor_params *p, ct_ctx **out);

/* Carrier count of each event as the library derives it: its holes
 * (Algorithm 1: round(1000 E / w) when n_carriers <= 0) plus, with
 * CT_ELECTRONS, its electrons.  Host only. */
ct_status ct_event_carriers(const ct_sensor_params *p, const ct_event_desc *ev, int32_t n_events,
                            int32_t *n_out);

/* Device bytes ct_seed_events needs for this batch (one buffer). */
size_t ct_workspace_bytes(const ct_sensor_params *p, const ct_event_desc *ev, int32_t n_events);

/* Use caller-owned device memory (e.g. a torch allocation) for the next
 * batches instead of library allocations.  NULL unbinds. */
ct_status ct_bind_workspace(ct_ctx *c, void *device_ptr, size_t bytes);

/* Replace the context's batch by n_events new events (ids first_event_id + b)
 * and seed their initial clouds on the device (Algorithm 1, initialisation).
 * Explicit positions that are not finite give CT_ENONFINITE. */
ct_status ct_seed_events(ct_ctx *c, const ct_event_desc *ev, int32_t n_events,
                         uint64_t first_event_id);

/* ct_seed_events for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same seeding and the same results, with no hipMalloc or hipFree.
 *   - The batch lives in the workspace the caller bound with
 *     ct_bind_workspace (at least ct_workspace_bytes for the batch); a context
 *     that ever let the library allocate a batch workspace is refused
 *     (CT_ESTATE), as are contexts without a bound workspace (CT_ESTATE) and
 *     CT_OPT_AUTOTUNE (CT_EINVAL: the tuner allocates).
 *   - The batch's work queue, partial fields and counters go to one static
 *     array of 128 MiB per GPU that the library holds until the process
 *     ends.  A batch whose queue does not fit it even at one step's worth of
 *     work items is refused with CT_ENOMEM, before the context changes (with
 *     the default FP32 launch the 256 events of 2222 holes of the 8 keV batch
 *     fit, or 7 events of 16,667 holes; the Newton-pair partial fields of one
 *     55,556-hole event, 175 MB, do not); a queue shorter than
 *     ct_seed_events' parks more events, which ct_step runs again (same
 *     results, more launches).
 *   - Every context on a GPU shares that GPU's array, which keeps the last
 *     user's contents (this call clears what must start at zero).  Seeding
 *     another context with this call on the same GPU takes the array over;
 *     ct_step, ct_collect, ct_field and ct_set_launch of the earlier context
 *     then return CT_ESTATE until it is seeded again.  Calls on contexts that
 *     share a GPU's array must not overlap in time: they race on it.
 * ct_step and ct_collect allocate nothing in any case; ct_field allocates its
 * output staging on first use. */
ct_status ct_seed_events_noalloc(ct_ctx *c, const ct_event_desc *ev, int32_t n_events,
                                 uint64_t first_event_id);

/* The time-step loop of Algorithm 1 (Appendix A): while an event has holes
 * drifting, evaluate the field of Eq. 4 at every drifting carrier from the
 * step-start positions, then move each carrier by Eqs. 3, 5 and 6 and
 * collect the holes that reach the pixel plane; the loop of an event ends
 * when its last hole is collected (Algorithm 1's loop condition: every hole
 * has reached the electrode) or after max_steps steps in this call
 * (max_steps <= 0: the context's max_steps).
 * Events advance independently: one persistent kernel works through a
 * device queue of (event, target tile, source chunk) items, and finishing an
 * event's step queues its next one, with no device-wide barrier between
 * steps.  steps_done (nullable): the most steps any event took in this call;
 * n_active (nullable): holes still drifting.  Returns CT_OK when none is
 * left, CT_EMAXSTEPS otherwise (state kept; call again to continue).  The
 * queue holds about 1024 steps of the batch at its seeded size (environment
 * variable CT_QUEUE_STEPS, read at seeding, sets another count); when it
 * fills, the events it cannot take are parked and run again by the same
 * call, which costs time but never changes results.  If no event step is
 * queued and no event finishes for 10 s, the kernel stops and the call
 * returns CT_EDEVICE (the context must then be destroyed). */
ct_status ct_step(ct_ctx *c, int64_t max_steps, int64_t *steps_done, int64_t *n_active);

/* The output of Algorithm 1 (the final carrier positions it returns) and the
 * carrier count per pixel of the collected holes (Sec. 4.2), copied to host
 * arrays (each nullable):
 *   pixel_counts [B][grid_n*grid_n + 1]  collected holes per pixel, last = outside the grid
 *                                         (electrons are never counted)
 *   xyz          [N_total][3]            position at collection, or current position if
 *                                         still drifting; events in order, carriers in
 *                                         their given order
 *   collect_step [N_total]               absolute step of collection, -1 = drifting
 *   event_steps  [B]                     steps each event has taken since seeding
 *   stats        run statistics */
ct_status ct_collect(ct_ctx *c, int32_t *pixel_counts, double *xyz, int32_t *collect_step,
                     int64_t *event_steps, ct_run_stats *stats);

/* Field of the other carriers (V/um, Eq. 4, each source with its sign; with
 * CT_SPHERICAL the field of Eq. 7) at every carrier, as the next step would
 * use it, computed by the same kernels and precision as ct_step
 * ([N_total][3], carrier order); drifting carriers only, NaN for
 * collected. */
ct_status ct_field(ct_ctx *c, double *field);

/* Philox4x32-10 blocks and the Box-Muller normals the kernels derive from
 * them, for n host counters [n][4] under the context's seed:
 * words [n][4] (nullable), normals [n][3] (nullable). */
ct_status ct_philox(ct_ctx *c, const uint32_t *counters, int64_t n, uint32_t *words,
                    double *normals);

/* Override the launch configuration: targets per thread (1, 2 or 4), block
 * size (64, 128 or 256; also the number of sources per LDS tile) and the
 * source chunk length (a multiple of the block size, at most 2^20): an event
 * of n holes is split into ceil(n / len) chunks of len sources, len being
 * chunk_len or, for events of more than 256 chunks, the shortest whole number
 * of tiles that keeps 256 chunks.  Each chunk of each target tile is one work
 * item.  With Newton pairs (see CT_OPT_ONE_SIDED) a tile of 256 holes meets
 * itself and about half of the other tiles, and an item takes chunk_len / 256
 * of them; longer chunks than 15 tiles, other block sizes or more targets per
 * thread select the one-sided kernel.  0 leaves a value unchanged.  The block size and the
 * chunk length set the grouping of the field sum, so they change results
 * within rounding. */
ct_status ct_set_launch(ct_ctx *c, int32_t targets_per_thread, int32_t block_size,
                        int32_t chunk_len);

/* Parameterised event generation (Sec. 4.2): photon events drawn from the
 * modelling of Sec. 3 instead of simulated.  Per event (id first_event_id + b):
 *   depth h from the entrance side, exponential with atten_um, conditioned on
 *   absorption inside the sensor; the drift time t of Eq. 9 for holes from h
 *   (Jacoboni-Canali hole mu0 and E_c of the context, the field of Eq. 6);
 *   alpha(t) = p_alpha[0] + p_alpha[1] sqrt(t) + p_alpha[2] t + p_alpha[3] t^2
 *   (Eq. 10) and beta(t) = 2 + p_beta[0] (t - p_beta[1])^p_beta[2]
 *   + p_beta[3] exp(p_beta[4] t) (Eq. 11); the carrier count
 *   N = max(0, floor(E/w + sqrt(fano E/w) g + 1/2)) with g standard normal;
 *   a sub-pixel shift (x0, y0) uniform over the central pixel; each carrier's
 *   pixel drawn from the generalized Gaussian of Eq. 8 (scale alpha, shape
 *   beta, centred on the shift, x and y independent) over the context's
 *   grid_n x grid_n pixels of pitch_um (outside: the overflow bin); pixel
 *   energies count * w + noise_kev * normal.
 * Random draws: Philox counters (0, 0, id, 5) for the depth and shift,
 * (1, 0, id, 5) for the count's normal, (j, 1, id, 5) for carriers 2j and
 * 2j + 1, (p / 3, 2, id, 5) for the noise of pixel p, under the context's seed.
 * Outputs are DEVICE pointers owned by the caller, each nullable:
 *   energy [n_events][grid_n^2] (keV), counts [n_events][grid_n^2 + 1] (the
 *   last is the overflow bin), info [n_events][5] = h (um), t (ns), N, x0, y0.
 * The work is queued on the context's stream; with kernel_ms (nullable, host)
 * the call waits for it and returns its duration.  Needs grid_n <= 8 and
 * 0 <= v_dep < v_bias; p_beta[1] < 0; alpha(t) and beta(t) positive for every
 * drift time of the sensor (CT_EINVAL otherwise).  No seeded batch needed. */
typedef struct {
    double energy_kev;  /* photon energy > 0 */
    double fano;        /* Fano factor >= 0 (0.13 in Sec. 4.2) */
    double noise_kev;   /* pixel noise sigma >= 0 (0.13 keV in Sec. 4.2) */
    double atten_um;    /* absorption length of the photons in the sensor > 0 */
    double p_alpha[4];  /* Eq. 10 */
    double p_beta[5];   /* Eq. 11 */
} ct_gen_params;

ct_status ct_generate(ct_ctx *c, const ct_gen_params *g, int64_t n_events,
                      uint64_t first_event_id, double *energy, int32_t *counts, double *info,
                      float *kernel_ms);

void ct_destroy(ct_ctx *c);

const char *ct_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CT_H */
