// Host side of the C ABI declared in include/ct.h: parameter validation,
// device workspace, batch seeding, the step loop and result collection.
// Every numerical step of the method runs in the kernels of ct_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include <sys/stat.h>

#include "ct.h"
#include "ct_internal.hpp"
#include "ct_sph_layout.hpp"
#include "ct_track.hpp"

namespace {

thread_local std::string g_err;

ct_status fail(ct_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define CT_HIP(call)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(CT_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));             \
    } while (0)

// SI exact values (e, k) and CODATA 2022 vacuum permittivity.
constexpr double kElementaryCharge = 1.602176634e-19;  // C
constexpr double kBoltzmann = 1.380649e-23;            // J/K
constexpr double kVacuumPermittivity = 8.8541878188e-12; // F/m
constexpr double kPi = 3.14159265358979323846;

// Jacoboni-Canali hole parameters at T in the Caughey-Thomas form:
// vm = 1.62e8 T^-0.52 cm/s, Ec = 1.24 T^1.68 V/cm, beta = 0.46 T^0.17;
// returned as mu0 = vm/Ec [um^2/(V ns)], Ec [V/um], beta.
void hole_mobility_params(const ct_sensor_params &p, double &mu0, double &ec, double &beta)
{
    const double T = p.temperature_k;
    const double vm_um_ns = 1.62e8 * std::pow(T, -0.52) * 1e-5;
    ec = 1.24 * std::pow(T, 1.68) * 1e-4;
    beta = 0.46 * std::pow(T, 0.17);
    mu0 = vm_um_ns / ec;
    if (!std::isnan(p.mu0_override)) mu0 = p.mu0_override;
    if (!std::isnan(p.ec_override)) ec = p.ec_override;
    if (!std::isnan(p.beta_override)) beta = p.beta_override;
}

// Jacoboni-Canali electron parameters at T: vm = 1.53e9 T^-0.87 cm/s,
// Ec = 1.01 T^1.55 V/cm, beta = 2.57e-2 T^0.66; mu0 = vm/Ec.
void electron_mobility_params(const ct_sensor_params &p, double &mu0, double &ec, double &beta)
{
    const double T = p.temperature_k;
    const double vm_um_ns = 1.53e9 * std::pow(T, -0.87) * 1e-5;
    ec = 1.01 * std::pow(T, 1.55) * 1e-4;
    beta = 2.57e-2 * std::pow(T, 0.66);
    mu0 = vm_um_ns / ec;
    if (!std::isnan(p.mu0_e_override)) mu0 = p.mu0_e_override;
    if (!std::isnan(p.ec_e_override)) ec = p.ec_e_override;
    if (!std::isnan(p.beta_e_override)) beta = p.beta_e_override;
}

ct_status check_params(const ct_sensor_params *p)
{
    if (!p) return fail(CT_EINVAL, "params is NULL");
    if (p->abi_version != CT_ABI_VERSION)
        return fail(CT_EINVAL, "abi_version %u, library has %u", p->abi_version, CT_ABI_VERSION);
    if (!(p->thickness_um > 0.0) || !std::isfinite(p->thickness_um))
        return fail(CT_EINVAL, "thickness_um must be finite and > 0");
    if (!(p->dt_ns > 0.0) || !std::isfinite(p->dt_ns)) return fail(CT_EINVAL, "dt_ns must be > 0");
    if (!(p->temperature_k > 0.0)) return fail(CT_EINVAL, "temperature_k must be > 0");
    if (!(p->pitch_um > 0.0)) return fail(CT_EINVAL, "pitch_um must be > 0");
    if (p->grid_n < 1 || p->grid_n > 64) return fail(CT_EINVAL, "grid_n must be in 1..64");
    if (!(p->softening_um >= 0.0) || !std::isfinite(p->softening_um))
        return fail(CT_EINVAL, "softening_um must be >= 0");
    if (!(p->eps_r > 0.0)) return fail(CT_EINVAL, "eps_r must be > 0");
    if (!(p->pair_energy_ev > 0.0)) return fail(CT_EINVAL, "pair_energy_ev must be > 0");
    if (p->mobility != CT_MOB_JACOBONI && p->mobility != CT_MOB_CONSTANT)
        return fail(CT_EINVAL, "unknown mobility model %d", p->mobility);
    if (p->precision != CT_FP64 && p->precision != CT_FP32)
        return fail(CT_EINVAL, "unknown precision %d", p->precision);
    if (p->physics_flags & ~31u) return fail(CT_EINVAL, "unknown physics flag bits");
    if ((p->physics_flags & CT_SPHERICAL) && (p->physics_flags & CT_ELECTRONS))
        return fail(CT_EINVAL, "the spherical model (Eq. 7) simulates holes only");
    if ((p->physics_flags & CT_DRIFT) && !(p->v_bias > p->v_dep && p->v_dep >= 0.0))
        return fail(CT_EINVAL, "the linear drift field needs 0 <= v_dep < v_bias (Eq. 6)");
    if (p->max_steps <= 0) return fail(CT_EINVAL, "max_steps must be > 0");
    if (p->options & ~(uint32_t)(CT_OPT_TIMING | CT_OPT_AUTOTUNE | CT_OPT_ONE_SIDED))
        return fail(CT_EINVAL, "unknown option bits 0x%x", p->options);
    double mu0, ec, beta;
    hole_mobility_params(*p, mu0, ec, beta);
    if (!(mu0 > 0.0) || !(ec > 0.0) || !(beta > 0.0) || !std::isfinite(mu0))
        return fail(CT_EINVAL, "mobility parameters must be > 0");
    electron_mobility_params(*p, mu0, ec, beta);
    if (!(mu0 > 0.0) || !(ec > 0.0) || !(beta > 0.0) || !std::isfinite(mu0))
        return fail(CT_EINVAL, "electron mobility parameters must be > 0");
    return CT_OK;
}

ct::DevParams make_dev_params(const ct_sensor_params &p)
{
    ct::DevParams d{};
    const double H = p.thickness_um;
    d.H = H;
    d.e0 = (p.v_bias + p.v_dep) / H;
    d.e1 = 2.0 * p.v_dep / (H * H);
    d.dt = p.dt_ns;
    d.K = kElementaryCharge / (4.0 * kPi * kVacuumPermittivity * p.eps_r) * 1e6;
    d.kT = kBoltzmann * p.temperature_k / kElementaryCharge;
    // A tiny floor keeps the self-pair term 0 * finite when s = 0.
    d.s2 = std::max(p.softening_um * p.softening_um, 1e-20);
    d.s2f = (float)d.s2;
    hole_mobility_params(p, d.mu0, d.ec, d.beta);
    d.inv_beta = 1.0 / d.beta;
    d.inv_ec = 1.0 / d.ec;
    electron_mobility_params(p, d.mu0_e, d.ec_e, d.beta_e);
    d.inv_beta_e = 1.0 / d.beta_e;
    d.inv_ec_e = 1.0 / d.ec_e;
    d.pitch = p.pitch_um;
    d.half_width = 0.5 * p.grid_n * p.pitch_um;
    d.grid_n = p.grid_n;
    d.mobility = p.mobility;
    d.flags = p.physics_flags;
    d.key0 = (uint32_t)p.seed;
    d.key1 = (uint32_t)(p.seed >> 32);
    return d;
}

// Holes of an event (Algorithm 1: round(1000 E / w) unless stated).
int32_t carrier_count(const ct_sensor_params &p, const ct_event_desc &e)
{
    if (e.n_carriers > 0) return e.n_carriers;
    const double n = std::floor(1000.0 * e.energy_kev / p.pair_energy_ev + 0.5);
    return n > 0.0 ? (int32_t)n : 0;
}

double initial_sigma(const ct_event_desc &e)
{
    if (e.sigma_um >= 0.0) return e.sigma_um;
    return 0.0044 * std::pow(e.energy_kev, 1.75);  // Eq. 2, um with E in keV
}

// Byte layout of one batch inside a single device buffer.
struct Layout {
    size_t off, n_act, n_hole, nh0, ev_step, ev_taken, call_steps, ref, pos, idx, nidx, rngid,
        out_xyz, out_cstep, pix, pairs, hsteps, sigma, dep_off, deposits, x_off, xyz_in, start,
        seg_len, sph, total;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// spherical: room for the keys of the spherical model (2 N doubles).
Layout make_layout(int64_t B, int64_t N, int64_t n_dep, int64_t n_exp, int G1, bool spherical)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + std::max<size_t>(bytes, 1));
        return at;
    };
    L.off = take(sizeof(int32_t) * (B + 1));
    L.n_act = take(sizeof(int32_t) * B);
    L.n_hole = take(sizeof(int32_t) * B);
    L.nh0 = take(sizeof(int32_t) * B);
    L.ev_step = take(sizeof(int64_t) * B);
    L.ev_taken = take(sizeof(int64_t) * B);
    L.call_steps = take(sizeof(int64_t) * B);
    L.ref = take(sizeof(double) * 4 * B);
    L.pos = take(sizeof(double) * 6 * N);
    L.idx = take(sizeof(int32_t) * N);
    L.nidx = take(sizeof(int32_t) * N);
    L.rngid = take(sizeof(int32_t) * N);
    L.out_xyz = take(sizeof(double) * 3 * N);
    L.out_cstep = take(sizeof(int32_t) * N);
    L.pix = take(sizeof(int32_t) * B * G1);
    L.pairs = take(sizeof(uint64_t) * B);
    L.hsteps = take(sizeof(uint64_t) * B);
    L.sigma = take(sizeof(double) * B);
    L.dep_off = take(sizeof(int32_t) * (B + 1));
    L.deposits = take(sizeof(double) * 3 * n_dep);
    L.x_off = take(sizeof(int32_t) * (B + 1));
    L.xyz_in = take(sizeof(double) * 3 * n_exp);
    L.start = take(sizeof(int64_t) * B);
    L.seg_len = take(sizeof(double) * B);
    L.sph = take(spherical ? sizeof(double) * 2 * N : 0);
    L.total = o;
    return L;
}

struct BatchShape {
    int64_t B = 0, N = 0, n_dep = 0, n_exp = 0;
    bool tracks = false;  // some event is a track (its deposits are computed at seeding)
    int32_t n_max = 0;
    std::vector<int32_t> n;   // carriers of each event (holes + electrons)
    std::vector<int32_t> nh;  // holes of each event
};

ct_status shape_of(const ct_sensor_params &p, const ct_event_desc *ev, int32_t B, BatchShape &s)
{
    if (B < 0) return fail(CT_EINVAL, "n_events must be >= 0");
    if (B > 0 && !ev) return fail(CT_EINVAL, "events is NULL");
    s = BatchShape{};
    s.B = B;
    s.n.resize(B);
    s.nh.resize(B);
    const bool electrons = (p.physics_flags & CT_ELECTRONS) != 0;
    for (int32_t b = 0; b < B; ++b) {
        const ct_event_desc &e = ev[b];
        if (e.n_deposits < 0) return fail(CT_EINVAL, "event %d: n_deposits < 0", b);
        if (e.n_deposits > 0 && !e.deposits) return fail(CT_EINVAL, "event %d: deposits missing", b);
        if (!(e.seg_len_um >= 0.0) || !std::isfinite(e.seg_len_um))
            return fail(CT_EINVAL, "event %d: seg_len_um must be finite and >= 0", b);
        if (e.seg_len_um > 0.0 && e.n_deposits == 0)
            return fail(CT_EINVAL, "event %d: a track has n_deposits >= 1 segments", b);
        if ((e.n_carriers <= 0 || e.sigma_um < 0.0) && !(e.energy_kev > 0.0) && e.n_deposits > 0)
            return fail(CT_EINVAL, "event %d: energy needed for the carrier count or width", b);
        if (e.n_deposits == 0 && e.n_carriers <= 0 && e.energy_kev != 0.0)
            return fail(CT_EINVAL, "event %d: explicit events state n_carriers", b);
        const int32_t nh = carrier_count(p, e);
        if (e.n_deposits > 0 && !std::isfinite(initial_sigma(e)))
            return fail(CT_EINVAL, "event %d: width not finite", b);
        int32_t ne = 0;
        if (electrons) ne = e.n_electrons >= 0 ? e.n_electrons : nh;
        else if (e.n_electrons > 0)
            return fail(CT_EINVAL, "event %d: electrons given without CT_ELECTRONS", b);
        if (e.n_deposits > 0 && ne != 0 && ne != nh)
            return fail(CT_EINVAL, "event %d: a cloud event has one electron per hole", b);
        if ((int64_t)nh + ne > INT32_MAX / 2) return fail(CT_EINVAL, "event %d too large", b);
        const int32_t n = nh + ne;
        if (e.n_deposits == 0 && n > 0 && !e.xyz)
            return fail(CT_EINVAL, "event %d: explicit positions missing", b);
        s.nh[b] = nh;
        s.n[b] = n;
        s.N += n;
        s.n_max = std::max(s.n_max, n);
        s.n_dep += e.n_deposits;
        if (e.n_deposits == 0) s.n_exp += n;
        if (e.seg_len_um > 0.0) s.tracks = true;
    }
    if (s.N > INT32_MAX / 2) return fail(CT_EINVAL, "batch has too many carriers (%lld)", (long long)s.N);
    return CT_OK;
}

// Launch configuration of a new context (ct_set_launch overrides it): one
// target per thread, 256-thread workgroups, sources in chunks of 1280 (the
// fastest whole-run length on batches of 2222- to 6111-hole events; longer
// chunks mean fewer partial fields per step, shorter ones more work items to
// spread over the workgroups).
ct::LaunchCfg default_cfg(const ct_sensor_params &p)
{
    (void)p;
    return ct::LaunchCfg{1, 256, 1280};
}

// Tickets the work queue holds per run: about 1024 steps of the batch at its
// initial size (the environment variable CT_QUEUE_STEPS overrides the 1024),
// at least one step, at most 2^26 tickets (36 B each: 2.4 GB at most); a run
// that fills it parks the events it could not queue and the host runs again,
// which costs a drain of the GPU per extra run.
constexpr int64_t kQueueSteps = 1024;
constexpr int64_t kQueueMax = int64_t(1) << 26;

int64_t queue_steps()
{
    const char *v = std::getenv("CT_QUEUE_STEPS");
    if (!v || !*v) return kQueueSteps;
    const long long k = std::atoll(v);
    return k >= 1 ? (int64_t)k : kQueueSteps;
}

// Work queue, completion counters and partial-field buffer of a batch for a
// launch configuration, in one device allocation.
struct QueueLayout {
    size_t sched, q, seq, tiles_left, chunks_left, tile_base, part_off, part, tk_off, grp_off, grp,
        single, total;
    uint32_t cap;
    int32_t n_tickets;
    std::vector<int32_t> tile_base_h, tk_off_h, single_h;
    std::vector<int64_t> part_off_h, grp_off_h;
};

// The spherical model runs without a work queue: it keeps the control block,
// its tickets (one per workgroup of each event; sph_max_group bounds the
// workgroups sharing an event) and the state of shared events.
QueueLayout make_queue_layout(const BatchShape &s, const ct::LaunchCfg &cfg, bool repulsion,
                              bool spherical, int sph_max_group, int64_t cap_max = kQueueMax)
{
    QueueLayout Q{};
    const int64_t T = (int64_t)cfg.kt * cfg.bs;
    Q.tile_base_h.assign(s.B + 1, 0);
    Q.part_off_h.assign(s.B + 1, 0);
    int64_t items = 0;
    for (int64_t b = 0; b < s.B; ++b) {
        const int64_t n0 = s.n[b];
        const int64_t tiles = spherical ? 0 : (n0 + T - 1) / T;
        // chunks of any later (smaller) count stay within this bound
        int64_t chunks = 1;
        if (repulsion && n0 > 0 && !spherical)
            chunks = std::min<int64_t>((n0 + cfg.chunk - 1) / cfg.chunk, ct::kMaxChunks);
        int64_t slots = chunks > 1 ? chunks : 0;
        int64_t ev_items = tiles * chunks;
        if (cfg.newton && n0 > 0) {
            // slots and items grow with the hole count within each of the two
            // splits: bound both at the largest count that takes each
            const int ct_ = cfg.chunk / ct::kSymTile;
            const int n_sym = (int)std::min<int64_t>(n0, (int64_t)ct::kSymMaxTiles * ct::kSymTile);
            const ct::SymSplit a = ct::sym_split(n_sym, ct_);
            const ct::SymSplit z = ct::sym_split((int)n0, ct_);
            slots = std::max<int64_t>(ct::sym_slots(a), z.newton ? 0 : chunks);
            ev_items = std::max<int64_t>((int64_t)a.T * a.R, z.newton ? 0 : tiles * chunks);
        }
        Q.tile_base_h[b + 1] = Q.tile_base_h[b] + (int32_t)tiles;
        Q.part_off_h[b + 1] = Q.part_off_h[b] + 3 * n0 * slots;
        items += ev_items;
    }
    Q.tk_off_h.assign(s.B + 1, 0);
    Q.grp_off_h.assign(s.B + 1, 0);
    for (int64_t b = 0; b < s.B; ++b) {
        const int G = spherical && repulsion ? ct::sph_group(s.n[b], sph_max_group) : 1;
        Q.tk_off_h[b + 1] = Q.tk_off_h[b] + G;
        Q.grp_off_h[b + 1] = Q.grp_off_h[b] + (G > 1 ? (int64_t)ct::sph_group_bytes(G) : 0);
        if (G == 1) Q.single_h.push_back((int32_t)b);
    }
    Q.n_tickets = Q.tk_off_h[s.B];
    int64_t cap = std::max<int64_t>(items, std::min<int64_t>(items * queue_steps(),
                                                             std::min(kQueueMax, cap_max)));
    cap = std::max<int64_t>(cap, 1);
    Q.cap = (uint32_t)cap;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + std::max<size_t>(bytes, 1));
        return at;
    };
    Q.sched = take(sizeof(ct::Sched));
    Q.q = take(sizeof(ct::QItem) * cap);
    Q.seq = take(sizeof(uint32_t) * cap);
    Q.tiles_left = take(sizeof(int32_t) * s.B * ct::kEventLine);
    Q.chunks_left = take(sizeof(int32_t) * Q.tile_base_h[s.B]);
    Q.tile_base = take(sizeof(int32_t) * (s.B + 1));
    Q.part_off = take(sizeof(int64_t) * (s.B + 1));
    Q.part = take(sizeof(double) * Q.part_off_h[s.B]);
    Q.tk_off = take(sizeof(int32_t) * (s.B + 1));
    Q.grp_off = take(sizeof(int64_t) * (s.B + 1));
    Q.grp = take((size_t)Q.grp_off_h[s.B]);
    Q.single = take(sizeof(int32_t) * Q.single_h.size());
    Q.total = o;
    return Q;
}

}  // namespace

struct ct_ctx {
    ct_sensor_params p{};
    ct::DevParams dp{};
    int device = 0;
    hipStream_t stream = nullptr;  // the caller's stream, or one of ours
    bool own_stream = false;
    ct::LaunchCfg cfg{1, 256, 1280};
    int cu_count = 0;
    std::string arch;  // gcnArchName of the device
    int grid = 0;  // resident workgroups of the run kernel for cfg
    int grid_shared = 0;  // spherical model: workgroups over the events shared by several

    // device workspace (the batch)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_bound = false;
    void *bound_ptr = nullptr;
    size_t bound_bytes = 0;
    double *field_buf = nullptr;
    size_t field_buf_n = 0;

    // work queue of the batch for cfg
    void *qbuf = nullptr;
    size_t qbuf_bytes = 0;
    ct::DevQueue dq{};
    bool in_scratch = false;  // the queue lives in the device's shared scratch (ct_seed_events_noalloc)
    uint32_t gen = 0;
    bool broken = false;  // a run reported an error; only ct_destroy is allowed

    // batch
    bool seeded = false;
    Layout L{};
    ct::DevBatch bt{};
    BatchShape shape;
    std::vector<int64_t> start_h;  // start step of each event (host copy, for re-seeding)
    int64_t n_active = 0;
    int64_t steps = 0;

    ct::Sched *h_sched = nullptr;  // pinned copy of the control block
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    int64_t field_launches = 0;
    double field_ms = 0.0;
    double step_wall_ms = 0.0;
};

namespace {

ct_status release_workspace(ct_ctx *c)
{
    if (c->ws && !c->ws_bound) CT_HIP(hipFree(c->ws));
    c->ws = nullptr;
    c->ws_bytes = 0;
    c->ws_bound = false;
    return CT_OK;
}

ct_status ensure_workspace(ct_ctx *c, size_t bytes)
{
    if (c->bound_ptr) {
        if (c->bound_bytes < bytes)
            return fail(CT_ENOMEM, "bound workspace has %zu bytes, batch needs %zu", c->bound_bytes,
                        bytes);
        if (c->ws && !c->ws_bound) CT_HIP(hipFree(c->ws));
        c->ws = c->bound_ptr;
        c->ws_bytes = c->bound_bytes;
        c->ws_bound = true;
        return CT_OK;
    }
    if (c->ws && !c->ws_bound && c->ws_bytes >= bytes) return CT_OK;
    ct_status st = release_workspace(c);
    if (st != CT_OK) return st;
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CT_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    c->ws = p;
    c->ws_bytes = bytes;
    c->ws_bound = false;
    return CT_OK;
}

template <class T>
T *at(void *base, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

ct_status set_device(ct_ctx *c)
{
    CT_HIP(hipSetDevice(c->device));
    return CT_OK;
}

// The context whose batch queue occupies each device's scratch (seeded with
// ct_seed_events_noalloc).  A later such seeding on the same device takes the
// scratch over; the earlier context's calls then fail with CT_ESTATE instead
// of running on a queue that is no longer its own.
std::mutex g_owner_mu;
std::map<int, const ct_ctx *> g_owner;

void claim_scratch(const ct_ctx *c)
{
    std::lock_guard<std::mutex> lk(g_owner_mu);
    g_owner[c->device] = c;
}

void release_scratch(const ct_ctx *c)
{
    std::lock_guard<std::mutex> lk(g_owner_mu);
    auto it = g_owner.find(c->device);
    if (it != g_owner.end() && it->second == c) g_owner.erase(it);
}

// CT_OK unless the context's queue was in the scratch and another context
// has taken the scratch over since.
ct_status check_scratch(const ct_ctx *c)
{
    if (!c->seeded || !c->in_scratch) return CT_OK;
    std::lock_guard<std::mutex> lk(g_owner_mu);
    auto it = g_owner.find(c->device);
    if (it == g_owner.end() || it->second != c)
        return fail(CT_ESTATE, "the scratch of device %d now holds another context's batch "
                               "(ct_seed_events_noalloc); seed this context again", c->device);
    return CT_OK;
}

// Work queue of the seeded batch for cfg, and the resident grid.  The queue
// memory is kept while it is large enough; its sequence words are cleared
// whenever it is (re)allocated, so no stale ticket can match a generation.
// The launch configuration with the Newton-pair kernel switched on where it
// applies: FP32 repulsion, one target per thread, blocks of kSymTile, at
// most kSymMaxC tiles per chunk (with electrons, the kernel that carries the
// carriers' charges).
ct::LaunchCfg resolve_cfg(const ct_ctx *c, ct::LaunchCfg cfg)
{
    const uint32_t f = c->p.physics_flags;
    const bool on = c->p.precision == CT_FP32 && (f & CT_REPULSION) && !(f & CT_SPHERICAL) &&
                    !(c->p.options & CT_OPT_ONE_SIDED) && cfg.kt == 1 && cfg.bs == ct::kSymTile &&
                    cfg.chunk % ct::kSymTile == 0 && cfg.chunk / ct::kSymTile <= ct::kSymMaxC;
    cfg.newton = on ? ((f & CT_ELECTRONS) ? 2 : 1) : 0;
    return cfg;
}

ct_status prepare_queue(ct_ctx *c, const ct::LaunchCfg &cfg_in)
{
    const ct::LaunchCfg cfg = resolve_cfg(c, cfg_in);
    const bool repulsion = (c->p.physics_flags & CT_REPULSION) != 0;
    const bool spherical = (c->p.physics_flags & CT_SPHERICAL) != 0;
    int sph_cap = 0;
    if (spherical) {
        const int occ = ct::sph_occupancy();
        if (occ <= 0) return fail(CT_EDEVICE, "spherical kernel occupancy query failed");
        sph_cap = occ * c->cu_count;
        if (sph_cap < 2) return fail(CT_EDEVICE, "fewer than 2 resident spherical workgroups");
    }
    QueueLayout Q = make_queue_layout(c->shape, cfg, repulsion, spherical, sph_cap);
    hipStream_t sm = c->stream;
    void *qmem = nullptr;
    if (c->in_scratch) {
        // the device's shared scratch: no allocation.  A queue of fewer
        // tickets than usual parks more events (run again by ct_step, same
        // results); everything is cleared, since the array keeps the
        // contents of the last context that used it.
        size_t sbytes = 0;
        CT_HIP(ct::scratch_memory(c->device, &qmem, &sbytes));
        if (Q.total > sbytes) {
            const QueueLayout Qmin = make_queue_layout(c->shape, cfg, repulsion, spherical, sph_cap, 1);
            if (Qmin.total > sbytes)
                return fail(CT_ENOMEM, "the batch's work queue needs %zu bytes; the scratch of "
                                       "ct_seed_events_noalloc has %zu", Qmin.total, sbytes);
            const int64_t per = sizeof(ct::QItem) + sizeof(uint32_t);
            int64_t cap = (int64_t)Qmin.cap + (int64_t)(sbytes - Qmin.total) / per;
            do {
                Q = make_queue_layout(c->shape, cfg, repulsion, spherical, sph_cap, cap);
                cap -= 64;
            } while (Q.total > sbytes);
        }
        CT_HIP(ct::launch_fill_i32((int32_t *)qmem, (int64_t)(Q.total / 4), 0, sm));
    } else if (Q.total > c->qbuf_bytes) {
        if (c->qbuf) {
            CT_HIP(hipStreamSynchronize(sm));
            CT_HIP(hipFree(c->qbuf));
        }
        c->qbuf = nullptr;
        c->qbuf_bytes = 0;
        if (hipMalloc(&c->qbuf, Q.total) != hipSuccess) {
            (void)hipGetLastError();
            c->qbuf = nullptr;
            return fail(CT_ENOMEM, "work queue of %zu bytes failed", Q.total);
        }
        c->qbuf_bytes = Q.total;
        CT_HIP(ct::launch_fill_i32((int32_t *)c->qbuf, (int64_t)(c->qbuf_bytes / 4), 0, sm));
        qmem = c->qbuf;
    } else {
        // the sequence words move with the layout: clear them for this one
        CT_HIP(ct::launch_fill_i32(at<int32_t>(c->qbuf, Q.seq), (int64_t)Q.cap, 0, sm));
        qmem = c->qbuf;
    }
    ct::DevQueue d{};
    d.sc = at<ct::Sched>(qmem, Q.sched);
    d.q = at<ct::QItem>(qmem, Q.q);
    d.seq = at<uint32_t>(qmem, Q.seq);
    d.cap = Q.cap;
    d.tiles_left = at<int32_t>(qmem, Q.tiles_left);
    d.chunks_left = at<int32_t>(qmem, Q.chunks_left);
    d.tile_base = at<int32_t>(qmem, Q.tile_base);
    d.part = at<double>(qmem, Q.part);
    d.part_off = at<int64_t>(qmem, Q.part_off);
    d.tk_off = at<int32_t>(qmem, Q.tk_off);
    d.grp_off = at<int64_t>(qmem, Q.grp_off);
    d.grp = at<char>(qmem, Q.grp);
    d.n_tickets = Q.n_tickets;
    d.single = at<int32_t>(qmem, Q.single);
    if (c->shape.B > 0) {
        CT_HIP(hipMemcpyAsync((void *)d.tile_base, Q.tile_base_h.data(),
                              sizeof(int32_t) * (c->shape.B + 1), hipMemcpyHostToDevice, sm));
        CT_HIP(hipMemcpyAsync((void *)d.part_off, Q.part_off_h.data(),
                              sizeof(int64_t) * (c->shape.B + 1), hipMemcpyHostToDevice, sm));
        CT_HIP(hipMemcpyAsync((void *)d.tk_off, Q.tk_off_h.data(),
                              sizeof(int32_t) * (c->shape.B + 1), hipMemcpyHostToDevice, sm));
        CT_HIP(hipMemcpyAsync((void *)d.grp_off, Q.grp_off_h.data(),
                              sizeof(int64_t) * (c->shape.B + 1), hipMemcpyHostToDevice, sm));
        if (!Q.single_h.empty())
            CT_HIP(hipMemcpyAsync((void *)d.single, Q.single_h.data(),
                                  sizeof(int32_t) * Q.single_h.size(), hipMemcpyHostToDevice, sm));
        CT_HIP(hipStreamSynchronize(sm));  // host vectors go out of scope
    }
    c->dq = d;
    if (spherical) {
        // resident workgroups claiming the tickets (at least the largest group)
        const int single = (int)Q.single_h.size();
        c->grid = single;  // one workgroup per single-workgroup event
        c->grid_shared = std::min<int>(Q.n_tickets - single, sph_cap);
        return CT_OK;
    }
    const int occ = ct::run_occupancy(cfg, c->p.precision == CT_FP32);
    if (occ <= 0) return fail(CT_EDEVICE, "run kernel occupancy query failed");
    c->grid = occ * c->cu_count;
    return CT_OK;
}

// One run of the persistent kernel: queue the first step of every eligible
// event, run until every event is finished or parked, then read back the
// control block (and the drifting-hole count and steps taken).
ct_status run_once(ct_ctx *c, const ct::LaunchCfg &cfg_in, int64_t max_steps, int field_only,
                   double *field_out, bool timing)
{
    const ct::LaunchCfg cfg = resolve_cfg(c, cfg_in);
    if (++c->gen == 0) ++c->gen;  // 0 is the cleared state of a sequence word
    c->dq.gen = c->gen;
    const int fp32 = c->p.precision == CT_FP32;
    const int repulsion = (c->p.physics_flags & CT_REPULSION) != 0;
    hipStream_t sm = c->stream;
    CT_HIP(ct::launch_init(c->bt, c->dq, cfg, max_steps, field_only, repulsion, sm));
    if (timing) CT_HIP(hipEventRecord(c->ev_a, sm));
    CT_HIP(ct::launch_run(c->dp, c->bt, c->dq, cfg, fp32, c->grid, max_steps, field_only, field_out,
                          sm));
    if (timing) CT_HIP(hipEventRecord(c->ev_b, sm));
    CT_HIP(ct::launch_summary(c->bt, c->dq.sc, sm));
    CT_HIP(hipMemcpyAsync(c->h_sched, c->dq.sc, sizeof(ct::Sched), hipMemcpyDeviceToHost, sm));
    CT_HIP(hipStreamSynchronize(sm));
    if (timing) {
        float ms = 0.0f;
        CT_HIP(hipEventElapsedTime(&ms, c->ev_a, c->ev_b));
        c->field_ms += ms;
        c->field_launches += 1;
    }
    if (c->h_sched->error.v) {
        c->broken = true;
        const uint32_t *w = c->h_sched->stall.pad;
        if (c->h_sched->error.v == 2u)
            return fail(CT_EDEVICE, "work queue too small for the first step (internal error)");
        return fail(CT_EDEVICE,
                    "step kernel stopped: no event step queued or finished for 10 s (waiting for "
                    "ticket %u; head %u, tail %u, events done %u of %d)",
                    w[0], w[1], w[2], w[3], (int)c->shape.B);
    }
    return CT_OK;
}

// One run of the spherical model: every event to completion or the step cap
// (or, field_only, the field of its drifting holes), then the drifting-hole
// count and steps taken.
ct_status run_sph(ct_ctx *c, int64_t max_steps, int field_only, double *field_out, bool timing)
{
    hipStream_t sm = c->stream;
    if (timing) CT_HIP(hipEventRecord(c->ev_a, sm));
    CT_HIP(ct::launch_sph(c->dp, c->bt, c->dq, at<double>(c->ws, c->L.sph), c->grid,
                          c->grid_shared, max_steps, field_only, field_out, sm));
    if (timing) CT_HIP(hipEventRecord(c->ev_b, sm));
    CT_HIP(ct::launch_summary(c->bt, c->dq.sc, sm));
    CT_HIP(hipMemcpyAsync(c->h_sched, c->dq.sc, sizeof(ct::Sched), hipMemcpyDeviceToHost, sm));
    CT_HIP(hipStreamSynchronize(sm));
    if (timing) {
        float ms = 0.0f;
        CT_HIP(hipEventElapsedTime(&ms, c->ev_a, c->ev_b));
        c->field_ms += ms;
        c->field_launches += 1;
    }
    if (c->h_sched->error.v) {
        c->broken = true;
        return fail(CT_EDEVICE, "spherical kernel stopped: the workgroups of a shared event did not "
                                "meet within 10 s");
    }
    return CT_OK;
}

bool spherical(const ct_ctx *c) { return (c->p.physics_flags & CT_SPHERICAL) != 0; }

ct_status ensure_field_buf(ct_ctx *c, int64_t N)
{
    if (c->field_buf_n >= (size_t)N) return CT_OK;
    if (c->field_buf) CT_HIP(hipFree(c->field_buf));
    c->field_buf = nullptr;
    c->field_buf_n = 0;
    if (hipMalloc((void **)&c->field_buf, sizeof(double) * 3 * std::max<int64_t>(N, 1)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CT_ENOMEM, "field buffer allocation failed");
    }
    c->field_buf_n = (size_t)N;
    return CT_OK;
}

// The field the next step would apply, into field_buf (NaN for collected).
ct_status field_into_buf(ct_ctx *c, const ct::LaunchCfg &cfg, bool timing)
{
    const int64_t N = c->shape.N;
    CT_HIP(ct::launch_fill_i32((int32_t *)c->field_buf, 6 * N, (int32_t)0xFFFFFFFF, c->stream));
    if (spherical(c)) return run_sph(c, INT64_MAX, 1, c->field_buf, timing);
    return run_once(c, cfg, INT64_MAX, 1, c->field_buf, timing);
}

ct_status reset_state(ct_ctx *c);

// Launch configurations chosen by the autotuner.  Key: device architecture,
// compute units, precision, physics switches, options that change the
// kernel, and the batch shape in powers of two (events, largest event, total
// carriers).  Kept in memory and in a text file (CT_TUNE_CACHE, default
// $XDG_CACHE_HOME or ~/.cache /ct_launch_cache.txt; one "key|kt bs chunk"
// line per entry), so that later processes reuse it.
std::map<std::string, ct::LaunchCfg> g_tuned;
std::mutex g_tuned_mu;
bool g_tuned_loaded = false;

int log2_bucket(int64_t v)
{
    int b = 0;
    while (v > 1) {
        v >>= 1;
        ++b;
    }
    return b;
}

std::string tune_cache_path()
{
    if (const char *v = std::getenv("CT_TUNE_CACHE")) return v;
    std::string dir;
    if (const char *x = std::getenv("XDG_CACHE_HOME")) dir = x;
    else if (const char *h = std::getenv("HOME")) dir = std::string(h) + "/.cache";
    else return "";
    return dir + "/ct_launch_cache.txt";
}

void load_tune_cache()  // g_tuned_mu held
{
    if (g_tuned_loaded) return;
    g_tuned_loaded = true;
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char *bar = std::strchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        ct::LaunchCfg cfg{};
        if (std::sscanf(bar + 1, "%d %d %d", &cfg.kt, &cfg.bs, &cfg.chunk) == 3 &&
            ct::launch_supported(cfg.kt, cfg.bs) && cfg.chunk >= cfg.bs && cfg.chunk % cfg.bs == 0)
            g_tuned[line] = cfg;
    }
    std::fclose(f);
}

void store_tune_cache(const std::string &key, const ct::LaunchCfg &cfg)  // g_tuned_mu held
{
    g_tuned[key] = cfg;
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        const std::string dir = path.substr(0, slash);
        std::string acc;
        for (size_t i = 0; i <= dir.size(); ++i)
            if (i == dir.size() || (dir[i] == '/' && i > 0)) {
                acc = dir.substr(0, i);
                (void)mkdir(acc.c_str(), 0755);
            }
    }
    if (FILE *f = std::fopen(path.c_str(), "a")) {  // one short line per append
        std::fprintf(f, "%s|%d %d %d\n", key.c_str(), cfg.kt, cfg.bs, cfg.chunk);
        std::fclose(f);
    }
}

// Least relative gain over the current launch that a candidate must show to
// replace it: timed on a prefix of the runs, or on whole runs (there only
// run-to-run noise, a few tenths of a percent, has to be outweighed).
constexpr float kTuneMargin = 0.03f;
constexpr float kTuneMarginWhole = 0.01f;

// Steps of the whole-run prefix each candidate is timed on: CT_TUNE_STEPS,
// else enough for about 6e11 pair evaluations at the first step's pair
// count, between 2 and 1000.

int64_t tune_steps(const BatchShape &s)
{
    const char *v = std::getenv("CT_TUNE_STEPS");
    const long long k = v ? std::atoll(v) : 0;
    if (k >= 1) return (int64_t)k;
    double pairs = 0.0;
    for (int32_t n : s.n) pairs += (double)n * (double)n;
    // about 6e11 pair evaluations (a second or two on this GPU): whole runs
    // of batches of small events, 10-40 steps of the large ones
    const double steps = pairs > 0.0 ? 6e11 / pairs : 1000.0;
    return (int64_t)std::max(2.0, std::min(1000.0, std::floor(steps)));
}

// Time the first tune_steps() steps of the seeded batch under each candidate
// launch (the persistent kernel only, HIP events; the best of three runs,
// each from the freshly seeded state) and keep the fastest.  Every candidate
// runs the same steps of the same events, so the fastest prefix is the one
// with the highest pair rate.  The fastest must beat the context's current
// launch by kTuneMarginWhole when the timed steps finished the batch, by
// kTuneMargin when they did not: a prefix does not rank launches whose
// whole runs differ by less than that (a 60 keV batch's first steps favour
// shorter chunks that lose over the whole run).  Near-ties keep the default.  Candidates keep Newton pairs
// where the context uses them (FP32, repulsion, CT_OPT_ONE_SIDED unset): one
// target per thread, blocks of 256, chunks of 1 to 15 tiles, each distinct
// split of the batch timed once.  The state is the seeded one afterwards.
ct_status autotune(ct_ctx *c)
{
    const bool newton = resolve_cfg(c, ct::LaunchCfg{1, ct::kSymTile, ct::kSymTile}).newton != 0;
    char key[256];
    std::snprintf(key, sizeof key, "%s cu%d p%d f%u o%u B%d n%d N%d", c->arch.c_str(), c->cu_count,
                  (int)c->p.precision, (unsigned)c->p.physics_flags,
                  (unsigned)(c->p.options & CT_OPT_ONE_SIDED), log2_bucket(c->shape.B),
                  log2_bucket(c->shape.n_max), log2_bucket(c->shape.N));
    ct::LaunchCfg best = c->cfg;
    bool cached = false;
    {
        std::lock_guard<std::mutex> lk(g_tuned_mu);
        load_tune_cache();
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            best = it->second;
            cached = true;
        }
    }
    ct_status st;
    if (!cached) {
        std::vector<ct::LaunchCfg> cand;
        // Newton chunks of P tiles or more, P the most tiles a tile of the
        // largest event meets, all give one item per tile and step: the same
        // split, timed once (as the shortest of them)
        const int T = (c->shape.n_max + ct::kSymTile - 1) / ct::kSymTile;
        const int P = T <= ct::kSymMaxTiles ? T / 2 + 1 : 1 << 30;
        auto split_of = [&](int chunk) { return std::min(chunk / ct::kSymTile, P); };
        if (newton) {
            for (int chunk : {256, 512, 768, 1024, 1280, 1792, 2304, 3840})
                if (cand.empty() || split_of(chunk) != split_of(cand.back().chunk))
                    cand.push_back(ct::LaunchCfg{1, ct::kSymTile, chunk});
        } else {
            cand = {{1, 256, 512}, {1, 256, 768}, {1, 256, 1280}, {1, 256, 2304},
                    {2, 256, 1280}, {1, 128, 256}, {1, 128, 512}};
        }
        const int64_t K = tune_steps(c->shape);
        float best_ms = 1e30f, current_ms = 1e30f;
        const ct::LaunchCfg current = best;
        bool whole_runs = true;  // every timed prefix finished the batch
        for (const ct::LaunchCfg &cfg : cand) {
            st = prepare_queue(c, cfg);
            if (st != CT_OK) return st;
            float ms_min = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                st = reset_state(c);
                if (st != CT_OK) return st;
                if (c->n_active == 0) break;
                CT_HIP(ct::launch_fill_i32((int32_t *)c->bt.call_steps, 2 * c->shape.B, 0, c->stream));
                const double before = c->field_ms;
                for (;;) {  // the prefix, including any parked events
                    st = run_once(c, cfg, K, 0, nullptr, true);
                    if (st != CT_OK) return st;
                    if (!c->h_sched->exhausted.v) break;
                }
                ms_min = std::min(ms_min, (float)(c->field_ms - before));
            }
            if (c->h_sched->active != 0) whole_runs = false;
            if (cfg.kt == current.kt && cfg.bs == current.bs &&
                (newton ? split_of(cfg.chunk) == split_of(current.chunk) : cfg.chunk == current.chunk))
                current_ms = ms_min;
            if (ms_min < best_ms) {
                best_ms = ms_min;
                best = cfg;
            }
        }
        if (best_ms > (1.0f - (whole_runs ? kTuneMarginWhole : kTuneMargin)) * current_ms)
            best = current;
        if (newton && best.kt == current.kt && best.bs == current.bs &&
            split_of(best.chunk) == split_of(current.chunk))
            best = current;  // the same split: keep the context's own launch
        std::lock_guard<std::mutex> lk(g_tuned_mu);
        store_tune_cache(key, best);
    }
    st = prepare_queue(c, best);
    if (st != CT_OK) return st;
    c->cfg = best;
    return reset_state(c);
}

}  // namespace

extern "C" {

const char *ct_last_error(void) { return g_err.c_str(); }

ct_status ct_event_carriers(const ct_sensor_params *p, const ct_event_desc *ev, int32_t n_events,
                            int32_t *n_out)
{
    ct_status st = check_params(p);
    if (st != CT_OK) return st;
    BatchShape s;
    st = shape_of(*p, ev, n_events, s);
    if (st != CT_OK) return st;
    if (n_events > 0 && !n_out) return fail(CT_EINVAL, "n_out is NULL");
    for (int32_t b = 0; b < n_events; ++b) n_out[b] = s.n[b];
    return CT_OK;
}

size_t ct_workspace_bytes(const ct_sensor_params *p, const ct_event_desc *ev, int32_t n_events)
{
    if (check_params(p) != CT_OK) return 0;
    BatchShape s;
    if (shape_of(*p, ev, n_events, s) != CT_OK) return 0;
    return make_layout(s.B, s.N, s.n_dep, s.n_exp, p->grid_n * p->grid_n + 1,
                       (p->physics_flags & CT_SPHERICAL) != 0)
        .total;
}

ct_status ct_init_sensor(const ct_sensor_params *p, ct_ctx **out)
{
    if (!out) return fail(CT_EINVAL, "out is NULL");
    *out = nullptr;
    ct_status st = check_params(p);
    if (st != CT_OK) return st;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return fail(CT_EDEVICE, "no HIP device");
    }
    int dev = p->device;
    if (dev < 0) {
        if (hipGetDevice(&dev) != hipSuccess) return fail(CT_EDEVICE, "hipGetDevice failed");
    }
    if (dev >= count) return fail(CT_EINVAL, "device %d out of range (%d devices)", dev, count);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(CT_EDEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(CT_EDEVICE, "device %d is %s; this library is built for gfx950", dev,
                    prop.gcnArchName);
    ct_ctx *c = new (std::nothrow) ct_ctx();
    if (!c) return fail(CT_ENOMEM, "host allocation failed");
    c->p = *p;
    c->dp = make_dev_params(*p);
    c->device = dev;
    c->cfg = default_cfg(*p);
    c->cu_count = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    auto bail = [&](ct_status s2) {
        ct_destroy(c);
        return s2;
    };
    if (hipSetDevice(dev) != hipSuccess) return bail(fail(CT_EDEVICE, "hipSetDevice failed"));
    if (p->hip_stream) {
        c->stream = (hipStream_t)p->hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(CT_EDEVICE, "hipStreamCreate failed"));
        c->own_stream = true;
    }
    if (hipEventCreate(&c->ev_a) != hipSuccess || hipEventCreate(&c->ev_b) != hipSuccess)
        return bail(fail(CT_EDEVICE, "hipEventCreate failed"));
    if (hipHostMalloc((void **)&c->h_sched, sizeof(ct::Sched), hipHostMallocDefault) != hipSuccess)
        return bail(fail(CT_EDEVICE, "hipHostMalloc failed"));
    *out = c;
    return CT_OK;
}

ct_status ct_bind_workspace(ct_ctx *c, void *device_ptr, size_t bytes)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    if (device_ptr && ((uintptr_t)device_ptr & 255u))
        return fail(CT_EINVAL, "workspace must be 256-byte aligned");
    if (c->seeded && c->ws_bound && device_ptr != c->ws) c->seeded = false;  // batch lived there
    c->bound_ptr = device_ptr;
    c->bound_bytes = device_ptr ? bytes : 0;
    return CT_OK;
}

ct_status ct_set_launch(ct_ctx *c, int32_t kt, int32_t bs, int32_t chunk_len)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    if (c->broken) return fail(CT_EDEVICE, "context unusable after a device error");
    ct::LaunchCfg n = c->cfg;
    if (kt) n.kt = kt;
    if (bs) n.bs = bs;
    if (chunk_len) n.chunk = chunk_len;
    if (!ct::launch_supported(n.kt, n.bs))
        return fail(CT_EINVAL, "unsupported launch (targets/thread %d, block %d)", n.kt, n.bs);
    if (!chunk_len && n.chunk % n.bs) n.chunk = (n.chunk + n.bs - 1) / n.bs * n.bs;
    if (n.chunk < n.bs || n.chunk > (1 << 20) || n.chunk % n.bs)
        return fail(CT_EINVAL, "chunk_len %d must be a multiple of the block size %d, at most 2^20",
                    n.chunk, n.bs);
    if (c->seeded) {
        ct_status st = check_scratch(c);
        if (st != CT_OK) return st;
        st = set_device(c);
        if (st != CT_OK) return st;
        st = prepare_queue(c, n);
        if (st != CT_OK) return st;
    }
    c->cfg = n;
    return CT_OK;
}

}  // extern "C"

namespace {

// The work queue of a batch of this shape fits the device's scratch (at the
// smallest ticket count that still holds one step of every event).
ct_status scratch_fits(ct_ctx *c, const BatchShape &s)
{
    void *mem = nullptr;
    size_t bytes = 0;
    CT_HIP(ct::scratch_memory(c->device, &mem, &bytes));
    const bool spherical = (c->p.physics_flags & CT_SPHERICAL) != 0;
    int sph_cap = 0;
    if (spherical) {
        const int occ = ct::sph_occupancy();
        if (occ <= 0) return fail(CT_EDEVICE, "spherical kernel occupancy query failed");
        sph_cap = occ * c->cu_count;
    }
    const QueueLayout Q = make_queue_layout(s, resolve_cfg(c, c->cfg),
                                            (c->p.physics_flags & CT_REPULSION) != 0, spherical,
                                            sph_cap, 1);
    if (Q.total > bytes)
        return fail(CT_ENOMEM, "the batch's work queue needs %zu bytes; the scratch of "
                               "ct_seed_events_noalloc has %zu", Q.total, bytes);
    return CT_OK;
}

// The state seeding leaves, rebuilt from the event descriptions already on
// the device: per-event counters, the initial clouds (k_seed) and their
// compaction.  Synchronises the context's stream.
ct_status reset_state(ct_ctx *c)
{
    const BatchShape &s = c->shape;
    const ct::DevBatch &bt = c->bt;
    const int G1 = c->p.grid_n * c->p.grid_n + 1;
    hipStream_t sm = c->stream;
    auto up = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, sm);
    };
    std::vector<double> ref(4 * s.B, 0.0);
    std::vector<int64_t> zeros64(s.B, 0);
    CT_HIP(up(bt.n_act, s.n.data(), sizeof(int32_t) * s.B));
    CT_HIP(up(bt.n_hole, s.nh.data(), sizeof(int32_t) * s.B));
    CT_HIP(up(bt.ev_step, c->start_h.data(), sizeof(int64_t) * s.B));
    CT_HIP(up(bt.ev_taken, zeros64.data(), sizeof(int64_t) * s.B));
    CT_HIP(up(bt.call_steps, zeros64.data(), sizeof(int64_t) * s.B));
    CT_HIP(up(bt.ref, ref.data(), sizeof(double) * 4 * s.B));
    CT_HIP(up(bt.pairs, zeros64.data(), sizeof(uint64_t) * s.B));
    CT_HIP(up(bt.hsteps, zeros64.data(), sizeof(uint64_t) * s.B));
    CT_HIP(ct::launch_fill_i32(bt.pix, s.B * G1, 0, sm));
    CT_HIP(ct::launch_seed(c->dp, bt, sm));
    CT_HIP(ct::launch_compact(c->dp, bt, sm));
    CT_HIP(ct::launch_summary(bt, c->dq.sc, sm));
    CT_HIP(hipMemcpyAsync(c->h_sched, c->dq.sc, sizeof(ct::Sched), hipMemcpyDeviceToHost, sm));
    CT_HIP(hipStreamSynchronize(sm));
    c->n_active = s.B > 0 ? c->h_sched->active : 0;
    c->steps = 0;
    c->field_launches = 0;
    c->field_ms = 0.0;
    c->step_wall_ms = 0.0;
    return CT_OK;
}

// ct_seed_events and ct_seed_events_noalloc: the batch goes to the context's
// workspace (allocated, or bound by the caller), its work queue to the
// context's own allocation or, with noalloc, to the device's scratch.
ct_status seed(ct_ctx *c, const ct_event_desc *ev, int32_t n_events, uint64_t first_event_id,
               bool noalloc)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    if (c->broken) return fail(CT_EDEVICE, "context unusable after a device error");
    BatchShape s;
    ct_status st = shape_of(c->p, ev, n_events, s);
    if (st != CT_OK) return st;
    if (s.B > 65535) return fail(CT_EINVAL, "at most 65535 events per batch");
    if (noalloc) {
        if (c->p.options & CT_OPT_AUTOTUNE)
            return fail(CT_EINVAL, "ct_seed_events_noalloc does not autotune (the tuner allocates)");
        if (!c->bound_ptr)
            return fail(CT_ESTATE, "ct_seed_events_noalloc needs a workspace bound with "
                                   "ct_bind_workspace");
        if (c->ws && !c->ws_bound)
            return fail(CT_ESTATE, "the context holds a batch workspace the library allocated; "
                                   "ct_seed_events_noalloc needs a context that never allocated one");
        const size_t need = make_layout(s.B, s.N, s.n_dep, s.n_exp, c->p.grid_n * c->p.grid_n + 1,
                                        (c->p.physics_flags & CT_SPHERICAL) != 0)
                                .total;
        if (c->bound_bytes < need)
            return fail(CT_ENOMEM, "bound workspace has %zu bytes, batch needs %zu", c->bound_bytes,
                        need);
        st = set_device(c);
        if (st != CT_OK) return st;
        st = scratch_fits(c, s);
        if (st != CT_OK) return st;
        c->in_scratch = true;
        claim_scratch(c);
    } else if (c->in_scratch) {
        release_scratch(c);
        c->in_scratch = false;
    }
    // host-side staging of the event descriptions
    const int G1 = c->p.grid_n * c->p.grid_n + 1;
    std::vector<int32_t> off(s.B + 1), dep_off(s.B + 1), x_off(s.B + 1), rngid(s.N);
    std::vector<double> sigma(s.B), deps(3 * s.n_dep), xyz(3 * s.n_exp), seg_len(s.B);
    std::vector<int64_t> start(s.B);
    off[0] = dep_off[0] = x_off[0] = 0;
    for (int32_t b = 0; b < s.B; ++b) {
        const ct_event_desc &e = ev[b];
        const int32_t n = s.n[b];
        off[b + 1] = off[b] + n;
        dep_off[b + 1] = dep_off[b] + e.n_deposits;
        x_off[b + 1] = x_off[b] + (e.n_deposits == 0 ? n : 0);
        sigma[b] = e.n_deposits > 0 ? initial_sigma(e) : 0.0;
        start[b] = e.start_step;
        seg_len[b] = e.seg_len_um;
        // a track lists its start only; the device fills its deposit slots
        const int32_t given = e.seg_len_um > 0.0 ? 3 : 3 * e.n_deposits;
        for (int32_t d = 0; d < given; ++d) {
            if (!std::isfinite(e.deposits[d]))
                return fail(CT_ENONFINITE, "event %d: deposit not finite", b);
            deps[3 * (size_t)dep_off[b] + d] = e.deposits[d];
        }
        if (e.n_deposits == 0) {
            for (int64_t d = 0; d < 3 * (int64_t)n; ++d) {
                const double v = e.xyz[d];
                if (!std::isfinite(v))
                    return fail(CT_ENONFINITE, "event %d carrier %lld: position not finite", b,
                                (long long)(d / 3));
                xyz[3 * (size_t)x_off[b] + d] = v;
            }
        }
        const int32_t nh = s.nh[b];
        for (int32_t k = 0; k < n; ++k) rngid[off[b] + k] = e.ids ? e.ids[k] : (k < nh ? k : k - nh);
    }
    st = set_device(c);
    if (st != CT_OK) return st;
    const Layout L = make_layout(s.B, s.N, s.n_dep, s.n_exp, G1, (c->p.physics_flags & CT_SPHERICAL) != 0);
    c->seeded = false;
    st = ensure_workspace(c, L.total);
    if (st != CT_OK) return st;
    void *w = c->ws;
    ct::DevBatch bt{};
    bt.n_events = (int32_t)s.B;
    bt.n_total = (int32_t)s.N;
    bt.first_event_id = first_event_id;
    bt.off = at<int32_t>(w, L.off);
    bt.n_act = at<int32_t>(w, L.n_act);
    bt.n_hole = at<int32_t>(w, L.n_hole);
    bt.nh0 = at<int32_t>(w, L.nh0);
    bt.ev_step = at<int64_t>(w, L.ev_step);
    bt.ev_taken = at<int64_t>(w, L.ev_taken);
    bt.call_steps = at<int64_t>(w, L.call_steps);
    bt.ref = at<double>(w, L.ref);
    double *pos = at<double>(w, L.pos);
    bt.cx = pos;
    bt.cy = pos + s.N;
    bt.cz = pos + 2 * s.N;
    bt.nx = pos + 3 * s.N;
    bt.ny = pos + 4 * s.N;
    bt.nz = pos + 5 * s.N;
    bt.idx = at<int32_t>(w, L.idx);
    bt.nidx = at<int32_t>(w, L.nidx);
    bt.rngid = at<int32_t>(w, L.rngid);
    bt.out_xyz = at<double>(w, L.out_xyz);
    bt.out_cstep = at<int32_t>(w, L.out_cstep);
    bt.pix = at<int32_t>(w, L.pix);
    bt.pairs = at<uint64_t>(w, L.pairs);
    bt.hsteps = at<uint64_t>(w, L.hsteps);
    bt.sigma = at<double>(w, L.sigma);
    bt.dep_off = at<int32_t>(w, L.dep_off);
    bt.deposits = at<double>(w, L.deposits);
    bt.x_off = at<int32_t>(w, L.x_off);
    bt.xyz_in = at<double>(w, L.xyz_in);
    bt.start = at<int64_t>(w, L.start);
    c->bt = bt;
    c->L = L;
    c->shape = s;
    st = prepare_queue(c, c->cfg);
    if (st != CT_OK) return st;

    hipStream_t sm = c->stream;
    auto up = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, sm);
    };
    // the event descriptions, once; then the state every seeding starts from
    CT_HIP(up((void *)bt.off, off.data(), sizeof(int32_t) * (s.B + 1)));
    CT_HIP(up((void *)bt.nh0, s.nh.data(), sizeof(int32_t) * s.B));
    CT_HIP(up((void *)bt.rngid, rngid.data(), sizeof(int32_t) * s.N));
    CT_HIP(up((void *)bt.sigma, sigma.data(), sizeof(double) * s.B));
    CT_HIP(up((void *)bt.dep_off, dep_off.data(), sizeof(int32_t) * (s.B + 1)));
    CT_HIP(up((void *)bt.deposits, deps.data(), sizeof(double) * deps.size()));
    CT_HIP(up((void *)bt.x_off, x_off.data(), sizeof(int32_t) * (s.B + 1)));
    CT_HIP(up((void *)bt.xyz_in, xyz.data(), sizeof(double) * xyz.size()));
    CT_HIP(up((void *)bt.start, start.data(), sizeof(int64_t) * s.B));
    if (s.tracks) {
        double *seg = at<double>(w, L.seg_len);
        CT_HIP(up(seg, seg_len.data(), sizeof(double) * s.B));
        CT_HIP(ct::launch_track(c->dp, (int32_t)s.B, first_event_id, bt.dep_off, seg,
                                const_cast<double *>(bt.deposits), sm));
    }
    c->start_h = start;
    st = reset_state(c);  // synchronises the stream (the host vectors may go)
    if (st != CT_OK) return st;
    c->seeded = true;
    if (!noalloc && (c->p.options & CT_OPT_AUTOTUNE) && (c->p.physics_flags & CT_REPULSION) &&
        s.N > 0 && !spherical(c)) {
        st = autotune(c);
        if (st != CT_OK) return st;
    }
    return CT_OK;
}

}  // namespace

extern "C" {

ct_status ct_seed_events(ct_ctx *c, const ct_event_desc *ev, int32_t n_events,
                         uint64_t first_event_id)
{
    return seed(c, ev, n_events, first_event_id, false);
}

ct_status ct_seed_events_noalloc(ct_ctx *c, const ct_event_desc *ev, int32_t n_events,
                                 uint64_t first_event_id)
{
    return seed(c, ev, n_events, first_event_id, true);
}

ct_status ct_step(ct_ctx *c, int64_t max_steps, int64_t *steps_done, int64_t *n_active)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    if (c->broken) return fail(CT_EDEVICE, "context unusable after a device error");
    if (!c->seeded) return fail(CT_ESTATE, "ct_step before ct_seed_events");
    ct_status st = check_scratch(c);
    if (st != CT_OK) return st;
    st = set_device(c);
    if (st != CT_OK) return st;
    if (max_steps <= 0) max_steps = c->p.max_steps;
    const auto t_start = std::chrono::steady_clock::now();
    const bool timing = (c->p.options & CT_OPT_TIMING) != 0;
    int64_t done = 0;
    if (c->n_active > 0) {
        CT_HIP(ct::launch_fill_i32((int32_t *)c->bt.call_steps, 2 * c->shape.B, 0, c->stream));
        if (spherical(c)) {
            st = run_sph(c, max_steps, 0, nullptr, timing);
            if (st != CT_OK) return st;
        } else {
            // one run takes every event to completion or to the step cap,
            // unless the work queue filled up and some events were parked
            for (;;) {
                st = run_once(c, c->cfg, max_steps, 0, nullptr, timing);
                if (st != CT_OK) return st;
                if (!c->h_sched->exhausted.v) break;
            }
        }
        c->n_active = c->h_sched->active;
        done = c->h_sched->max_steps;
    }
    c->steps += done;
    if (steps_done) *steps_done = done;
    if (n_active) *n_active = c->n_active;
    c->step_wall_ms +=
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (c->n_active > 0)
        return fail(CT_EMAXSTEPS, "%lld holes still drifting after %lld steps",
                    (long long)c->n_active, (long long)done);
    return CT_OK;
}

ct_status ct_collect(ct_ctx *c, int32_t *pixel_counts, double *xyz, int32_t *collect_step,
                     int64_t *event_steps, ct_run_stats *stats)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    if (c->broken) return fail(CT_EDEVICE, "context unusable after a device error");
    if (!c->seeded) return fail(CT_ESTATE, "ct_collect before ct_seed_events");
    ct_status st = check_scratch(c);
    if (st != CT_OK) return st;
    st = set_device(c);
    if (st != CT_OK) return st;
    const int64_t B = c->shape.B, N = c->shape.N;
    const int G1 = c->p.grid_n * c->p.grid_n + 1;
    hipStream_t sm = c->stream;
    if (xyz) CT_HIP(ct::launch_scatter_alive(c->bt, c->shape.n_max, sm));
    if (pixel_counts && B)
        CT_HIP(hipMemcpyAsync(pixel_counts, c->bt.pix, sizeof(int32_t) * B * G1,
                              hipMemcpyDeviceToHost, sm));
    if (xyz && N)
        CT_HIP(hipMemcpyAsync(xyz, c->bt.out_xyz, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, sm));
    if (collect_step && N)
        CT_HIP(hipMemcpyAsync(collect_step, c->bt.out_cstep, sizeof(int32_t) * N,
                              hipMemcpyDeviceToHost, sm));
    if (event_steps && B)
        CT_HIP(hipMemcpyAsync(event_steps, c->bt.ev_taken, sizeof(int64_t) * B,
                              hipMemcpyDeviceToHost, sm));
    std::vector<uint64_t> pairs(B), hsteps(B);
    if (stats && B) {
        CT_HIP(hipMemcpyAsync(pairs.data(), c->bt.pairs, sizeof(uint64_t) * B,
                              hipMemcpyDeviceToHost, sm));
        CT_HIP(hipMemcpyAsync(hsteps.data(), c->bt.hsteps, sizeof(uint64_t) * B,
                              hipMemcpyDeviceToHost, sm));
    }
    CT_HIP(hipStreamSynchronize(sm));
    if (stats) {
        ct_run_stats r{};
        r.steps = c->steps;
        for (uint64_t v : pairs) r.pairs += v;
        for (uint64_t v : hsteps) r.hole_steps += v;
        r.n_total = N;
        r.n_active = c->n_active;
        r.field_launches = c->field_launches;
        r.field_kernel_ms = c->field_ms;
        r.step_wall_ms = c->step_wall_ms;
        r.targets_per_thread = spherical(c) ? 1 : c->cfg.kt;
        r.block_size = spherical(c) ? ct::kSphBlock : c->cfg.bs;
        r.chunk_len = spherical(c) ? 0 : c->cfg.chunk;
        r.workgroups = c->grid + (spherical(c) ? c->grid_shared : 0);
        r.newton_pairs = resolve_cfg(c, c->cfg).newton != 0;
        *stats = r;
    }
    return CT_OK;
}

ct_status ct_field(ct_ctx *c, double *field)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    if (c->broken) return fail(CT_EDEVICE, "context unusable after a device error");
    if (!c->seeded) return fail(CT_ESTATE, "ct_field before ct_seed_events");
    if (!field) return fail(CT_EINVAL, "field is NULL");
    ct_status st = check_scratch(c);
    if (st != CT_OK) return st;
    st = set_device(c);
    if (st != CT_OK) return st;
    const int64_t N = c->shape.N;
    if (N == 0) return CT_OK;
    st = ensure_field_buf(c, N);
    if (st != CT_OK) return st;
    st = field_into_buf(c, c->cfg, false);
    if (st != CT_OK) return st;
    CT_HIP(hipMemcpyAsync(field, c->field_buf, sizeof(double) * 3 * N, hipMemcpyDeviceToHost,
                          c->stream));
    CT_HIP(hipStreamSynchronize(c->stream));
    return CT_OK;
}

ct_status ct_philox(ct_ctx *c, const uint32_t *counters, int64_t n, uint32_t *words,
                    double *normals)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    if (n < 0 || (n > 0 && !counters)) return fail(CT_EINVAL, "bad counters");
    if (n == 0) return CT_OK;
    ct_status st = set_device(c);
    if (st != CT_OK) return st;
    uint32_t *d_ctr = nullptr, *d_w = nullptr;
    double *d_n = nullptr;
    auto cleanup = [&]() {
        if (d_ctr) (void)hipFree(d_ctr);
        if (d_w) (void)hipFree(d_w);
        if (d_n) (void)hipFree(d_n);
    };
    if (hipMalloc((void **)&d_ctr, 16 * n) != hipSuccess ||
        (words && hipMalloc((void **)&d_w, 16 * n) != hipSuccess) ||
        (normals && hipMalloc((void **)&d_n, 24 * n) != hipSuccess)) {
        cleanup();
        return fail(CT_ENOMEM, "device allocation failed");
    }
    hipError_t e = hipMemcpyAsync(d_ctr, counters, 16 * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = ct::launch_philox(c->dp, d_ctr, n, d_w, d_n, c->stream);
    if (e == hipSuccess && words)
        e = hipMemcpyAsync(words, d_w, 16 * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && normals)
        e = hipMemcpyAsync(normals, d_n, 24 * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    cleanup();
    if (e != hipSuccess) return fail(CT_EDEVICE, "philox kernel failed: %s", hipGetErrorString(e));
    return CT_OK;
}

ct_status ct_generate(ct_ctx *c, const ct_gen_params *g, int64_t n_events,
                      uint64_t first_event_id, double *energy, int32_t *counts, double *info,
                      float *kernel_ms)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    if (c->broken) return fail(CT_EDEVICE, "context unusable after a device error");
    if (!g) return fail(CT_EINVAL, "generator parameters are NULL");
    if (n_events < 0 || n_events > INT32_MAX) return fail(CT_EINVAL, "n_events out of range");
    const ct_sensor_params &p = c->p;
    if (p.grid_n > 8) return fail(CT_EINVAL, "the generator supports grids of at most 8 x 8 pixels");
    if (!(p.v_bias > p.v_dep && p.v_dep >= 0.0))
        return fail(CT_EINVAL, "the drift time (Eq. 9) needs 0 <= v_dep < v_bias");
    bool finite = std::isfinite(g->energy_kev) && std::isfinite(g->fano) &&
                  std::isfinite(g->noise_kev) && std::isfinite(g->atten_um);
    for (double v : g->p_alpha) finite = finite && std::isfinite(v);
    for (double v : g->p_beta) finite = finite && std::isfinite(v);
    if (!finite) return fail(CT_EINVAL, "generator parameters must be finite");
    if (!(g->energy_kev > 0.0) || g->fano < 0.0 || g->noise_kev < 0.0 || !(g->atten_um > 0.0))
        return fail(CT_EINVAL, "need energy_kev > 0, fano >= 0, noise_kev >= 0, atten_um > 0");
    if (!(g->p_beta[1] < 0.0)) return fail(CT_EINVAL, "p_beta[1] must be < 0 (Eq. 11 at t >= 0)");
    ct::GenDev d{};
    const double H = p.thickness_um;
    d.H = H;
    d.e_entrance = (p.v_bias - p.v_dep) / H;
    d.e_pixels = (p.v_bias + p.v_dep) / H;
    d.k = 2.0 * p.v_dep / (H * H);
    double mu0, ec, beta;
    hole_mobility_params(p, mu0, ec, beta);
    d.inv_mu0 = 1.0 / mu0;
    d.inv_ec = 1.0 / ec;
    d.atten = g->atten_um;
    d.keep = -std::expm1(-H / g->atten_um);
    d.mean_n = 1000.0 * g->energy_kev / p.pair_energy_ev;
    d.sd_n = std::sqrt(g->fano * d.mean_n);
    d.w_kev = p.pair_energy_ev / 1000.0;
    d.noise = g->noise_kev;
    d.pitch = p.pitch_um;
    for (int i = 0; i < 4; ++i) d.pa[i] = g->p_alpha[i];
    for (int i = 0; i < 5; ++i) d.pb[i] = g->p_beta[i];
    d.grid_n = p.grid_n;
    d.key0 = (uint32_t)p.seed;
    d.key1 = (uint32_t)(p.seed >> 32);
    d.first_event_id = first_event_id;
    // alpha(t) and beta(t) must be positive over every drift time that occurs
    const double t_max = d.k > 0.0
                             ? (std::log(d.e_pixels / d.e_entrance) / d.k + H * d.inv_ec) * d.inv_mu0
                             : H * (1.0 / d.e_entrance + d.inv_ec) * d.inv_mu0;
    for (int i = 0; i <= 1000; ++i) {
        const double t = t_max * i / 1000.0;
        const double a = d.pa[0] + d.pa[1] * std::sqrt(t) + d.pa[2] * t + d.pa[3] * t * t;
        const double b = 2.0 + d.pb[0] * std::pow(t - d.pb[1], d.pb[2]) + d.pb[3] * std::exp(d.pb[4] * t);
        if (!(a > 0.0) || !(b > 0.0) || !std::isfinite(a) || !std::isfinite(b))
            return fail(CT_EINVAL, "alpha(t) = %g, beta(t) = %g at t = %g ns: both must be positive "
                                   "for every drift time in [0, %g] ns", a, b, t, t_max);
    }
    if (n_events == 0) return CT_OK;
    ct_status st = set_device(c);
    if (st != CT_OK) return st;
    hipStream_t sm = c->stream;
    if (kernel_ms) CT_HIP(hipEventRecord(c->ev_a, sm));
    CT_HIP(ct::launch_gen(d, n_events, energy, counts, info, sm));
    if (kernel_ms) {
        CT_HIP(hipEventRecord(c->ev_b, sm));
        CT_HIP(hipEventSynchronize(c->ev_b));
        CT_HIP(hipEventElapsedTime(kernel_ms, c->ev_a, c->ev_b));
    }
    return CT_OK;
}

void ct_destroy(ct_ctx *c)
{
    if (!c) return;
    release_scratch(c);
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->ws && !c->ws_bound) (void)hipFree(c->ws);
    if (c->qbuf) (void)hipFree(c->qbuf);
    if (c->field_buf) (void)hipFree(c->field_buf);
    if (c->h_sched) (void)hipHostFree(c->h_sched);
    if (c->ev_a) (void)hipEventDestroy(c->ev_a);
    if (c->ev_b) (void)hipEventDestroy(c->ev_b);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"
