// Host side of the C ABI declared in include/ct.h: parameter validation,
// device workspace, batch seeding, the step loop and result collection.
// Every numerical step of the method runs in the kernels of ct_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "ct.h"
#include "ct_internal.hpp"

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
    if (p->physics_flags & ~7u) return fail(CT_EINVAL, "unknown physics flag bits");
    if ((p->physics_flags & CT_DRIFT) && !(p->v_bias > p->v_dep && p->v_dep >= 0.0))
        return fail(CT_EINVAL, "the linear drift field needs 0 <= v_dep < v_bias (Eq. 6)");
    if (p->max_steps <= 0) return fail(CT_EINVAL, "max_steps must be > 0");
    double mu0, ec, beta;
    hole_mobility_params(*p, mu0, ec, beta);
    if (!(mu0 > 0.0) || !(ec > 0.0) || !(beta > 0.0) || !std::isfinite(mu0))
        return fail(CT_EINVAL, "mobility parameters must be > 0");
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
    d.pitch = p.pitch_um;
    d.half_width = 0.5 * p.grid_n * p.pitch_um;
    d.grid_n = p.grid_n;
    d.mobility = p.mobility;
    d.flags = p.physics_flags;
    d.key0 = (uint32_t)p.seed;
    d.key1 = (uint32_t)(p.seed >> 32);
    return d;
}

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
    size_t off, n_act, ev_step, ev_taken, ref, pos, idx, rngid, out_xyz, out_cstep, pix, pairs,
        hsteps, active, item_base, n_items, counter, sigma, dep_off, deposits, x_off, xyz_in, start,
        total;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

Layout make_layout(int64_t B, int64_t N, int64_t n_dep, int64_t n_exp, int G1)
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
    L.ev_step = take(sizeof(int64_t) * B);
    L.ev_taken = take(sizeof(int64_t) * B);
    L.ref = take(sizeof(double) * 4 * B);
    L.pos = take(sizeof(double) * 6 * N);
    L.idx = take(sizeof(int32_t) * N);
    L.rngid = take(sizeof(int32_t) * N);
    L.out_xyz = take(sizeof(double) * 3 * N);
    L.out_cstep = take(sizeof(int32_t) * N);
    L.pix = take(sizeof(int32_t) * B * G1);
    L.pairs = take(sizeof(uint64_t) * B);
    L.hsteps = take(sizeof(uint64_t) * B);
    L.active = take(sizeof(int64_t));
    L.item_base = take(sizeof(int32_t) * B);
    L.n_items = take(sizeof(int32_t));
    L.counter = take(sizeof(uint32_t));
    L.sigma = take(sizeof(double) * B);
    L.dep_off = take(sizeof(int32_t) * (B + 1));
    L.deposits = take(sizeof(double) * 3 * n_dep);
    L.x_off = take(sizeof(int32_t) * (B + 1));
    L.xyz_in = take(sizeof(double) * 3 * n_exp);
    L.start = take(sizeof(int64_t) * B);
    L.total = o;
    return L;
}

struct BatchShape {
    int64_t B = 0, N = 0, n_dep = 0, n_exp = 0;
    int32_t n_max = 0;
    std::vector<int32_t> n;
};

ct_status shape_of(const ct_sensor_params &p, const ct_event_desc *ev, int32_t B, BatchShape &s)
{
    if (B < 0) return fail(CT_EINVAL, "n_events must be >= 0");
    if (B > 0 && !ev) return fail(CT_EINVAL, "events is NULL");
    s = BatchShape{};
    s.B = B;
    s.n.resize(B);
    for (int32_t b = 0; b < B; ++b) {
        const ct_event_desc &e = ev[b];
        if (e.n_deposits < 0) return fail(CT_EINVAL, "event %d: n_deposits < 0", b);
        if (e.n_deposits == 0 && e.n_carriers > 0 && !e.xyz)
            return fail(CT_EINVAL, "event %d: explicit positions missing", b);
        if (e.n_deposits > 0 && !e.deposits) return fail(CT_EINVAL, "event %d: deposits missing", b);
        if ((e.n_carriers <= 0 || e.sigma_um < 0.0) && !(e.energy_kev > 0.0) && e.n_deposits > 0)
            return fail(CT_EINVAL, "event %d: energy needed for the carrier count or width", b);
        if (e.n_deposits == 0 && e.n_carriers <= 0 && e.energy_kev != 0.0)
            return fail(CT_EINVAL, "event %d: explicit events state n_carriers", b);
        const int32_t n = carrier_count(p, e);
        if (e.n_deposits > 0 && !std::isfinite(initial_sigma(e)))
            return fail(CT_EINVAL, "event %d: width not finite", b);
        s.n[b] = n;
        s.N += n;
        s.n_max = std::max(s.n_max, n);
        s.n_dep += e.n_deposits;
        if (e.n_deposits == 0) s.n_exp += n;
    }
    if (s.N > INT32_MAX / 2) return fail(CT_EINVAL, "batch has too many carriers (%lld)", (long long)s.N);
    return CT_OK;
}

// Launch configuration of a new context (ct_set_launch overrides it).
ct::LaunchCfg default_cfg(const ct_sensor_params &p)
{
    // measured best on 256 events of 2222 holes (one target per thread,
    // 256-thread workgroups, sources split into chunks of <= 768 / 512)
    return p.precision == CT_FP32 ? ct::LaunchCfg{1, 256, 768} : ct::LaunchCfg{1, 256, 512};
}

constexpr int kGraphSteps = 16;  // steps per captured graph (and per host poll)

int default_chunks(int chunk, int32_t n_max)
{
    if (chunk <= 0 || n_max <= chunk) return 1;
    return (n_max + chunk - 1) / chunk;
}

}  // namespace

struct ct_ctx {
    ct_sensor_params p{};
    ct::DevParams dp{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    ct::LaunchCfg cfg{2, 256, 0};

    // device workspace
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_bound = false;
    void *bound_ptr = nullptr;
    size_t bound_bytes = 0;
    double *field_buf = nullptr;
    size_t field_buf_n = 0;
    double *part_buf = nullptr;  // partial fields of split events (library-owned)
    size_t part_cap = 0;         // doubles
    ct::Item *work_buf = nullptr;  // step work list (library-owned)
    size_t work_cap = 0;
    int cu_count = 0;
    int grid = 0;                // persistent step-kernel workgroups for cfg

    // captured step loop, reused while the batch layout and launch are unchanged
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    ct::DevBatch graph_bt{};
    ct::LaunchCfg graph_cfg{};
    int graph_grid = 0;

    // batch
    bool seeded = false;
    Layout L{};
    ct::DevBatch bt{};
    BatchShape shape;
    int64_t n_active = 0;
    int64_t steps = 0;

    int64_t *h_pinned = nullptr;  // [0] active count
    hipEvent_t ev_a[64] = {}, ev_b[64] = {};
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

// Partial-field buffer for events split into source chunks: [chunks][3][N].
ct_status ensure_part(ct_ctx *c, const ct::LaunchCfg &cfg, int64_t N, int32_t n_max)
{
    const int chunks = default_chunks(cfg.chunk, n_max);
    const size_t need = chunks > 1 ? (size_t)3 * N * chunks : 0;
    if (need > c->part_cap) {
        if (c->part_buf) CT_HIP(hipFree(c->part_buf));
        c->part_buf = nullptr;
        c->part_cap = 0;
        if (hipMalloc((void **)&c->part_buf, need * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CT_ENOMEM, "partial-field buffer of %zu bytes failed", need * sizeof(double));
        }
        c->part_cap = need;
    }
    c->bt.part = c->part_buf;
    c->bt.part_chunks = chunks;
    return CT_OK;
}

int64_t work_items_for(const ct::LaunchCfg &cfg, const std::vector<int32_t> &n)
{
    const int64_t T = (int64_t)cfg.bs * cfg.kt;
    int64_t items = 0;
    for (int32_t v : n)
        if (v > 0) items += ((v + T - 1) / T) * (cfg.chunk > 0 ? (v + cfg.chunk - 1) / cfg.chunk : 1);
    return items;
}

// Work-list buffer sized for the batch's initial sizes (holes only retire,
// so later steps need fewer items) and the persistent grid for cfg.
ct_status ensure_work(ct_ctx *c, const ct::LaunchCfg &cfg, const std::vector<int32_t> &n)
{
    const int64_t need = std::max<int64_t>(work_items_for(cfg, n), 1);
    if (need > INT32_MAX) return fail(CT_EINVAL, "work list too long (%lld items)", (long long)need);
    if ((size_t)need > c->work_cap) {
        if (c->work_buf) CT_HIP(hipFree(c->work_buf));
        c->work_buf = nullptr;
        c->work_cap = 0;
        if (hipMalloc((void **)&c->work_buf, need * sizeof(ct::Item)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CT_ENOMEM, "work list of %lld items failed", (long long)need);
        }
        c->work_cap = (size_t)need;
    }
    const int occ = ct::step_occupancy(cfg, c->p.precision == CT_FP32);
    if (occ <= 0) return fail(CT_EDEVICE, "step kernel occupancy query failed");
    c->grid = occ * c->cu_count;
    c->bt.work = c->work_buf;
    c->bt.work_cap = (int32_t)c->work_cap;
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

ct_status sync_active(ct_ctx *c)
{
    CT_HIP(hipMemcpyAsync(c->h_pinned, c->bt.active, sizeof(int64_t), hipMemcpyDeviceToHost,
                          c->stream));
    CT_HIP(hipStreamSynchronize(c->stream));
    c->n_active = c->h_pinned[0];
    return CT_OK;
}

ct_status drop_graph(ct_ctx *c)
{
    if (c->graph_exec) CT_HIP(hipGraphExecDestroy(c->graph_exec));
    if (c->graph) CT_HIP(hipGraphDestroy(c->graph));
    c->graph_exec = nullptr;
    c->graph = nullptr;
    return CT_OK;
}

// One time step: work list, pair kernel (+ partial-sum update), compaction.
// With timing, HIP events bracket the pair kernel (slot i of the event pool).
hipError_t issue_step(ct_ctx *c, const ct::LaunchCfg &cfg, int slot, bool timing)
{
    const int fp32 = c->p.precision == CT_FP32;
    hipError_t e = ct::launch_plan(c->bt, cfg, c->stream);
    if (e == hipSuccess && timing) e = hipEventRecord(c->ev_a[slot], c->stream);
    if (e == hipSuccess) e = ct::launch_step(c->dp, c->bt, cfg, fp32, c->grid, 0, nullptr, c->stream);
    if (e == hipSuccess && timing) e = hipEventRecord(c->ev_b[slot], c->stream);
    if (e == hipSuccess) e = ct::launch_update(c->dp, c->bt, cfg, c->shape.n_max, 0, nullptr, c->stream);
    if (e == hipSuccess) e = ct::launch_compact(c->dp, c->bt, 1, c->stream);
    return e;
}

// Capture kGraphSteps steps into one executable graph (per batch and launch
// configuration); every kernel reads its sizes from device memory, so the
// same graph serves every chunk of the run.
ct_status ensure_graph(ct_ctx *c, const ct::LaunchCfg &cfg)
{
    if (c->graph_exec && std::memcmp(&c->graph_bt, &c->bt, sizeof c->bt) == 0 &&
        c->graph_cfg.kt == cfg.kt && c->graph_cfg.bs == cfg.bs && c->graph_cfg.chunk == cfg.chunk &&
        c->graph_grid == c->grid)
        return CT_OK;
    ct_status st = drop_graph(c);
    if (st != CT_OK) return st;
    CT_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int i = 0; i < kGraphSteps && e == hipSuccess; ++i) e = issue_step(c, cfg, i, false);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(CT_EDEVICE, "step-loop capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    c->graph = g;
    CT_HIP(hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
    c->graph_bt = c->bt;
    c->graph_cfg = cfg;
    c->graph_grid = c->grid;
    return CT_OK;
}

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

// Launch configurations chosen by the autotuner, per precision and batch
// shape bucket (events, largest event, total holes; powers of two).
using TuneKey = std::tuple<int, int, int, int, int>;
std::map<TuneKey, ct::LaunchCfg> g_tuned;
std::mutex g_tuned_mu;

int log2_bucket(int64_t v)
{
    int b = 0;
    while (v > 1) {
        v >>= 1;
        ++b;
    }
    return b;
}

// Time one field evaluation of the seeded state per candidate (work list,
// persistent pair kernel, partial-sum update) and keep the fastest.  The
// state is not advanced.
ct_status autotune(ct_ctx *c)
{
    const int fp32 = c->p.precision == CT_FP32;
    const TuneKey key{fp32, c->device, log2_bucket(c->shape.B), log2_bucket(c->shape.n_max),
                      log2_bucket(c->shape.N)};
    {
        std::lock_guard<std::mutex> lk(g_tuned_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            ct::LaunchCfg best = it->second;
            ct_status st = ensure_part(c, best, c->shape.N, c->shape.n_max);
            if (st == CT_OK) st = ensure_work(c, best, c->shape.n);
            if (st == CT_OK) c->cfg = best;
            return st;
        }
    }
    ct_status st = ensure_field_buf(c, c->shape.N);
    if (st != CT_OK) return st;
    std::vector<ct::LaunchCfg> cand;
    for (int bs : {128, 256})
        for (int chunk : {0, 512, 768, 1024, 2048, 4096}) {
            if (chunk && (chunk % bs || chunk >= c->shape.n_max)) continue;
            cand.push_back(ct::LaunchCfg{1, bs, chunk});
        }
    cand.push_back(ct::LaunchCfg{2, 128, 0});
    ct::LaunchCfg best = c->cfg;
    float best_ms = 1e30f;
    for (const ct::LaunchCfg &cfg : cand) {
        st = ensure_part(c, cfg, c->shape.N, c->shape.n_max);
        if (st == CT_OK) st = ensure_work(c, cfg, c->shape.n);
        if (st != CT_OK) return st;
        float ms_min = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            CT_HIP(hipEventRecord(c->ev_a[0], c->stream));
            CT_HIP(ct::launch_plan(c->bt, cfg, c->stream));
            CT_HIP(ct::launch_step(c->dp, c->bt, cfg, fp32, c->grid, 1, c->field_buf, c->stream));
            CT_HIP(ct::launch_update(c->dp, c->bt, cfg, c->shape.n_max, 1, c->field_buf, c->stream));
            CT_HIP(hipEventRecord(c->ev_b[0], c->stream));
            CT_HIP(hipEventSynchronize(c->ev_b[0]));
            float ms = 0.0f;
            CT_HIP(hipEventElapsedTime(&ms, c->ev_a[0], c->ev_b[0]));
            if (rep > 0) ms_min = std::min(ms_min, ms);
        }
        if (ms_min < best_ms) {
            best_ms = ms_min;
            best = cfg;
        }
    }
    st = ensure_part(c, best, c->shape.N, c->shape.n_max);
    if (st == CT_OK) st = ensure_work(c, best, c->shape.n);
    if (st != CT_OK) return st;
    c->cfg = best;
    // the field pass reset the drifting-hole total on the device: restore it
    CT_HIP(hipMemcpyAsync(c->bt.active, &c->n_active, sizeof(int64_t), hipMemcpyHostToDevice,
                          c->stream));
    CT_HIP(hipStreamSynchronize(c->stream));
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    g_tuned[key] = best;
    return CT_OK;
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
    return make_layout(s.B, s.N, s.n_dep, s.n_exp, p->grid_n * p->grid_n + 1).total;
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
    if (hipHostMalloc((void **)&c->h_pinned, 64, hipHostMallocDefault) != hipSuccess)
        return bail(fail(CT_EDEVICE, "hipHostMalloc failed"));
    for (int i = 0; i < 64; ++i) {
        if (hipEventCreate(&c->ev_a[i]) != hipSuccess || hipEventCreate(&c->ev_b[i]) != hipSuccess)
            return bail(fail(CT_EDEVICE, "hipEventCreate failed"));
    }
    *out = c;
    return CT_OK;
}

ct_status ct_bind_workspace(ct_ctx *c, void *device_ptr, size_t bytes)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    if (device_ptr && ((uintptr_t)device_ptr & 255u))
        return fail(CT_EINVAL, "workspace must be 256-byte aligned");
    if (c->seeded && c->ws_bound) c->seeded = false;  // the batch lived in the old buffer
    c->bound_ptr = device_ptr;
    c->bound_bytes = device_ptr ? bytes : 0;
    return CT_OK;
}

ct_status ct_set_launch(ct_ctx *c, int32_t kt, int32_t bs, int32_t chunk)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    ct::LaunchCfg n = c->cfg;
    if (kt) n.kt = kt;
    if (bs) n.bs = bs;
    if (chunk) n.chunk = chunk < 0 ? 0 : chunk;
    if (!ct::launch_supported(n.kt, n.bs))
        return fail(CT_EINVAL, "unsupported launch (targets/thread %d, block %d)", n.kt, n.bs);
    if (n.chunk > 0 && (n.chunk < n.bs || n.chunk % n.bs))
        return fail(CT_EINVAL, "chunk_len must be a multiple of the block size");
    if (c->seeded) {
        ct_status st = set_device(c);
        if (st != CT_OK) return st;
        st = ensure_part(c, n, c->shape.N, c->shape.n_max);
        if (st != CT_OK) return st;
        st = ensure_work(c, n, c->shape.n);
        if (st != CT_OK) return st;
        st = drop_graph(c);
        if (st != CT_OK) return st;
    }
    c->cfg = n;
    return CT_OK;
}

ct_status ct_seed_events(ct_ctx *c, const ct_event_desc *ev, int32_t n_events,
                         uint64_t first_event_id)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    BatchShape s;
    ct_status st = shape_of(c->p, ev, n_events, s);
    if (st != CT_OK) return st;
    // host-side staging of the event descriptions
    const int G1 = c->p.grid_n * c->p.grid_n + 1;
    std::vector<int32_t> off(s.B + 1), dep_off(s.B + 1), x_off(s.B + 1), rngid(s.N);
    std::vector<double> sigma(s.B), deps(3 * s.n_dep), xyz(3 * s.n_exp);
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
        for (int32_t d = 0; d < 3 * e.n_deposits; ++d) deps[3 * (size_t)dep_off[b] + d] = e.deposits[d];
        if (e.n_deposits == 0) {
            for (int64_t d = 0; d < 3 * (int64_t)n; ++d) {
                const double v = e.xyz[d];
                if (!std::isfinite(v))
                    return fail(CT_ENONFINITE, "event %d carrier %lld: position not finite", b,
                                (long long)(d / 3));
                xyz[3 * (size_t)x_off[b] + d] = v;
            }
        }
        for (int32_t k = 0; k < n; ++k) rngid[off[b] + k] = e.ids ? e.ids[k] : k;
        for (int32_t d = 0; d < 3 * e.n_deposits; ++d)
            if (!std::isfinite(e.deposits[d]))
                return fail(CT_ENONFINITE, "event %d: deposit not finite", b);
    }
    st = set_device(c);
    if (st != CT_OK) return st;
    const Layout L = make_layout(s.B, s.N, s.n_dep, s.n_exp, G1);
    c->seeded = false;
    st = ensure_workspace(c, L.total);
    if (st != CT_OK) return st;
    st = ensure_part(c, c->cfg, s.N, s.n_max);
    if (st != CT_OK) return st;
    st = ensure_work(c, c->cfg, s.n);
    if (st != CT_OK) return st;
    void *w = c->ws;
    ct::DevBatch bt;
    std::memset(&bt, 0, sizeof bt);  // compared bytewise against the captured graph
    bt.n_events = (int32_t)s.B;
    bt.n_total = (int32_t)s.N;
    bt.first_event_id = first_event_id;
    bt.off = at<int32_t>(w, L.off);
    bt.n_act = at<int32_t>(w, L.n_act);
    bt.ev_step = at<int64_t>(w, L.ev_step);
    bt.ev_taken = at<int64_t>(w, L.ev_taken);
    bt.ref = at<double>(w, L.ref);
    double *pos = at<double>(w, L.pos);
    bt.cx = pos;
    bt.cy = pos + s.N;
    bt.cz = pos + 2 * s.N;
    bt.nx = pos + 3 * s.N;
    bt.ny = pos + 4 * s.N;
    bt.nz = pos + 5 * s.N;
    bt.idx = at<int32_t>(w, L.idx);
    bt.rngid = at<int32_t>(w, L.rngid);
    bt.out_xyz = at<double>(w, L.out_xyz);
    bt.out_cstep = at<int32_t>(w, L.out_cstep);
    bt.pix = at<int32_t>(w, L.pix);
    bt.pairs = at<uint64_t>(w, L.pairs);
    bt.hsteps = at<uint64_t>(w, L.hsteps);
    bt.active = at<int64_t>(w, L.active);
    bt.item_base = at<int32_t>(w, L.item_base);
    bt.n_items = at<int32_t>(w, L.n_items);
    bt.counter = at<uint32_t>(w, L.counter);
    bt.work = c->work_buf;
    bt.work_cap = (int32_t)c->work_cap;
    bt.part = c->part_buf;
    bt.part_chunks = default_chunks(c->cfg.chunk, s.n_max);
    bt.sigma = at<double>(w, L.sigma);
    bt.dep_off = at<int32_t>(w, L.dep_off);
    bt.deposits = at<double>(w, L.deposits);
    bt.x_off = at<int32_t>(w, L.x_off);
    bt.xyz_in = at<double>(w, L.xyz_in);
    bt.start = at<int64_t>(w, L.start);

    hipStream_t sm = c->stream;
    auto up = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, sm);
    };
    std::vector<int32_t> n_act(s.n);
    std::vector<double> ref(4 * s.B, 0.0);
    std::vector<int64_t> zeros64(std::max<int64_t>(s.B, 2), 0);
    CT_HIP(up((void *)bt.off, off.data(), sizeof(int32_t) * (s.B + 1)));
    CT_HIP(up(bt.n_act, n_act.data(), sizeof(int32_t) * s.B));
    CT_HIP(up(bt.ev_step, start.data(), sizeof(int64_t) * s.B));
    CT_HIP(up(bt.ev_taken, zeros64.data(), sizeof(int64_t) * s.B));
    CT_HIP(up(bt.ref, ref.data(), sizeof(double) * 4 * s.B));
    CT_HIP(up((void *)bt.rngid, rngid.data(), sizeof(int32_t) * s.N));
    CT_HIP(up(bt.pairs, zeros64.data(), sizeof(uint64_t) * s.B));
    CT_HIP(up(bt.hsteps, zeros64.data(), sizeof(uint64_t) * s.B));
    CT_HIP(up(bt.active, zeros64.data(), sizeof(int64_t)));
    CT_HIP(up((void *)bt.sigma, sigma.data(), sizeof(double) * s.B));
    CT_HIP(up((void *)bt.dep_off, dep_off.data(), sizeof(int32_t) * (s.B + 1)));
    CT_HIP(up((void *)bt.deposits, deps.data(), sizeof(double) * deps.size()));
    CT_HIP(up((void *)bt.x_off, x_off.data(), sizeof(int32_t) * (s.B + 1)));
    CT_HIP(up((void *)bt.xyz_in, xyz.data(), sizeof(double) * xyz.size()));
    CT_HIP(up((void *)bt.start, start.data(), sizeof(int64_t) * s.B));
    CT_HIP(ct::launch_fill_i32(bt.pix, s.B * G1, 0, sm));
    CT_HIP(ct::launch_seed(c->dp, bt, sm));
    CT_HIP(ct::launch_compact(c->dp, bt, 0, sm));
    c->bt = bt;
    c->L = L;
    c->shape = s;
    c->steps = 0;
    c->field_launches = 0;
    c->field_ms = 0.0;
    c->step_wall_ms = 0.0;
    st = sync_active(c);
    if (st != CT_OK) return st;
    c->seeded = true;
    if ((c->p.options & CT_OPT_AUTOTUNE) && (c->p.physics_flags & CT_REPULSION) && s.N > 0) {
        st = autotune(c);
        if (st != CT_OK) return st;
    }
    return CT_OK;
}

ct_status ct_step(ct_ctx *c, int64_t max_steps, int64_t *steps_done, int64_t *n_active)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    if (!c->seeded) return fail(CT_ESTATE, "ct_step before ct_seed_events");
    ct_status st = set_device(c);
    if (st != CT_OK) return st;
    if (max_steps <= 0) max_steps = c->p.max_steps;
    const auto t_start = std::chrono::steady_clock::now();
    const bool timing = (c->p.options & CT_OPT_TIMING) != 0;
    const bool use_graph = !(c->p.options & CT_OPT_NO_GRAPH);
    std::vector<int64_t> taken0(c->shape.B), taken1(c->shape.B);
    if (c->shape.B > 0) {
        CT_HIP(hipMemcpyAsync(taken0.data(), c->bt.ev_taken, sizeof(int64_t) * c->shape.B,
                              hipMemcpyDeviceToHost, c->stream));
        CT_HIP(hipStreamSynchronize(c->stream));
    }
    ct::LaunchCfg cfg = c->cfg;
    if (!(c->p.physics_flags & CT_REPULSION)) cfg.chunk = 0;
    int64_t issued = 0;
    while (c->n_active > 0 && issued < max_steps) {
        // one chunk: kGraphSteps captured steps, or the remainder issued eagerly;
        // steps after the last hole is collected find empty work lists
        const int k = (int)std::min<int64_t>(kGraphSteps, max_steps - issued);
        // HIP events recorded inside a graph replay carry no timestamps, so
        // timed runs issue their steps eagerly
        if (use_graph && !timing && k == kGraphSteps) {
            st = ensure_graph(c, cfg);
            if (st != CT_OK) return st;
            CT_HIP(hipGraphLaunch(c->graph_exec, c->stream));
        } else {
            for (int i = 0; i < k; ++i) CT_HIP(issue_step(c, cfg, i, timing));
        }
        issued += k;
        c->steps += k;
        st = sync_active(c);
        if (st != CT_OK) return st;
        if (timing) {
            for (int i = 0; i < k; ++i) {
                float ms = 0.0f;
                CT_HIP(hipEventElapsedTime(&ms, c->ev_a[i], c->ev_b[i]));
                c->field_ms += ms;
            }
            c->field_launches += k;
        }
    }
    if (c->shape.B > 0) {
        CT_HIP(hipMemcpyAsync(taken1.data(), c->bt.ev_taken, sizeof(int64_t) * c->shape.B,
                              hipMemcpyDeviceToHost, c->stream));
        CT_HIP(hipStreamSynchronize(c->stream));
    }
    int64_t done = 0;
    for (int64_t b = 0; b < c->shape.B; ++b) done = std::max(done, taken1[b] - taken0[b]);
    if (steps_done) *steps_done = done;
    if (n_active) *n_active = c->n_active;
    c->step_wall_ms +=
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (c->n_active > 0)
        return fail(CT_EMAXSTEPS, "%lld holes still drifting after %lld steps",
                    (long long)c->n_active, (long long)issued);
    return CT_OK;
}

ct_status ct_collect(ct_ctx *c, int32_t *pixel_counts, double *xyz, int32_t *collect_step,
                     int64_t *event_steps, ct_run_stats *stats)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    if (!c->seeded) return fail(CT_ESTATE, "ct_collect before ct_seed_events");
    ct_status st = set_device(c);
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
        r.targets_per_thread = c->cfg.kt;
        r.block_size = c->cfg.bs;
        r.chunk_len = c->cfg.chunk;
        *stats = r;
    }
    return CT_OK;
}

ct_status ct_field(ct_ctx *c, double *field)
{
    if (!c) return fail(CT_EINVAL, "ctx is NULL");
    if (!c->seeded) return fail(CT_ESTATE, "ct_field before ct_seed_events");
    if (!field) return fail(CT_EINVAL, "field is NULL");
    ct_status st = set_device(c);
    if (st != CT_OK) return st;
    const int64_t N = c->shape.N;
    if (N == 0) return CT_OK;
    st = ensure_field_buf(c, N);
    if (st != CT_OK) return st;
    // NaN everywhere, then the drifting carriers' fields
    CT_HIP(ct::launch_fill_i32((int32_t *)c->field_buf, 6 * N, (int32_t)0xFFFFFFFF, c->stream));
    ct::LaunchCfg cfg = c->cfg;
    if (!(c->p.physics_flags & CT_REPULSION)) cfg.chunk = 0;
    const int fp32 = c->p.precision == CT_FP32;
    CT_HIP(ct::launch_plan(c->bt, cfg, c->stream));
    CT_HIP(ct::launch_step(c->dp, c->bt, cfg, fp32, c->grid, 1, c->field_buf, c->stream));
    CT_HIP(ct::launch_update(c->dp, c->bt, cfg, c->shape.n_max, 1, c->field_buf, c->stream));
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

void ct_destroy(ct_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->ws && !c->ws_bound) (void)hipFree(c->ws);
    if (c->field_buf) (void)hipFree(c->field_buf);
    if (c->part_buf) (void)hipFree(c->part_buf);
    if (c->work_buf) (void)hipFree(c->work_buf);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    for (int i = 0; i < 64; ++i) {
        if (c->ev_a[i]) (void)hipEventDestroy(c->ev_a[i]);
        if (c->ev_b[i]) (void)hipEventDestroy(c->ev_b[i]);
    }
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"
