/*
 * FP64 CPU oracle of the brute-force charge-transport Monte Carlo of
 * Xie et al., "Optimization and validation of charge transport simulation
 * for hybrid pixel detectors incorporating the repulsion effect"
 * (arXiv:2506.09712): the comprehensive method of Sec. 2.1, Eqs. 2-6, as
 * laid out in Appendix A, Algorithm 1.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP library is checked against.  It shares no code, header or constant
 * table with the library; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  The product path never calls
 * it.
 *
 * Conventions (units: micrometre, nanosecond, volt, kelvin):
 *  - z is the distance from the pixel (collecting) plane; the paper's z
 *    (measured from the entrance side, Eq. 6 and the limits of Eq. 9) is
 *    H - z here.  Holes drift towards z = 0 and are collected once an update
 *    leaves them at z <= 0.  An update that crosses the entrance side z = H
 *    is mirrored back (z -> 2H - z).
 *  - Repulsion field (Eq. 4):
 *        E_i = K * sum_{j != i, alive} q_j (r_i - r_j) / (|r_i - r_j|^2 + s^2)^(3/2)
 *    with q_j = +1 for holes and -1 for electrons, K = e / (4 pi eps0 eps_r)
 *    and Plummer softening s (s = 0 is Eq. 4 exactly).  Eq. 4 prints
 *    q_i q_j, which is a force: the field at carrier i is the sum of
 *    q_j r_ij / (4 pi eps0 eps_r r^3), and carrier i moves along q_i times
 *    it (holes along the field, electrons against it), which makes like
 *    charges repel and opposite charges attract (Sec. 2.1 and its footnote).
 *  - Two species (optional, physics bit 3): besides its holes, an event
 *    simulates electrons (Sec. 2.1 follows every electron and every hole as
 *    a carrier of its own).  Electron k of a cloud event starts at
 *    the position of hole k (the pair is created at one point).  Electrons
 *    drift away from the pixel plane with the Jacoboni-Canali electron laws,
 *    are collected at the entrance side (an update that leaves them at
 *    z >= H) and mirrored at the pixel plane (z -> -z); they are not counted
 *    in pixels.  An event ends when its last hole is collected (Algorithm 1's
 *    loop ends when every hole has reached the readout electrode); electrons
 *    still drifting then keep their current position.
 *  - Simplified spherical model (optional, physics bit 4; Sec. 2.2, Eq. 7):
 *    the repulsion field at hole i is that of the holes strictly closer to
 *    the cloud centre c than i, as if concentrated at c:
 *        E_i = K Q_i (r_i - c) / (|r_i - c|^2 + s^2)^(3/2),
 *        Q_i = #{ j drifting : |r_j - c|^2 < |r_i - c|^2 },
 *    with c the mean position of the drifting holes at the step start; a
 *    hole at the same distance as i does not count, and Q_i = 0 gives
 *    E_i = 0.  Holes only (the model updates hole coordinates only).
 *  - Drift field (Eq. 6, rewritten for this z axis):
 *        E_z(z) = -[(Vb + Vd)/H - 2 Vd z / H^2]
 *  - Mobility: Caughey-Thomas form mu = mu0 / (1 + (E/Ec)^beta)^(1/beta)
 *    evaluated at |E_drift + E_rep| (Sec. 2.1, Algorithm 1), with the
 *    Jacoboni-Canali temperature laws for mu0 = vm/Ec, Ec and beta of each
 *    species.
 *  - Diffusion: D = mu k T / e (Einstein relation, Eq. 1); each axis moves
 *    by sqrt(2 D dt) times a standard normal draw (Eqs. 3 and 5).
 *  - Update order: every alive carrier is moved from the same snapshot of
 *    the step-start positions (the field loop of Algorithm 1 runs before the
 *    per-carrier update loop).
 *  - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *    key = (seed low 32 bits, seed high 32 bits), counter =
 *    (carrier id, step, event id, domain); domain 0 = hole diffusion at a
 *    step, domain 1 = initial cloud, domain 4 = electron diffusion at a step.  Uniforms (w + 0.5) 2^-32, Box-Muller
 *    normals: n0, n1 from (u0, u1), n2 from (u2, u3).
 *  - Tracks (an event with seg_len_um > 0): the deposits are the midpoints
 *    of a walk of n_deposits straight segments of length seg_len_um that
 *    starts at the given point; the first segment points along -z (into
 *    the sensor from the entrance side), each later segment k along an
 *    isotropic unit vector from the Philox block of counter
 *    (k, 0, event id, 3): cos(theta) = 1 - 2 u0, phi = 2 pi u1.  Walk points
 *    and midpoints are folded back into [0, H] (mirror at either face).  The
 *    paper has no track model; this is the reading of its deposit-based
 *    seeding for an extended track.
 *  - Pixel integration: a grid_n x grid_n array of square pixels of side
 *    pitch centred on (0, 0); bin index floor((x + grid_n pitch / 2) / pitch)
 *    per axis; carriers outside the grid go to one overflow bin.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- types */

typedef struct {
    double thickness_um, v_bias, v_dep, temperature_k;
    double pitch_um;
    int32_t grid_n;
    double dt_ns, softening_um, eps_r, pair_energy_ev;
    int32_t mobility; /* 0 = Caughey-Thomas with Jacoboni-Canali laws, 1 = constant mu0 */
    double mu0_override, ec_override, beta_override; /* holes; NaN = model value at T */
    uint32_t physics; /* bit 0 repulsion, bit 1 drift, bit 2 diffusion, bit 3 electrons */
    uint64_t seed;
    int64_t max_steps;
    double mu0_e_override, ec_e_override, beta_e_override; /* electrons; NaN = model value */
} oc_params;

typedef struct {
    double energy_kev;
    int32_t n_carriers; /* <= 0: round(1000 E / w) */
    int32_t n_deposits; /* 0: explicit positions */
    double sigma_um;    /* < 0: Eq. 2 */
    const double *deposits; /* [n_deposits][3] */
    const double *xyz;      /* [n_carriers][3] when n_deposits == 0 */
    const int32_t *ids;     /* optional carrier ids for the RNG counter (default: index
                               within the species) */
    int64_t start_step;
    int32_t n_electrons;    /* with electrons: < 0 = one per hole; explicit events list the
                               electrons' positions (and ids) after the holes' */
    double seg_len_um;      /* > 0: a track of n_deposits segments starting at deposits[0] */
} oc_event;

enum { OC_OK = 0, OC_EINVAL = -1, OC_EMAXSTEPS = -5, OC_ENONFINITE = -6 };
enum { OC_REPULSION = 1u, OC_DRIFT = 2u, OC_DIFFUSION = 4u, OC_ELECTRONS = 8u, OC_SPHERICAL = 16u };

/* SI exact values (e, k) and CODATA 2022 vacuum permittivity */
static const double E_CHARGE = 1.602176634e-19; /* C */
static const double K_BOLTZ = 1.380649e-23;     /* J/K */
static const double EPS0 = 8.8541878188e-12;    /* F/m */
static const double PI = 3.14159265358979323846;

/* --------------------------------------------------------------- Philox */

/* One Philox4x32 round: two 32x32->64 multiplications whose high halves are
 * mixed with the other two words and the round key (SC'11, Sec. 4.2). */
static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void oc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { /* Weyl key schedule: golden ratio and sqrt(3)-1 */
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

static double to_unit(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* Three independent standard normals from one Philox block (Box-Muller). */
void oc_normals3(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, double n[3])
{
    const uint32_t ctr[4] = {c0, c1, c2, c3};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oc_philox4x32_10(ctr, key, w);
    const double u0 = to_unit(w[0]), u1 = to_unit(w[1]);
    const double u2 = to_unit(w[2]), u3 = to_unit(w[3]);
    const double ra = sqrt(-2.0 * log(u0));
    const double rb = sqrt(-2.0 * log(u2));
    n[0] = ra * cos(2.0 * PI * u1);
    n[1] = ra * sin(2.0 * PI * u1);
    n[2] = rb * cos(2.0 * PI * u3);
}

/* Philox blocks for n counters ([n][4] in, [n][4] out) under a 64-bit seed. */
void oc_philox_many(uint64_t seed, int64_t n, const uint32_t *ctr, uint32_t *out)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < n; ++i) oc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* Box-Muller normals for n counters ([n][4] in, [n][3] out). */
void oc_normals_many(uint64_t seed, int64_t n, const uint32_t *ctr, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        oc_normals3(seed, ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], out + 3 * i);
}

/* ------------------------------------------------------------- physics */

/* e / (4 pi eps0 eps_r) in V um: field of one elementary charge is K / r^2. */
double oc_coulomb_k(const oc_params *p) { return E_CHARGE / (4.0 * PI * EPS0 * p->eps_r) * 1e6; }

/* k T / e in volts. */
double oc_thermal_voltage(const oc_params *p) { return K_BOLTZ * p->temperature_k / E_CHARGE; }

/* Mobility-model parameters at temperature T: mu0 [um^2/(V ns)], Ec [V/um],
 * beta, for holes (electron = 0) or electrons (electron = 1).
 * Jacoboni-Canali laws (Solid-State Electron. 20 (1977) 77), with mu0 = vm/Ec:
 *   holes:     vm = 1.62e8 T^-0.52 cm/s, Ec = 1.24 T^1.68 V/cm, beta = 0.46 T^0.17
 *   electrons: vm = 1.53e9 T^-0.87 cm/s, Ec = 1.01 T^1.55 V/cm, beta = 2.57e-2 T^0.66 */
void oc_mobility_params_of(const oc_params *p, int electron, double out[3])
{
    const double T = p->temperature_k;
    double vm, ec, beta;
    if (electron) {
        vm = 1.53e9 * pow(T, -0.87) * 1e-5; /* cm/s -> um/ns */
        ec = 1.01 * pow(T, 1.55) * 1e-4;    /* V/cm -> V/um */
        beta = 2.57e-2 * pow(T, 0.66);
    } else {
        vm = 1.62e8 * pow(T, -0.52) * 1e-5;
        ec = 1.24 * pow(T, 1.68) * 1e-4;
        beta = 0.46 * pow(T, 0.17);
    }
    double mu0 = vm / ec;
    const double o_mu0 = electron ? p->mu0_e_override : p->mu0_override;
    const double o_ec = electron ? p->ec_e_override : p->ec_override;
    const double o_beta = electron ? p->beta_e_override : p->beta_override;
    if (!isnan(o_mu0)) mu0 = o_mu0;
    if (!isnan(o_ec)) ec = o_ec;
    if (!isnan(o_beta)) beta = o_beta;
    out[0] = mu0;
    out[1] = ec;
    out[2] = beta;
}

void oc_mobility_params(const oc_params *p, double out[3]) { oc_mobility_params_of(p, 0, out); }

double oc_mobility_of(const oc_params *p, int electron, double e_mag)
{
    double m[3];
    oc_mobility_params_of(p, electron, m);
    if (p->mobility == 1) return m[0];
    return m[0] / pow(1.0 + pow(e_mag / m[1], m[2]), 1.0 / m[2]);
}

double oc_mobility(const oc_params *p, double e_mag) { return oc_mobility_of(p, 0, e_mag); }

/* Eq. 6 along the z axis used here (negative: towards the pixel plane). */
double oc_drift_field(const oc_params *p, double z)
{
    if (!(p->physics & OC_DRIFT)) return 0.0;
    const double H = p->thickness_um;
    return -((p->v_bias + p->v_dep) / H - 2.0 * p->v_dep * z / (H * H));
}

/* Eq. 4 field on carrier a from the n carriers in (x, y, z) with charges q
 * (+1 hole, -1 electron; NULL = all holes), skipping a. */
static void repulsion_one(const oc_params *p, int64_t n, const double *x, const double *y,
                          const double *z, const double *q, int64_t a, double K, double E[3])
{
    const double s2 = p->softening_um * p->softening_um;
    double ex = 0.0, ey = 0.0, ez = 0.0;
    for (int64_t b = 0; b < n; ++b) {
        if (b == a) continue;
        const double dx = x[a] - x[b], dy = y[a] - y[b], dz = z[a] - z[b];
        const double r2 = dx * dx + dy * dy + dz * dz + s2;
        const double inv_r3 = (q ? q[b] : 1.0) / (r2 * sqrt(r2));
        ex += dx * inv_r3;
        ey += dy * inv_r3;
        ez += dz * inv_r3;
    }
    E[0] = K * ex;
    E[1] = K * ey;
    E[2] = K * ez;
}

/* Field of n carriers with charges q (+1 / -1; NULL = all holes) on each
 * other ([n][3] in, [n][3] out). */
void oc_field_q(const oc_params *p, int64_t n, const double *xyz, const double *q, double *E)
{
    double *x = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *y = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *z = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        x[i] = xyz[3 * i];
        y[i] = xyz[3 * i + 1];
        z[i] = xyz[3 * i + 2];
    }
    const double K = oc_coulomb_k(p);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) repulsion_one(p, n, x, y, z, q, i, K, E + 3 * i);
    free(x);
    free(y);
    free(z);
}

/* Repulsion field of n holes on each other ([n][3] in, [n][3] out). */
void oc_field(const oc_params *p, int64_t n, const double *xyz, double *E)
{
    oc_field_q(p, n, xyz, NULL, E);
}

static int cmp_double(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Eq. 7 field of n holes at (x, y, z) on each other (E* [n]).  The centre
 * is the mean position; Q_i, the number of holes strictly closer to it than
 * hole i, is the lower-bound position of i's squared distance in the sorted
 * list of all squared distances. */
static void spherical_field(const oc_params *p, int64_t n, const double *x, const double *y,
                            const double *z, double *Ex, double *Ey, double *Ez)
{
    if (n <= 0) return;
    const double K = oc_coulomb_k(p);
    const double s2 = p->softening_um * p->softening_um;
    double cx = 0.0, cy = 0.0, cz = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        cx += x[i];
        cy += y[i];
        cz += z[i];
    }
    cx /= (double)n;
    cy /= (double)n;
    cz /= (double)n;
    double *r2 = malloc(sizeof(double) * (size_t)n);
    double *sorted = malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        const double dx = x[i] - cx, dy = y[i] - cy, dz = z[i] - cz;
        r2[i] = dx * dx + dy * dy + dz * dz;
        sorted[i] = r2[i];
    }
    qsort(sorted, (size_t)n, sizeof(double), cmp_double);
    for (int64_t i = 0; i < n; ++i) {
        int64_t lo = 0, hi = n; /* first entry not below r2[i] */
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (sorted[mid] < r2[i]) lo = mid + 1;
            else hi = mid;
        }
        const int64_t Q = lo;
        if (Q == 0) {
            Ex[i] = Ey[i] = Ez[i] = 0.0;
            continue;
        }
        const double w = r2[i] + s2;
        const double f = K * (double)Q / (w * sqrt(w));
        Ex[i] = f * (x[i] - cx);
        Ey[i] = f * (y[i] - cy);
        Ez[i] = f * (z[i] - cz);
    }
    free(r2);
    free(sorted);
}

/* Eq. 7 field of n holes on each other ([n][3] in, [n][3] out). */
void oc_field_spherical(const oc_params *p, int64_t n, const double *xyz, double *E)
{
    const size_t m = (size_t)(n > 0 ? n : 1);
    double *x = malloc(sizeof(double) * m), *y = malloc(sizeof(double) * m);
    double *z = malloc(sizeof(double) * m), *ex = malloc(sizeof(double) * m);
    double *ey = malloc(sizeof(double) * m), *ez = malloc(sizeof(double) * m);
    for (int64_t i = 0; i < n; ++i) {
        x[i] = xyz[3 * i];
        y[i] = xyz[3 * i + 1];
        z[i] = xyz[3 * i + 2];
    }
    spherical_field(p, n, x, y, z, ex, ey, ez);
    for (int64_t i = 0; i < n; ++i) {
        E[3 * i] = ex[i];
        E[3 * i + 1] = ey[i];
        E[3 * i + 2] = ez[i];
    }
    free(x); free(y); free(z); free(ex); free(ey); free(ez);
}

/* Repulsion field on selected carriers only: E[t] for carrier targets[t] of
 * the n carriers in xyz (each target costs O(n)). */
void oc_field_targets(const oc_params *p, int64_t n, const double *xyz, int64_t n_t,
                      const int64_t *targets, double *E)
{
    double *x = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *y = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *z = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        x[i] = xyz[3 * i];
        y[i] = xyz[3 * i + 1];
        z[i] = xyz[3 * i + 2];
    }
    const double K = oc_coulomb_k(p);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n_t; ++t) repulsion_one(p, n, x, y, z, NULL, targets[t], K, E + 3 * t);
    free(x);
    free(y);
    free(z);
}

/* Algorithm 1, initialisation: N = round(E / w) holes. */
int32_t oc_carrier_count(const oc_params *p, const oc_event *ev)
{
    if (ev->n_carriers > 0) return ev->n_carriers;
    return (int32_t)floor(1000.0 * ev->energy_kev / p->pair_energy_ev + 0.5);
}

/* Electrons of an event: none without the electron species, else one per
 * hole unless an explicit count is given. */
int32_t oc_electron_count(const oc_params *p, const oc_event *ev)
{
    if (!(p->physics & OC_ELECTRONS)) return 0;
    return ev->n_electrons >= 0 ? ev->n_electrons : oc_carrier_count(p, ev);
}

/* Eq. 2: sigma = 0.0044 E^1.75 (um, E in keV) unless the event states one. */
double oc_initial_sigma(const oc_event *ev)
{
    if (ev->sigma_um >= 0.0) return ev->sigma_um;
    return 0.0044 * pow(ev->energy_kev, 1.75);
}

/* Mirror z at either face of the sensor until it lies in [0, H]. */
static double fold_into_sensor(double z, double H)
{
    while (z < 0.0 || z > H) z = z < 0.0 ? -z : 2.0 * H - z;
    return z;
}

/* The deposits of a track event: n_deposits segment midpoints of the walk
 * described in the header ([n_deposits][3] out). */
void oc_track_deposits(const oc_params *p, const oc_event *ev, uint64_t eid, double *out)
{
    const double H = p->thickness_um, L = ev->seg_len_um;
    const uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    double px = ev->deposits[0], py = ev->deposits[1], pz = ev->deposits[2];
    for (int32_t k = 0; k < ev->n_deposits; ++k) {
        double dx = 0.0, dy = 0.0, dz = -1.0;
        if (k > 0) {
            const uint32_t ctr[4] = {(uint32_t)k, 0u, (uint32_t)eid, 3u};
            uint32_t w[4];
            oc_philox4x32_10(ctr, key, w);
            const double cos_t = 1.0 - 2.0 * to_unit(w[0]);
            const double sin_t = sqrt(1.0 - cos_t * cos_t);
            const double phi = 2.0 * PI * to_unit(w[1]);
            dx = sin_t * cos(phi);
            dy = sin_t * sin(phi);
            dz = cos_t;
        }
        const double qx = px + L * dx, qy = py + L * dy, qz = pz + L * dz;
        out[3 * k + 0] = 0.5 * (px + qx);
        out[3 * k + 1] = 0.5 * (py + qy);
        out[3 * k + 2] = fold_into_sensor(0.5 * (pz + qz), H);
        px = qx;
        py = qy;
        pz = fold_into_sensor(qz, H);
    }
}

int32_t oc_pixel_bin(const oc_params *p, double x, double y)
{
    const int32_t G = p->grid_n;
    const double half = 0.5 * G * p->pitch_um;
    const double fx = floor((x + half) / p->pitch_um);
    const double fy = floor((y + half) / p->pitch_um);
    if (fx >= 0.0 && fx < G && fy >= 0.0 && fy < G) return (int32_t)fy * G + (int32_t)fx;
    return G * G;
}

static int check_params(const oc_params *p)
{
    if (!(p->thickness_um > 0.0) || !(p->dt_ns > 0.0) || !(p->temperature_k > 0.0)) return OC_EINVAL;
    if (!(p->pitch_um > 0.0) || p->grid_n < 1 || !(p->softening_um >= 0.0) || !(p->eps_r > 0.0))
        return OC_EINVAL;
    if (!(p->pair_energy_ev > 0.0) || p->mobility < 0 || p->mobility > 1) return OC_EINVAL;
    if ((p->physics & OC_DRIFT) && !(p->v_bias > p->v_dep && p->v_dep >= 0.0)) return OC_EINVAL;
    if (p->physics & ~31u) return OC_EINVAL;
    if ((p->physics & OC_SPHERICAL) && (p->physics & OC_ELECTRONS)) return OC_EINVAL;
    for (int e = 0; e < 2; ++e) {
        double m[3];
        oc_mobility_params_of(p, e, m);
        if (!(m[0] > 0.0) || !(m[1] > 0.0) || !(m[2] > 0.0)) return OC_EINVAL;
    }
    return OC_OK;
}

typedef struct {
    int32_t n, nh;  /* carriers; the first nh are holes, the rest electrons */
    double *x, *y, *z;
    double *nx, *ny, *nz;
    int32_t *id;
    unsigned char *alive;
    int64_t *act; /* indices of the alive carriers, in carrier order */
    double *ax, *ay, *az, *aq;
    double *sx, *sy, *sz; /* spherical-model field of the alive set */
} oc_work;

static void retire(const oc_params *p, oc_work *w, int32_t i, int64_t step, int32_t *pix,
                   double *xyz_out, int32_t *cstep)
{
    w->alive[i] = 0;
    xyz_out[3 * i] = w->x[i];
    xyz_out[3 * i + 1] = w->y[i];
    xyz_out[3 * i + 2] = w->z[i];
    cstep[i] = (int32_t)step;
    if (i < w->nh) pix[oc_pixel_bin(p, w->x[i], w->y[i])] += 1;  /* holes reach the pixels */
}

/* Boundaries after an update: holes are mirrored at the entrance side and
 * collected at the pixel plane; electrons are mirrored at the pixel plane
 * and collected at the entrance side.  Returns 1 when collected. */
static int boundary(const oc_work *w, int32_t i, double H, double *z)
{
    if (i < w->nh) {
        if (*z > H) *z = 2.0 * H - *z;
        return *z <= 0.0;
    }
    if (*z < 0.0) *z = -*z;
    return *z >= H;
}

/* Simulate one event to completion (or max_steps).  Outputs are indexed by
 * the carrier's position in the event: holes, then electrons. */
static int run_event(const oc_params *p, const oc_event *ev, uint64_t eid, int parallel_targets,
                     int32_t *pix, double *xyz_out, int32_t *cstep, int64_t *steps_out,
                     uint64_t *pairs_out, uint64_t *hole_steps_out)
{
    const int32_t nh = oc_carrier_count(p, ev);
    const int32_t ne = oc_electron_count(p, ev);
    const int32_t n = (nh > 0 ? nh : 0) + (ne > 0 ? ne : 0);
    const double H = p->thickness_um;
    const double sigma = oc_initial_sigma(ev);
    const double K = oc_coulomb_k(p);
    const double kT = oc_thermal_voltage(p);
    const double dt = p->dt_ns;
    for (int32_t g = 0; g <= p->grid_n * p->grid_n; ++g) pix[g] = 0;
    *steps_out = 0;
    *pairs_out = 0;
    *hole_steps_out = 0;
    if (n <= 0) return OC_OK;
    if (ev->n_deposits > 0 && ne > 0 && ne != nh) return OC_EINVAL;
    /* a track's deposits come from its walk */
    double *track = NULL;
    const double *deposits = ev->deposits;
    if (ev->seg_len_um > 0.0) {
        track = malloc(3 * sizeof(double) * (size_t)ev->n_deposits);
        oc_track_deposits(p, ev, eid, track);
        deposits = track;
    }

    oc_work w;
    const size_t nd = (size_t)n;
    w.n = n;
    w.nh = nh > 0 ? nh : 0;
    w.x = malloc(nd * sizeof(double));
    w.y = malloc(nd * sizeof(double));
    w.z = malloc(nd * sizeof(double));
    w.nx = malloc(nd * sizeof(double));
    w.ny = malloc(nd * sizeof(double));
    w.nz = malloc(nd * sizeof(double));
    w.ax = malloc(nd * sizeof(double));
    w.ay = malloc(nd * sizeof(double));
    w.az = malloc(nd * sizeof(double));
    w.aq = malloc(nd * sizeof(double));
    w.sx = malloc(nd * sizeof(double));
    w.sy = malloc(nd * sizeof(double));
    w.sz = malloc(nd * sizeof(double));
    w.id = malloc(nd * sizeof(int32_t));
    w.alive = malloc(nd);
    w.act = malloc(nd * sizeof(int64_t));
    int status = OC_OK;

    /* initial cloud: Gaussian around each deposit (Algorithm 1, Eq. 2); the
     * electron of a pair starts where its hole does */
    for (int32_t i = 0; i < n; ++i) {
        const int32_t k = i < w.nh ? i : i - w.nh; /* index within the species */
        w.id[i] = ev->ids ? ev->ids[i] : k;
        cstep[i] = -1;
        if (ev->n_deposits > 0) {
            if (i < w.nh) {
                const double *d = deposits + 3 * (i % ev->n_deposits);
                double g[3];
                oc_normals3(p->seed, (uint32_t)w.id[i], 0u, (uint32_t)eid, 1u, g);
                w.x[i] = d[0] + sigma * g[0];
                w.y[i] = d[1] + sigma * g[1];
                w.z[i] = d[2] + sigma * g[2];
            } else {
                w.x[i] = w.x[k];
                w.y[i] = w.y[k];
                w.z[i] = w.z[k];
            }
        } else {
            w.x[i] = ev->xyz[3 * i];
            w.y[i] = ev->xyz[3 * i + 1];
            w.z[i] = ev->xyz[3 * i + 2];
            if (!isfinite(w.x[i]) || !isfinite(w.y[i]) || !isfinite(w.z[i])) status = OC_ENONFINITE;
        }
        w.alive[i] = 1;
    }
    if (status != OC_OK) goto done;
    for (int32_t i = 0; i < n; ++i)
        if (boundary(&w, i, H, &w.z[i])) retire(p, &w, i, ev->start_step, pix, xyz_out, cstep);

    int64_t step = ev->start_step;
    for (;;) {
        /* snapshot of the alive set, in carrier order; the event ends with
         * its last hole */
        int64_t na = 0, holes = 0;
        for (int32_t i = 0; i < n; ++i)
            if (w.alive[i]) {
                w.ax[na] = w.x[i];
                w.ay[na] = w.y[i];
                w.az[na] = w.z[i];
                w.aq[na] = i < w.nh ? 1.0 : -1.0;
                w.act[na++] = i;
                holes += i < w.nh;
            }
        if (holes == 0) break;
        if (step - ev->start_step >= p->max_steps) {
            status = OC_EMAXSTEPS;
            break;
        }
        *pairs_out += (uint64_t)na * (uint64_t)(na - 1);
        *hole_steps_out += (uint64_t)na;
        const int spherical = (p->physics & OC_SPHERICAL) && (p->physics & OC_REPULSION);
        if (spherical) spherical_field(p, na, w.ax, w.ay, w.az, w.sx, w.sy, w.sz);
#pragma omp parallel for schedule(static) if (parallel_targets)
        for (int64_t a = 0; a < na; ++a) {
            const int64_t i = w.act[a];
            const int electron = i >= w.nh;
            const double sign = electron ? -1.0 : 1.0; /* velocity along q_i E */
            double Er[3] = {0.0, 0.0, 0.0};
            if (spherical) {
                Er[0] = w.sx[a];
                Er[1] = w.sy[a];
                Er[2] = w.sz[a];
            } else if (p->physics & OC_REPULSION) {
                repulsion_one(p, na, w.ax, w.ay, w.az, w.aq, a, K, Er);
            }
            const double Ex = Er[0], Ey = Er[1], Ez = Er[2] + oc_drift_field(p, w.az[a]);
            const double Emag = sqrt(Ex * Ex + Ey * Ey + Ez * Ez);
            const double mu = oc_mobility_of(p, electron, Emag);
            double g[3] = {0.0, 0.0, 0.0};
            double hop = 0.0;
            if (p->physics & OC_DIFFUSION) {
                const double D = mu * kT;
                hop = sqrt(2.0 * D * dt);
                oc_normals3(p->seed, (uint32_t)w.id[i], (uint32_t)step, (uint32_t)eid,
                            electron ? 4u : 0u, g);
            }
            w.nx[i] = w.ax[a] + sign * mu * Ex * dt + hop * g[0];
            w.ny[i] = w.ay[a] + sign * mu * Ey * dt + hop * g[1];
            w.nz[i] = w.az[a] + sign * mu * Ez * dt + hop * g[2];
        }
        step += 1;
        for (int64_t a = 0; a < na; ++a) {
            const int64_t i = w.act[a];
            w.x[i] = w.nx[i];
            w.y[i] = w.ny[i];
            w.z[i] = w.nz[i];
            if (boundary(&w, (int32_t)i, H, &w.z[i]))
                retire(p, &w, (int32_t)i, step, pix, xyz_out, cstep);
        }
    }
    *steps_out = step - ev->start_step;
    /* carriers still drifting report their current position */
    for (int32_t i = 0; i < n; ++i)
        if (w.alive[i]) {
            xyz_out[3 * i] = w.x[i];
            xyz_out[3 * i + 1] = w.y[i];
            xyz_out[3 * i + 2] = w.z[i];
        }
done:
    free(w.x); free(w.y); free(w.z);
    free(w.nx); free(w.ny); free(w.nz);
    free(w.ax); free(w.ay); free(w.az); free(w.aq);
    free(w.sx); free(w.sy); free(w.sz);
    free(w.id); free(w.alive); free(w.act);
    free(track);
    return status;
}

/* Run a batch.  Event b uses RNG event id first_event_id + b.  Outputs:
 * pix [B][grid_n^2 + 1] (holes), xyz_out [sum N_e][3], cstep [sum N_e]
 * (-1 = still drifting), where N_e counts the event's holes and electrons,
 * steps [B], pairs = sum over steps of N_a (N_a - 1), hole_steps = sum over
 * steps of N_a (carrier updates of both species).  Returns the worst status
 * over events. */
int oc_run(const oc_params *p, const oc_event *ev, int32_t n_events, uint64_t first_event_id,
           int32_t *pix, double *xyz_out, int32_t *cstep, int64_t *steps, uint64_t *pairs,
           uint64_t *hole_steps)
{
    int st = check_params(p);
    if (st != OC_OK) return st;
    if (n_events < 0) return OC_EINVAL;
    int64_t *off = malloc(sizeof(int64_t) * (size_t)(n_events + 1));
    off[0] = 0;
    for (int32_t b = 0; b < n_events; ++b) {
        if (ev[b].n_deposits < 0 || (ev[b].n_deposits == 0 && ev[b].n_carriers > 0 && !ev[b].xyz) ||
            (ev[b].n_deposits > 0 && !ev[b].deposits) || !(ev[b].seg_len_um >= 0.0) ||
            !isfinite(ev[b].seg_len_um) || (ev[b].seg_len_um > 0.0 && ev[b].n_deposits == 0)) {
            free(off);
            return OC_EINVAL;
        }
        const int32_t nh = oc_carrier_count(p, &ev[b]), ne = oc_electron_count(p, &ev[b]);
        off[b + 1] = off[b] + (nh > 0 ? nh : 0) + (ne > 0 ? ne : 0);
    }
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    const int outer = n_events >= 2 * nthreads;
    const int G1 = p->grid_n * p->grid_n + 1;
    uint64_t total_pairs = 0, total_hs = 0;
    int worst = OC_OK;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total_pairs, total_hs) if (outer)
    for (int32_t b = 0; b < n_events; ++b) {
        uint64_t pr = 0, hs = 0;
        const int s = run_event(p, &ev[b], first_event_id + (uint64_t)b, !outer, pix + (size_t)b * G1,
                                xyz_out + 3 * off[b], cstep + off[b], steps + b, &pr, &hs);
        total_pairs += pr;
        total_hs += hs;
        if (s != OC_OK) {
#pragma omp critical
            {
                if (worst == OC_OK || s < worst) worst = s;
            }
        }
    }
    if (pairs) *pairs = total_pairs;
    if (hole_steps) *hole_steps = total_hs;
    free(off);
    return worst;
}

void oc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
