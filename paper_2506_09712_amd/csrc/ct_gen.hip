// Parameterised event generation of arXiv:2506.09712 (Sec. 4.2) for gfx950:
// events drawn from the drift-time approximation (Eq. 9) and the fitted
// generalized Gaussian parameters alpha(t), beta(t) (Eqs. 8, 10, 11), with
// Fano fluctuation of the carrier count, a sub-pixel shift, and pixel noise.
//
// One 64-lane wave per event.  Every lane derives the event's draws (depth,
// drift time, alpha, beta, carrier count, shift) from the same Philox blocks;
// lanes 0..G and 32..32+G evaluate the CDF of the GGD at the pixel edges in
// x and y (regularized incomplete gamma), shared through LDS.  A carrier's
// column is the pixel whose edge CDFs bracket its uniform draw, its row
// likewise: the same distribution as drawing its position from the GGD and
// binning it, without evaluating the inverse CDF.  Each lane counts its
// carriers in a private LDS histogram (odd stride, no bank conflicts); the
// lanes' histograms are summed, converted to energy and given their noise.
#include "ct_device.hpp"

namespace ct {

namespace {

constexpr uint32_t kDomainGenerator = 5u;

// Regularized lower incomplete gamma P(a, x) for a > 0, x >= 0 (FP64), by
// the two classical expansions, each used where it converges fast:
//  * x < a + 1: the power series of DLMF 8.7.1 (Abramowitz and Stegun
//    6.5.29), P = x^a e^-x sum_k x^k / Gamma(a + k + 1), written as
//    x^a e^-x / Gamma(a) times sum_k x^k / (a (a + 1) ... (a + k)), each term
//    the previous one times x / (a + k);
//  * otherwise P = 1 - Q, Q = x^a e^-x / Gamma(a) times the even contraction
//    of the continued fraction of DLMF 8.9.2 (Abramowitz and Stegun 6.5.31),
//    1 / (x + 1 - a - 1 (1 - a) / (x + 3 - a - 2 (2 - a) / (x + 5 - a - ...))),
//    evaluated front to back with the modified Lentz algorithm (Lentz,
//    Appl. Opt. 15, 668 (1976); Thompson and Barnett, J. Comput. Phys. 64,
//    490 (1986)): the convergent is a running product of ratios of
//    successive numerator and denominator recurrences.
__device__ double gamma_p(double a, double x)
{
    if (!(x > 0.0)) return 0.0;
    const double log_prefactor = -x + a * log(x) - lgamma(a);  // log of x^a e^-x / Gamma(a)
    if (x < a + 1.0) {
        double shifted = a, term = 1.0 / a, series = term;
        for (int k = 0; k < 400; ++k) {
            shifted += 1.0;
            term *= x / shifted;
            series += term;
            if (fabs(term) < fabs(series) * 1e-17) break;
        }
        return series * exp(log_prefactor);
    }
    // Lentz: partial numerators -k (k - a), partial denominators x + 2k + 1 - a;
    // `floor_` replaces a recurrence ratio that would vanish
    const double floor_ = 1e-300;
    double denom = x + 1.0 - a, num_ratio = 1.0 / floor_, den_ratio = 1.0 / denom;
    double convergent = den_ratio;
    for (int k = 1; k < 400; ++k) {
        const double numer = -k * (k - a);
        denom += 2.0;
        den_ratio = numer * den_ratio + denom;
        if (fabs(den_ratio) < floor_) den_ratio = floor_;
        num_ratio = denom + numer / num_ratio;
        if (fabs(num_ratio) < floor_) num_ratio = floor_;
        den_ratio = 1.0 / den_ratio;
        const double step = den_ratio * num_ratio;
        convergent *= step;
        if (fabs(step - 1.0) < 1e-17) break;
    }
    return 1.0 - exp(log_prefactor) * convergent;
}

// CDF of the symmetric GGD (Eq. 8) of scale alpha and shape beta at x.
__device__ double ggd_cdf(double x, double alpha, double beta)
{
    const double p = 0.5 * gamma_p(1.0 / beta, pow(fabs(x) / alpha, beta));
    return x < 0.0 ? 0.5 - p : 0.5 + p;
}

// Column (row) of a draw: the pixel i with cdf[i] <= u < cdf[i + 1], -1 or G
// outside the grid, for the uniform u = (w + 0.5) 2^-32 of a Philox word w.
// Compared in the word's own scale: with t = cdf 2^32 - 0.5 (exact in FP64
// for cdf in [0, 1], and for cdf < 1/4 only its sign matters), cdf <= u
// exactly when t <= w, so each edge costs one conversion-free compare.
// t (the scaled edges) is non-decreasing.
template <int G>
__device__ __forceinline__ int pixel_of(const double (&t)[G + 1], uint32_t w)
{
    const double wd = (double)w;
    int i = -1;
#pragma unroll
    for (int e = 0; e <= G; ++e) i += t[e] <= wd ? 1 : 0;
    return i;
}

// One event per 64-lane workgroup; G = pixels per side (compile-time, so the
// edge CDFs stay in registers and the searches unroll).
template <int G>
__global__ __launch_bounds__(64) void k_gen(GenDev g, int64_t n_events, double *energy,
                                            int32_t *counts, double *info)
{
    constexpr int B = G * G + 1, stride = B | 1;  // odd stride per lane
    __shared__ double cdf[2 * (G + 1)];
    __shared__ int32_t hist[64 * stride];
    const int64_t b = blockIdx.x;
    if (b >= n_events) return;
    const int lane = threadIdx.x;
    const uint32_t eid = (uint32_t)(g.first_event_id + (uint64_t)b);

    // the event: depth, drift time (Eq. 9), GGD parameters (Eqs. 10, 11),
    // carrier count with Fano fluctuation, sub-pixel shift
    const Ctr w = philox10(Ctr{0u, 0u, eid, kDomainGenerator}, g.key0, g.key1);
    const double h = -g.atten * log(1.0 - to_unit(w.c0) * g.keep);
    const double e_h = g.e_entrance + g.k * h;
    const double t = g.k > 0.0 ? (log(g.e_pixels / e_h) / g.k + (g.H - h) * g.inv_ec) * g.inv_mu0
                               : (g.H - h) * (1.0 / e_h + g.inv_ec) * g.inv_mu0;
    const double rt = sqrt(t);
    const double alpha = fmax(g.pa[0] + g.pa[1] * rt + g.pa[2] * t + g.pa[3] * t * t, 1e-300);
    const double beta = fmax(2.0 + g.pb[0] * pow(t - g.pb[1], g.pb[2]) + g.pb[3] * exp(g.pb[4] * t),
                             1e-3);
    double nrm[3];
    normals3(g.key0, g.key1, Ctr{1u, 0u, eid, kDomainGenerator}, nrm);
    const int n = (int)fmax(0.0, floor(g.mean_n + g.sd_n * nrm[0] + 0.5));
    const double x0 = (to_unit(w.c1) - 0.5) * g.pitch, y0 = (to_unit(w.c2) - 0.5) * g.pitch;

    // edge CDFs: lanes 0..G for x, 32..32+G for y
    const int q = lane & 31;
    if (q <= G) {
        const double edge = (q - 0.5 * G) * g.pitch;
        cdf[(lane >> 5) * (G + 1) + q] = ggd_cdf(edge - (lane < 32 ? x0 : y0), alpha, beta);
    }
    for (int i = lane; i < 64 * stride; i += 64) hist[i] = 0;
    __syncthreads();
    double cx[G + 1], cy[G + 1];  // edge CDFs in the scale of a Philox word
#pragma unroll
    for (int e = 0; e <= G; ++e) {
        cx[e] = fma(cdf[e], 4294967296.0, -0.5);
        cy[e] = fma(cdf[G + 1 + e], 4294967296.0, -0.5);
    }
    int32_t *mine = hist + lane * stride;
    // carriers 2j and 2j + 1 share Philox block (j, 1, event, 5)
    const int pairs = (n + 1) >> 1;
    for (int j = lane; j < pairs; j += 64) {
        const Ctr c = philox10(Ctr{(uint32_t)j, 1u, eid, kDomainGenerator}, g.key0, g.key1);
        {
            const int col = pixel_of<G>(cx, c.c0), row = pixel_of<G>(cy, c.c1);
            const bool in = (unsigned)col < (unsigned)G && (unsigned)row < (unsigned)G;
            mine[in ? row * G + col : G * G] += 1;
        }
        if (2 * j + 1 < n) {
            const int col = pixel_of<G>(cx, c.c2), row = pixel_of<G>(cy, c.c3);
            const bool in = (unsigned)col < (unsigned)G && (unsigned)row < (unsigned)G;
            mine[in ? row * G + col : G * G] += 1;
        }
    }
    __syncthreads();
    // sum the lanes' histograms; energies with noise (normal (p mod 3) of
    // block (p div 3, 2, event, 5))
    for (int p = lane; p < B; p += 64) {
        int cnt = 0;
        for (int l = 0; l < 64; ++l) cnt += hist[l * stride + p];
        if (counts) counts[b * B + p] = cnt;
        if (energy && p < G * G) {
            double nz[3];
            normals3(g.key0, g.key1, Ctr{(uint32_t)(p / 3), 2u, eid, kDomainGenerator}, nz);
            energy[b * (G * G) + p] = cnt * g.w_kev + g.noise * nz[p % 3];
        }
    }
    if (info && lane == 0) {
        double *o = info + 5 * b;
        o[0] = h;
        o[1] = t;
        o[2] = (double)n;
        o[3] = x0;
        o[4] = y0;
    }
}

}  // namespace

hipError_t launch_gen(const GenDev &g, int64_t n_events, double *energy, int32_t *counts,
                      double *info, hipStream_t s)
{
    if (n_events <= 0) return hipSuccess;
    switch (g.grid_n) {
#define CT_GEN_CASE(G_)                                                                          \
    case G_:                                                                                     \
        hipLaunchKernelGGL(k_gen<G_>, dim3((unsigned)n_events), dim3(64), 0, s, g, n_events,     \
                           energy, counts, info);                                                \
        break;
        CT_GEN_CASE(1) CT_GEN_CASE(2) CT_GEN_CASE(3) CT_GEN_CASE(4)
        CT_GEN_CASE(5) CT_GEN_CASE(6) CT_GEN_CASE(7) CT_GEN_CASE(8)
#undef CT_GEN_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ct
