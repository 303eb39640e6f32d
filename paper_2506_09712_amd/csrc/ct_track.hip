// Track events: the deposits of an event described by its start point and a
// segment length (ct_event_desc.seg_len_um > 0).  The paper seeds each event
// as Gaussian clouds around deposit points (Algorithm 1, Eq. 2) and has no
// model of an extended track; a track here is the chain of midpoints of a
// walk of straight segments, whose directions come from the counter-based
// generator, so that the library and any other implementation of the same
// definition place the same deposits.  The walk is event-level work (tens of
// segments per event): one thread per event, once per seeding, before the
// carriers are seeded around the deposits.
#include "ct_device.hpp"
#include "ct_track.hpp"

namespace ct {

namespace {

constexpr uint32_t kDomainTrack = 3u;

// z mirrored at the faces z = 0 and z = H until it lies in [0, H]: an even
// function with period 2H, taken in closed form (fmod is exact), so that a
// walk far outside the sensor costs no loop.
__device__ __forceinline__ double fold_into_sensor(double z, double H)
{
    if (z >= 0.0 && z <= H) return z;
    double t = fabs(fmod(z, 2.0 * H));
    if (t > H) t = 2.0 * H - t;
    return t;
}

// deposits[dep_off[b]] holds event b's start on entry and its first
// midpoint on exit; the event's other deposit slots are written.
__global__ __launch_bounds__(64) void k_track(DevParams dp, int32_t n_events, uint64_t first_event_id,
                                              const int32_t *__restrict__ dep_off,
                                              const double *__restrict__ seg_len,
                                              double *__restrict__ deposits)
{
    const int b = blockIdx.x * 64 + threadIdx.x;
    if (b >= n_events) return;
    const double L = seg_len[b];
    if (!(L > 0.0)) return;
    const int d0 = dep_off[b], nd = dep_off[b + 1] - d0;
    double *dep = deposits + 3 * (int64_t)d0;
    const double H = dp.H;
    double px = dep[0], py = dep[1], pz = dep[2];
    for (int k = 0; k < nd; ++k) {
        double dx = 0.0, dy = 0.0, dz = -1.0;  // the first segment enters along -z
        if (k > 0) {
            const Ctr w = philox10(Ctr{(uint32_t)k, 0u, (uint32_t)(first_event_id + b), kDomainTrack},
                                   dp.key0, dp.key1);
            const double cos_t = 1.0 - 2.0 * to_unit(w.c0);
            const double sin_t = sqrt(1.0 - cos_t * cos_t);
            double sp, cp;
            sincospi(2.0 * to_unit(w.c1), &sp, &cp);
            dx = sin_t * cp;
            dy = sin_t * sp;
            dz = cos_t;
        }
        const double qx = px + L * dx, qy = py + L * dy, qz = pz + L * dz;
        dep[3 * k + 0] = 0.5 * (px + qx);
        dep[3 * k + 1] = 0.5 * (py + qy);
        dep[3 * k + 2] = fold_into_sensor(0.5 * (pz + qz), H);
        px = qx;
        py = qy;
        pz = fold_into_sensor(qz, H);
    }
}

}  // namespace

hipError_t launch_track(const DevParams &dp, int32_t n_events, uint64_t first_event_id,
                        const int32_t *dep_off, const double *seg_len, double *deposits, hipStream_t s)
{
    if (n_events <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_track, dim3((n_events + 63) / 64), dim3(64), 0, s, dp, n_events,
                       first_event_id, dep_off, seg_len, deposits);
    return hipGetLastError();
}

}  // namespace ct
