// Layout of the simplified spherical model's work (ct_sph.hip) shared with
// the host side (ct_capi.cpp): block sizes, the group size of large events and
// the byte layout of the state their workgroups share.  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ct {

// One workgroup of kSphBlock threads ranks the holes of an event by distance
// from its centre with a counting sort over kSphBins bins.  An event of more
// than kSphGroupMin holes at seeding is shared by sph_group(n0) workgroups of
// kSphSharedBlock threads, each owning a contiguous slice of its drifting
// holes (at most about kSphSlice); the workgroups of an event meet at
// barriers on a counter of their own.  The group size depends on the event's
// seeded size alone (and on the device's resident capacity), so an event's
// result does not depend on its batch.
constexpr int kSphBlock = 512;
constexpr int kSphSharedBlock = 1024;
constexpr int kSphBins = 8192;
constexpr int kSphGroupMin = 8192;
constexpr int kSphSlice = 5120;
constexpr int kSphMaxGroup = 32;

// Workgroups of an event of n0 holes at seeding (with repulsion): 1 up to
// kSphGroupMin holes, else one per kSphSlice holes, at least 2 and at most
// max_group (>= 2: the resident workgroups of the device) and kSphMaxGroup.
inline int sph_group(int64_t n0, int max_group)
{
    if (n0 <= kSphGroupMin) return 1;
    const int64_t g = (n0 + kSphSlice - 1) / kSphSlice;
    const int64_t cap = max_group < kSphMaxGroup ? max_group : kSphMaxGroup;
    return (int)(g < cap ? g : cap);
}

// Shared state of an event's G workgroups (device memory, 256-byte aligned
// pieces): the barrier counter, each workgroup's largest key, survivor count
// and coordinate sums, the bin histograms of the slices (turned into each
// slice's first position within every bin), the exclusive scan of the bin
// totals within each workgroup's range of bins, and the totals of the ranges.
struct SphGroupView {
    uint32_t *bar;
    double *gmax;        // [G]
    double *sums;        // [G][3]
    int32_t *kept;       // [G]
    int32_t *range_tot;  // [G]
    int32_t *colscan;    // [kSphBins]
    int32_t *ghist;      // [G][kSphBins]
};

__host__ __device__ inline size_t sph_align(size_t v) { return (v + 255) & ~(size_t)255; }

__host__ __device__ inline size_t sph_group_bytes(int G)
{
    return 256 + sph_align(8 * (size_t)G) + sph_align(24 * (size_t)G) + sph_align(4 * (size_t)G) +
           sph_align(4 * (size_t)G) + sph_align(4 * (size_t)kSphBins) +
           sph_align(4 * (size_t)kSphBins * G);
}

__host__ __device__ inline SphGroupView sph_group_view(char *p, int G)
{
    SphGroupView v;
    size_t o = 0;
    v.bar = reinterpret_cast<uint32_t *>(p + o);
    o += 256;
    v.gmax = reinterpret_cast<double *>(p + o);
    o += sph_align(8 * (size_t)G);
    v.sums = reinterpret_cast<double *>(p + o);
    o += sph_align(24 * (size_t)G);
    v.kept = reinterpret_cast<int32_t *>(p + o);
    o += sph_align(4 * (size_t)G);
    v.range_tot = reinterpret_cast<int32_t *>(p + o);
    o += sph_align(4 * (size_t)G);
    v.colscan = reinterpret_cast<int32_t *>(p + o);
    o += sph_align(4 * (size_t)kSphBins);
    v.ghist = reinterpret_cast<int32_t *>(p + o);
    return v;
}

}  // namespace ct
