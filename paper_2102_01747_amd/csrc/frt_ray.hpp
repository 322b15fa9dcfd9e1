// frt_ray.hpp -- per-ray helpers shared by the forward and adjoint kernels:
// orbit parameters of a job, primary ray of a pixel, the search interval
// (bounding sphere and cut planes), the batch ray index -> (job, pixel) map
// and wave-level lane utilities.
#pragma once

#include <hip/hip_runtime.h>

#include "frt_fractal.hpp"
#include "frt_job.hpp"

namespace frt {

__device__ __forceinline__ OrbitParams orbit_params(const JobDev& J) {
    OrbitParams p;
    p.c0 = J.c[0];
    p.c1 = J.c[1];
    p.c2 = J.c[2];
    p.c3 = J.c[3];
    p.n = J.power;
    p.nm1_half = 0.5f * (J.power - 1.0f);
    p.n_rev = J.n_rev;
    p.ipow = J.int_power;
    p.kind = J.kind;
    p.max_iter = J.max_iter;
    p.bail2 = J.bailout2;
    return p;
}

// Search interval of a ray (text around Listing 3): [tmin, t_max] cut by the
// bounding sphere and the kept half-spaces.  Returns false when empty;
// `entry` is the plane whose crossing sets the start strictly after every
// other lower bound (-1 if none).
__device__ __forceinline__ bool ray_interval(const JobDev& J, float ox, float oy, float oz, float dx, float dy,
                                             float dz, float tmin, float& lo, float& hi, int& entry) {
    const float b = fmaf(ox, dx, fmaf(oy, dy, oz * dz));
    const float cc = fmaf(ox, ox, fmaf(oy, oy, oz * oz)) - J.radius * J.radius;
    const float disc = fmaf(b, b, -cc);
    if (disc < 0.0f) return false;
    const float sq = sqrtf(disc);
    lo = fmaxf(tmin, -b - sq);
    hi = fminf(J.t_max, -b + sq);
    entry = -1;
    for (int k = 0; k < J.n_planes; ++k) {
        const float denom = fmaf(J.pn[k][0], dx, fmaf(J.pn[k][1], dy, J.pn[k][2] * dz));
        const float num = J.pd[k] - fmaf(J.pn[k][0], ox, fmaf(J.pn[k][1], oy, J.pn[k][2] * oz));
        if (denom == 0.0f) {
            if (num < 0.0f) return false;
        } else if (denom > 0.0f) {
            hi = fminf(hi, num / denom);
        } else {
            const float tk = num / denom;
            if (tk > lo) {
                lo = tk;
                entry = k;
            }
        }
    }
    return lo <= hi;
}

// Primary ray through pixel (px, py): pinhole, pixel centre, row 0 at the top.
__device__ __forceinline__ void primary_dir(const JobDev& J, int px, int py, float& dx, float& dy, float& dz) {
    const float u = fmaf(px + 0.5f, J.inv_w2, -1.0f) * J.sx;
    const float v = fmaf(-(py + 0.5f), J.inv_h2, 1.0f) * J.sy;
    const float rx = fmaf(u, J.right[0], fmaf(v, J.upv[0], J.fwd[0]));
    const float ry = fmaf(u, J.right[1], fmaf(v, J.upv[1], J.fwd[1]));
    const float rz = fmaf(u, J.right[2], fmaf(v, J.upv[2], J.fwd[2]));
    const float inv = hw_rsq(fmaf(rx, rx, fmaf(ry, ry, rz * rz)));
    dx = rx * inv;
    dy = ry * inv;
    dz = rz * inv;
}

// The same ray in FP64 from the FP64 camera basis (used by the adjoint).
__device__ __forceinline__ void primary_dir_f64(const JobDev& J, int px, int py, double& dx, double& dy, double& dz) {
    const double u = (2.0 * (px + 0.5) / J.width - 1.0) * J.sx_d;
    const double v = (1.0 - 2.0 * (py + 0.5) / J.height) * J.sy_d;
    const double rx = fma(u, J.right_d[0], fma(v, J.upv_d[0], J.fwd_d[0]));
    const double ry = fma(u, J.right_d[1], fma(v, J.upv_d[1], J.fwd_d[1]));
    const double rz = fma(u, J.right_d[2], fma(v, J.upv_d[2], J.fwd_d[2]));
    const double inv = 1.0 / sqrt(fma(rx, rx, fma(ry, ry, rz * rz)));
    dx = rx * inv;
    dy = ry * inv;
    dz = rz * inv;
}

// Work-item and dispatch geometry along x (every grid here is 1-D and made of
// whole blocks), read from the hardware registers and the dispatch packet.
// HIP's threadIdx / blockIdx / blockDim / gridDim go through device-library
// functions, which are not inlined into kernels built with another
// floating-point mode than the library's and then become real calls.
__device__ __forceinline__ unsigned thread_x() { return __builtin_amdgcn_workitem_id_x(); }
__device__ __forceinline__ unsigned block_x() { return __builtin_amdgcn_workgroup_id_x(); }
__device__ __forceinline__ unsigned block_threads() { return __builtin_amdgcn_workgroup_size_x(); }
__device__ __forceinline__ unsigned grid_threads() { return __builtin_amdgcn_grid_size_x(); }

__device__ __forceinline__ unsigned long long bcast_first(unsigned long long v) {
    const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(v));
    const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(v >> 32));
    return (static_cast<unsigned long long>(hi) << 32) | lo;
}

__device__ __forceinline__ unsigned lane_rank(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<unsigned>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<unsigned>(mask), 0u));
}

template <bool BATCH>
__device__ __forceinline__ const JobDev& job_ref(const JobDev* __restrict__ jobs, const JobDev& job1, int j) {
    if constexpr (BATCH) return jobs[j]; else return job1;
}

// Pixel of ray r of a job (r counted from the job's first ray; 64 rays per
// 8 x 8 pixel tile, tiles in row-major order); false for the padding lanes
// of edge tiles.
__device__ __forceinline__ bool tile_pixel(const JobDev& J, long long r, int& px, int& py) {
    const int tile = static_cast<int>(r >> 6), wl = static_cast<int>(r & 63);
    const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
    px = tx * kTile + (wl & (kTile - 1));
    py = ty * kTile + (wl >> 3);
    return px < J.width && py < J.height;
}

// Wave-uniform cursor over the job table: the job whose ray range holds the
// wave's current claim.  Every job's range is a whole number of 64-ray
// tiles, so a tile never spans two jobs, and consecutive claims of a wave
// need no search of the table and read the job through scalar loads.
struct JobCursor {
    int j = 0;
    unsigned long long begin = 0, end = 0;
};

// Point the cursor at the job holding ray g (g must be wave-uniform).
template <bool BATCH>
__device__ __forceinline__ void job_seek(const JobDev* __restrict__ jobs, const JobDev& job1, int n_jobs,
                                         unsigned long long g, JobCursor& c) {
    if (g >= c.begin && g < c.end) return;
    if constexpr (BATCH) {
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (static_cast<unsigned long long>(jobs[mid].ray_begin) <= g) lo = mid; else hi = mid - 1;
        }
        c.j = __builtin_amdgcn_readfirstlane(lo);
        c.begin = static_cast<unsigned long long>(jobs[c.j].ray_begin);
        c.end = c.begin + static_cast<unsigned long long>(jobs[c.j].ray_count);
    } else {
        c.j = 0;
        c.begin = static_cast<unsigned long long>(job1.ray_begin);
        c.end = c.begin + static_cast<unsigned long long>(job1.ray_count);
    }
}

// Map a ray index of the batch to (job, pixel); false for the padding lanes
// of edge tiles.
template <bool BATCH>
__device__ __forceinline__ bool ray_pixel(const JobDev* __restrict__ jobs, const JobDev& job1, int n_jobs,
                                          long long g, int& j, int& px, int& py) {
    j = 0;
    if constexpr (BATCH) {
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].ray_begin <= g) lo = mid; else hi = mid - 1;
        }
        j = lo;
    }
    const JobDev& J = job_ref<BATCH>(jobs, job1, j);
    return tile_pixel(J, g - J.ray_begin, px, py);
}

}  // namespace frt
