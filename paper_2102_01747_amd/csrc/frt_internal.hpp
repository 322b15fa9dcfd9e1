// frt_internal.hpp -- launch interface between the host API and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "frt.h"
#include "frt_job.hpp"

namespace frt {

struct LaunchCfg {
    int grid;             // workgroups of the march kernels (persistent: fill the chip once)
    int normal_grid;      // workgroups of the normal kernel (grid-stride)
    int block;            // threads per workgroup, multiple of 64
    int chunk;            // rays claimed from the queue per refill
    int orbit_lanes;      // keep iterating orbits while this many lanes still iterate
    int rare_lanes;       // waiting lanes that trigger shading / refill
};

// One group of a forward launch: the rays of one kernel variant.
struct TraceGroup {
    int variant;
    LaunchCfg cfg;
    bool any_shadow;   // some job of the group casts shadow rays
};

// Forward pass: resets the ray queues in the workspace header, then launches
// the primary march of every group, the normal kernel of every group and the
// shadow march of every group that has shadow rays.  batch = false reads the
// job from `job1` (kernel argument, one group); batch = true reads `jobs`
// (device table) and each group's ray range from `hdr`.
// marks[0..3] (optional, may be null): events recorded on `stream` before the
// primary marches, before the normal kernels, before the shadow marches and
// after the last kernel.
// fork = true (eager calls only: not under graph capture, not from the
// entry point that allocates nothing, not with marks): groups after the first
// run on the library's side streams, forked after the counter reset and
// joined back into `stream` at the end, so one group's kernels fill the
// device while another's drain.
hipError_t launch_trace(const TraceGroup* groups, int n_groups, bool batch, const JobDev* jobs, const JobDev& job1,
                        WorkspaceHeader* hdr, hipStream_t stream, hipEvent_t* marks = nullptr, bool fork = false);

// Side streams of the current device (default priority, non-blocking),
// created on first use.  fork_streams makes the first n wait for everything
// queued on `main` so far and returns them; join_streams makes `main` wait
// for everything queued on them.  Both hold a lock across their records and
// waits.
constexpr int kSideStreams = 4;
hipError_t fork_streams(hipStream_t main, int n, hipStream_t* side);
hipError_t join_streams(hipStream_t main, int n);
const void* trace_kernel_symbol(int variant, bool batch);

// Batch set-up shared by the batch entry points (frt_api.cpp): validates
// every job before anything is packed, then packs the jobs variant by
// variant (the order of the ray index space) and hands each JobDev, in
// table order, to sink(ctx, J) (false aborts with FRT_EHIP); fills the
// header's ranges, ray total and job count (the claim counters stay zero)
// and one launch group per variant present (groups holds kNumVariants).
// Errors are recorded for frt_last_error().
// With closest_hit_elsewhere, jobs with the closest-hit shading model pass
// validation and are left out of the table (hdr.n_jobs counts the table);
// otherwise they are refused with FRT_EUNSUPPORTED.
frt_status batch_layout(const frt_job* jobs, int32_t n_jobs, WorkspaceHeader& hdr, TraceGroup* groups, int& n_groups,
                        bool (*sink)(void* ctx, const JobDev& J), void* ctx, bool closest_hit_elsewhere);
// The validation pass of batch_layout alone (host only, no device call).
frt_status batch_validate(const frt_job* jobs, int32_t n_jobs, bool allow_closest_hit);
// A job with the closest-hit shading model as a one-object scene (identity
// placement) and the scene kernel's camera / output descriptor.
void pack_scene_job(const frt_job& jb, SceneObject& S, JobDev& camJ);
// frt_last_error() bookkeeping for entry points outside frt_api.cpp.
void set_last_error(const char* msg);
frt_status record_error(frt_status s, const char* msg);

// Writes `bytes` (a multiple of 16, at most kUploadBytes) from host memory
// to the 16-byte aligned device address dst by a kernel that carries them in
// its arguments: no staging buffer, nothing allocated (frt_noalloc.hip).
constexpr int kUploadBytes = 3072;
hipError_t launch_upload(void* dst, const void* src, int bytes, hipStream_t stream);
// The library's own device scratch on the current device (file-scope
// device array; its address is looked up once per device), and its size.
void* noalloc_scratch(hipError_t& err);
size_t noalloc_scratch_bytes();

// Point queries (frt_query.hip).
struct OrbitParams;
hipError_t launch_distance(int variant, const OrbitParams& P, const float* pts, long long n, float* d, int* it,
                           hipStream_t stream);
// Unit normals at n points by the renderer's rule for `mode` ((0, 0, 0) for
// a zero or non-finite gradient).
hipError_t launch_normal_query(int variant, const OrbitParams& P, int mode, const float* pts, const float* eps,
                               long long n, float* out, hipStream_t stream);
// One view of a scene (frt_scene.hip): objs is the device table of n_obj
// objects, cam the world camera, march and output planes.
hipError_t launch_scene(const SceneObject* objs, int n_obj, const JobDev& cam, int* object_id, float* trap,
                        hipStream_t stream);
hipError_t launch_math(int func, const float* x, const float* y, float* out, long long n, hipStream_t stream);

// Issue-rate probes of the vector unit (frt_rates.hip): `blocks` workgroups
// of kRateBlock threads, each lane running `iters` rounds of
// rate_ops_per_iter(op) lane operations; sink holds one float per thread.
enum RateOp {
    kRateFma = 0, kRateExp2, kRateLog2, kRateRsq, kRateRcp, kRateSqrt, kRateSin, kRateMix,
    kRateFAdd, kRateFMul, kRateIntShiftAdd, kNumRateOps
};
constexpr int kRateBlock = 256;
int rate_ops_per_iter(int op);
hipError_t launch_rate(int op, int iters, float* sink, int blocks, hipStream_t stream);

// Adjoint over the hit pixels of a batch (frt_adjoint.hip): zeroes the
// gradient outputs and the tile counters, then one persistent launch per
// fractal kind present (grid[kind] workgroups of 256 threads, 0 = none)
// drains the batch's 64-ray tiles.
struct AdjointArgs {
    const JobDev* jobs;        // device job table
    const AdjointJob* ajobs;   // device table of upstream-gradient pointers
    float* grad_c;             // [n_jobs][4]
    float* grad_power;         // [n_jobs]
    float* grad_plane;         // [n_jobs][2][4]
    int n_jobs;
    int grid[2];
};
hipError_t launch_adjoint(const AdjointArgs& a, WorkspaceHeader* hdr, hipStream_t stream);
const void* adjoint_kernel_symbol(int kind);

}  // namespace frt
