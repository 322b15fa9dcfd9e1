// frt_job.hpp -- device-side job descriptor, built by the host API from the
// public frt_job (camera basis, bounding radius and unit plane normals are
// precomputed once per render) and read by the kernels.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace frt {

enum Kind : int32_t { kJulia = 0, kBulb = 1 };

// kernel variants (template argument and autotuner key); a batch is split
// into one group of rays per variant present, each traced by its own kernels
enum Variant : int32_t {
    kVarJulia = 0,      // quaternion Julia z^2 + c
    kVarBulbReal = 1,   // Mandelbulb, real power (trigonometric map)
    kVarBulbInt = 2,    // Mandelbulb, integer power read at run time
    kVarBulb8 = 3,      // Mandelbulb, power 8 fixed at compile time
    kVarJuliaDeg = 4,   // quaternion Julia z^p + c, integer degree p >= 3 read at run time
    kNumVariants = 5
};

// status byte
enum : uint8_t {
    kMissBounds = 0,
    kMissTmax = 1,
    kHit = 2,
    kHitCut = 3,
    kHitExhausted = 4,
    kFlagShadowed = 8,
    kFlagUnrefined = 16,
    kFlagShadowRay = 64,   // set by the normal kernel on hits that cast a shadow ray
    kFlagReflectHit = 128, // scenes with the closest-hit shading: the reflection ray hit
};

constexpr int kCounterPlanes = 8;      // optional per-pixel work counters
constexpr int kTile = 8;               // rays are issued in 8x8 pixel tiles
constexpr int kRaysPerTile = kTile * kTile;

struct alignas(16) JobDev {
    // camera
    float eye[3];
    float fwd[3];
    float right[3];
    float upv[3];
    float sx, sy;          // s*W/H and s, s = tan(fov_y/2)
    float inv_w2, inv_h2;  // 2/W and 2/H
    int32_t width, height, tiles_x, tiles_y;
    // fractal
    int32_t kind, int_power, max_iter, n_planes;   // int_power: Julia degree, integer Mandelbulb n, or 0
    float c[4];
    float power, n_rev, bailout2, radius;   // n_rev = n / (2 pi)
    // planes (unit normals)
    float pn[2][3];
    float pd[2];
    // march / shading
    int32_t max_steps, normal_mode, refine_iters, shadow;
    float eps_abs, eps_rel, clamp, t_max;
    float light[3];
    float albedo[3];
    float k_a, k_d;
    int32_t shading;
    float k_s, shininess, k_r;
    float trap_pal[4][3];    // closest-hit shading: albedo change per unit trap component
    int32_t trap_colour;     // trap_pal has a non-zero entry
    // outputs (SoA planes of npix)
    float* depth;
    float* normal;
    float* colour;
    uint8_t* status;
    uint32_t* counters;
    int64_t npix;
    // position in the batch's ray index space (multiples of 64)
    int64_t ray_begin;
    int64_t ray_count;
    // camera basis and screen scales in FP64 (the adjoint's rays)
    double fwd_d[3];
    double right_d[3];
    double upv_d[3];
    double sx_d, sy_d;
};

// One object of a scene: its fractal, planes and march settings in object
// units (eps_abs, step_clamp and t_max divided by the scale), and the
// similarity x_obj = R^T (x - T) / s from world space (rot row-major R).
constexpr int kMaxSceneObjects = 16;
struct alignas(16) SceneObject {
    JobDev job;
    float rot[9];
    float trans[3];
    float scale, inv_scale;
    int32_t variant;
    int32_t pad[3];
};

// Gradient slots per job: c0..c3, power, plane 0 (raw n xyz, d), plane 1.
constexpr int kGradSlots = 13;

// Upstream gradients of one job for the adjoint (device pointers; any may
// be null).
struct AdjointJob {
    const float* g_colour;   // [3][P]
    const float* g_depth;    // [P]
    const float* g_normal;   // [3][P]
    float* g_pixel;          // [kGradSlots][P] per-pixel contributions (optional)
    float raw_n[2][3];       // raw plane normals (the job holds unit ones)
    int32_t out_index;       // the job's index in the caller's arrays (gradient outputs)
    int32_t pad;
};

// Workspace layout: a 1 KiB header, the job table, then the table of
// upstream-gradient pointers (AdjointJob, read by the adjoint only).  In a
// forward call the jobs are laid out in the ray index space variant by
// variant; group v holds the rays [range[v][0], range[v][1]) and drains them
// through its own counters (one for the primary march, one for the shadow
// march).  In a backward call they are laid out kind by kind (Julia, then
// Mandelbulb), and range[k] holds kind k's rays.  Either way the table is in
// ray order, so a ray's job is found by a search over ray_begin.
// Claim counters per variant and stage: one per group of workgroups (blocks
// are dealt to the XCDs in turn, so block b's group is b mod kQueueSlots),
// each on its own 256-byte line: one address serves about 80 device-scope
// atomics per microsecond, eight addresses about 540.
constexpr int kQueueSlots = 8;

struct alignas(256) WorkspaceHeader {
    unsigned long long range[kNumVariants][2];   // each group's [begin, end) in the ray index space
    unsigned long long adj_queue[2];             // tile groups claimed by the adjoint kernels (per kind)
    unsigned long long total_rays;
    int32_t n_jobs;
    int32_t pad0[(512 - 16 * kNumVariants - 28) / 4];
    // per-stage trip statistics of the march kernels, summed over their
    // waves; written only by a build with FRT_TRIP_COUNTERS defined (the host
    // zeroes the header's first KiB on every call): [stage * 16 + k], stage
    // 0 primary and 1 shadow march, k as in TripCounter
    unsigned long long trips[32];
    // index checks of a build with FRT_DEBUG_CHECKS defined: bit k set when
    // check k (CheckBit) failed somewhere; the failing item was skipped
    unsigned long long checks;
    int32_t pad1[(1024 - 512 - 256 - 8) / 4];
    // [(variant * 2 + stage) * kQueueSlots + slot][0]: chunks claimed from
    // that slot's share (stage 0 primary march, 1 shadow march)
    unsigned long long queue[kNumVariants * 2 * kQueueSlots][32];
};
enum TripCounter {
    kTripLoops = 0,      // trips round the wave's outer loop
    kTripRefills,        // trips that wrote finished rays and refilled lanes
    kTripBodyIters,      // iterations of the orbit loop (wave level)
    kTripSteps,          // trips whose step path had a lane to step
    kTripClaims,         // claim attempts on the work queue
    kTripLiveLanes,      // live lanes summed over orbit-loop iterations (orbit bodies)
    kTripStepLanes,      // lanes summed over step paths (distance estimates used)
    kTripCount,          // the counters above are sums over the waves
    // FRT_WAVE_TIMES: stamps of the 100 MHz real-time counter, each kept as
    // the latest and (complemented, so one atomic max serves) the earliest:
    // the waves' starts, their first finding the queue dry and their exits;
    // and the sum of the exit stamps and the number of waves
    kTripStartMax = kTripCount,
    kTripStartMinNot,
    kTripDrainMax,
    kTripDrainMinNot,
    kTripExitMax,
    kTripExitMinNot,
    kTripLifeSum,
    kTripWaves,
    kTripSlots
};
static_assert(kTripSlots <= 16, "each march stage has 16 trip counter slots");
enum CheckBit {
    kCheckRay = 0,     // a claimed ray index outside its group or its job
    kCheckPixel = 1,   // a pixel index outside its job's planes
    kCheckJob = 2,     // a job-table index outside the table
    kCheckList = 3,    // an LDS list or slot index outside its array
};
static_assert(offsetof(WorkspaceHeader, trips) == 512, "trip counters at byte 512 of the header");
static_assert(offsetof(WorkspaceHeader, checks) == 768, "check bits at byte 768 of the header");

// FRT_CHECK(hdr, cond, bit): true when cond holds.  In a build with
// FRT_DEBUG_CHECKS a failure sets the bit in hdr->checks (and the caller
// skips the item); otherwise the check compiles away.
#ifdef FRT_DEBUG_CHECKS
#define FRT_CHECK(hdr, cond, bit) ((cond) ? true : (atomicOr(&(hdr)->checks, 1ull << (bit)), false))
#else
#define FRT_CHECK(hdr, cond, bit) true
#endif
static_assert(sizeof(WorkspaceHeader) == 1024 + kNumVariants * 2 * kQueueSlots * 256,
              "workspace header: 1 KiB of fields, then the claim counters");

// Workspace bytes per job after the header: a job-table entry and the
// adjoint's entry, or an object-table entry for a job traced as a scene.
constexpr unsigned kWorkspaceBytesPerJob =
    sizeof(JobDev) + sizeof(AdjointJob) > sizeof(SceneObject) ? sizeof(JobDev) + sizeof(AdjointJob)
                                                               : sizeof(SceneObject);

}  // namespace frt
