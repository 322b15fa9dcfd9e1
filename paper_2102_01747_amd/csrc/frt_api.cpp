// frt_api.cpp -- host side of the C ABI declared in include/frt.h:
// argument validation, packing of public jobs into device descriptors,
// persistent-grid sizing, batch graph capture and the autotune table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "frt.h"
#include "frt_fractal.hpp"
#include "frt_internal.hpp"
#include "frt_job.hpp"

using frt::JobDev;
using frt::LaunchCfg;
using frt::WorkspaceHeader;

namespace {

thread_local std::string g_last_error;

frt_status fail(frt_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

frt_status hip_fail(hipError_t e, const char* what) {
    return fail(FRT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ----------------------------------------------------------- stage timing
// When enabled, every forward call records four events on its stream (before
// the primary march, the normal kernel and the shadow march, and after the
// last); frt_stage_times() reads the last call's stage durations.
std::mutex g_time_mu;
bool g_timing = false;
hipEvent_t g_marks[4] = {nullptr, nullptr, nullptr, nullptr};
bool g_marks_recorded = false;

hipEvent_t* timing_marks() {
    std::lock_guard<std::mutex> lk(g_time_mu);
    if (!g_timing) return nullptr;
    for (hipEvent_t& ev : g_marks)
        if (!ev && hipEventCreate(&ev) != hipSuccess) return nullptr;
    g_marks_recorded = true;
    return g_marks;
}

// ---------------------------------------------------------------- tuning
struct Tune {
    int block;
    int chunk;
    int waves_per_simd;
    int orbit_lanes;
    int rare_lanes;
};
std::mutex g_mu;
Tune g_tune[frt::kNumVariants] = {
    {64, 256, 0, 8, 16},   // Julia
    {64, 256, 0, 8, 16},   // Mandelbulb, real power
    {64, 256, 0, 8, 16},   // Mandelbulb, integer power
    {64, 256, 0, 8, 16},   // Mandelbulb, n = 8
    {64, 256, 0, 8, 16},   // Julia, degree >= 3
};

int device_cus() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

// Resident workgroups per CU of (kernel, block) on the current device,
// queried once per (kernel, block, device).
bool occupancy(const void* kernel, int block, int& per_cu, std::string& why) {
    struct OccEntry {
        const void* kernel;
        int block;
        int device;
        int per_cu;
    };
    // a fixed table: (kernel symbols x 4 block sizes x devices in use) stays
    // far below its size; when full, queries are simply not cached
    static std::mutex occ_mu;
    static OccEntry occ_cache[256];
    static int occ_n = 0;
    int dev = 0;
    (void)hipGetDevice(&dev);
    per_cu = 0;
    {
        std::lock_guard<std::mutex> lk(occ_mu);
        for (int i = 0; i < occ_n; ++i) {
            const OccEntry& o = occ_cache[i];
            if (o.kernel == kernel && o.block == block && o.device == dev) per_cu = o.per_cu;
        }
    }
    if (per_cu > 0) return true;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0);
    if (e != hipSuccess || per_cu <= 0) {
        why = std::string("occupancy query failed: ") + hipGetErrorString(e);
        return false;
    }
    std::lock_guard<std::mutex> lk(occ_mu);
    if (occ_n < 256) occ_cache[occ_n++] = OccEntry{kernel, block, dev, per_cu};
    return true;
}

bool make_cfg(const void* kernel, int variant, long long total_rays, LaunchCfg& cfg, std::string& why) {
    Tune t;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        t = g_tune[variant];
    }
    int per_cu = 0;
    if (!occupancy(kernel, t.block, per_cu, why)) return false;
    if (t.waves_per_simd > 0) {
        const int want = (t.waves_per_simd * 4 * 64) / t.block;   // 4 SIMDs per CU
        per_cu = std::max(1, std::min(per_cu, want));
    }
    // never more waves than 64-ray tiles to trace
    const long long tiles = std::max(1ll, (total_rays + 63) / 64);
    const long long waves_per_block = t.block / 64;
    const long long need = (tiles + waves_per_block - 1) / waves_per_block;
    cfg.grid = static_cast<int>(std::min<long long>(static_cast<long long>(per_cu) * device_cus(), need));
    cfg.normal_grid = static_cast<int>(std::min<long long>(8ll * device_cus(), (total_rays + 255) / 256));
    cfg.block = t.block;
    cfg.chunk = t.chunk;
    cfg.orbit_lanes = t.orbit_lanes;
    cfg.rare_lanes = t.rare_lanes;
    return true;
}

// ------------------------------------------------------------ validation
bool finite(float x) { return std::isfinite(x); }
bool finite_n(const float* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!finite(v[i])) return false;
    return true;
}
double norm3(const float* v) {
    return std::sqrt(double(v[0]) * v[0] + double(v[1]) * v[1] + double(v[2]) * v[2]);
}

bool validate(const frt_camera* cam, const frt_fractal* fr, const frt_plane* planes, int32_t n_planes,
              const frt_march* mc, const frt_frame* out, bool need_outputs, std::string& why) {
    if (!cam || !fr || !mc) { why = "null parameter block"; return false; }
    if (cam->width < 1 || cam->height < 1) { why = "width and height must be >= 1"; return false; }
    if ((long long)cam->width * cam->height > (1ll << 31) - 1) { why = "image larger than 2^31 pixels"; return false; }
    if (!finite_n(cam->eye, 3) || !finite_n(cam->target, 3) || !finite_n(cam->up, 3) || !finite(cam->fov_y_deg)) {
        why = "non-finite camera"; return false;
    }
    if (!(cam->fov_y_deg > 0.0f && cam->fov_y_deg < 180.0f)) { why = "fov_y_deg must be in (0, 180)"; return false; }
    const float f[3] = {cam->target[0] - cam->eye[0], cam->target[1] - cam->eye[1], cam->target[2] - cam->eye[2]};
    const double fl = norm3(f);
    if (!(fl > 0.0)) { why = "eye and target coincide"; return false; }
    const double c0 = double(f[1]) * cam->up[2] - double(f[2]) * cam->up[1];
    const double c1 = double(f[2]) * cam->up[0] - double(f[0]) * cam->up[2];
    const double c2 = double(f[0]) * cam->up[1] - double(f[1]) * cam->up[0];
    if (!(std::sqrt(c0 * c0 + c1 * c1 + c2 * c2) > 1e-12 * fl * norm3(cam->up))) {
        why = "up is parallel to the view direction"; return false;
    }
    if (fr->kind != FRT_JULIA && fr->kind != FRT_MANDELBULB) { why = "unknown fractal kind"; return false; }
    if (!finite_n(fr->c, 4) || !finite(fr->power) || !finite(fr->bailout2) || !finite(fr->bound_radius)) {
        why = "non-finite fractal parameter"; return false;
    }
    if (fr->max_iter < 1 || fr->max_iter > 4096) { why = "max_iter must be in [1, 4096]"; return false; }
    if (!(fr->bailout2 > 0.0f)) { why = "bailout2 must be > 0"; return false; }
    if (!(fr->bound_radius >= 0.0f)) { why = "bound_radius must be >= 0"; return false; }
    if (fr->kind == FRT_MANDELBULB && !(fr->power >= 2.0f)) { why = "Mandelbulb power must be >= 2"; return false; }
    if (fr->kind == FRT_JULIA) {
        if (!(fr->power >= 2.0f && fr->power <= 16.0f && std::floor(fr->power) == fr->power)) {
            why = "Julia degree (power) must be an integer in [2, 16]"; return false;
        }
        // the escaping body's |z|^2 is at most about bailout2^p: keep it finite in float
        if (!(double(fr->power) * std::log2(double(fr->bailout2)) <= 120.0)) {
            why = "Julia bailout2^degree must be below 2^120"; return false;
        }
    }
    if (n_planes < 0 || n_planes > 2) { why = "n_planes must be in [0, 2]"; return false; }
    if (n_planes > 0 && !planes) { why = "planes is null"; return false; }
    for (int k = 0; k < n_planes; ++k) {
        if (!finite_n(planes[k].n, 3) || !finite(planes[k].d)) { why = "non-finite plane"; return false; }
        if (!(norm3(planes[k].n) > 0.0)) { why = "plane normal is zero"; return false; }
    }
    if (mc->max_steps < 1 || mc->max_steps > 65536) { why = "max_steps must be in [1, 65536]"; return false; }
    if (!finite(mc->eps_abs) || !finite(mc->eps_rel) || !finite(mc->step_clamp) || !finite(mc->t_max) ||
        !finite_n(mc->light_dir, 3) || !finite_n(mc->albedo, 3) || !finite(mc->k_ambient) || !finite(mc->k_diffuse)) {
        why = "non-finite march parameter"; return false;
    }
    if (mc->eps_abs < 0.0f || mc->eps_rel < 0.0f || (mc->eps_abs == 0.0f && mc->eps_rel == 0.0f)) {
        why = "eps_abs and eps_rel must be >= 0 and not both 0"; return false;
    }
    if (!(mc->step_clamp > 0.0f)) { why = "step_clamp must be > 0"; return false; }
    if (!(mc->t_max > mc->eps_abs)) { why = "t_max must exceed eps_abs"; return false; }
    if (mc->normal_mode != FRT_NORMAL_TETRA && mc->normal_mode != FRT_NORMAL_CENTRAL &&
        mc->normal_mode != FRT_NORMAL_ANALYTIC) {
        why = "unknown normal_mode"; return false;
    }
    if (mc->refine_iters < 0 || mc->refine_iters > 32) { why = "refine_iters must be in [0, 32]"; return false; }
    if (mc->shadow != 0 && mc->shadow != 1) { why = "shadow must be 0 or 1"; return false; }
    if (!(norm3(mc->light_dir) > 0.0)) { why = "light_dir is zero"; return false; }
    if (mc->shading != FRT_SHADING_LAMBERT && mc->shading != FRT_SHADING_PHONG) {
        why = "unknown shading model"; return false;
    }
    if (mc->shading == FRT_SHADING_PHONG) {
        if (!(mc->k_specular >= 0.0f && mc->k_specular <= 1e30f)) {
            why = "k_specular must be finite and >= 0"; return false;
        }
        if (!(mc->shininess >= 1.0f && mc->shininess <= 1e4f)) { why = "shininess must be in [1, 10000]"; return false; }
        if (!(mc->k_reflect >= 0.0f && mc->k_reflect <= 1.0f)) { why = "k_reflect must be in [0, 1]"; return false; }
        if (!finite_n(&mc->trap_colour[0][0], 12)) { why = "non-finite trap_colour"; return false; }
    }
    if (need_outputs) {
        if (!out || !out->depth || !out->normal || !out->colour || !out->status) {
            why = "null output plane"; return false;
        }
    }
    return true;
}

// --------------------------------------------------------------- packing
int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// The integer power a kernel variant may use: the Julia degree, an integral
// Mandelbulb n in [2, 64], or 0 (real n).
int int_power_of(const frt_fractal* fr) {
    if (fr->kind == FRT_JULIA) return int(fr->power);
    const float ip = std::floor(fr->power);
    return (ip == fr->power && ip >= 2.0f && ip <= 64.0f) ? int(ip) : 0;
}

int variant_of_frac(const frt_fractal* fr) {
    const int ip = int_power_of(fr);
    if (fr->kind == FRT_JULIA) return ip == 2 ? frt::kVarJulia : frt::kVarJuliaDeg;
    if (ip == 8) return frt::kVarBulb8;
    return ip > 0 ? frt::kVarBulbInt : frt::kVarBulbReal;
}

// Rays of one render in the ray index space: whole 8x8 tiles.
int64_t ray_count_of(const frt_camera* cam) {
    const int64_t tx = (cam->width + frt::kTile - 1) / frt::kTile, ty = (cam->height + frt::kTile - 1) / frt::kTile;
    return tx * ty * frt::kRaysPerTile;
}

void pack(const frt_camera* cam, const frt_fractal* fr, const frt_plane* planes, int32_t n_planes,
          const frt_march* mc, const frt_frame& out, int64_t ray_begin, JobDev& J) {
    std::memset(&J, 0, sizeof(J));
    // camera basis in double, rounded once
    double f[3] = {double(cam->target[0]) - cam->eye[0], double(cam->target[1]) - cam->eye[1],
                   double(cam->target[2]) - cam->eye[2]};
    double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    for (double& v : f) v /= fl;
    double r[3] = {f[1] * cam->up[2] - f[2] * cam->up[1], f[2] * cam->up[0] - f[0] * cam->up[2],
                   f[0] * cam->up[1] - f[1] * cam->up[0]};
    double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    for (double& v : r) v /= rl;
    const double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    const double s = std::tan(0.5 * double(cam->fov_y_deg) * M_PI / 180.0);
    for (int k = 0; k < 3; ++k) {
        J.eye[k] = cam->eye[k];
        J.fwd[k] = float(f[k]);
        J.right[k] = float(r[k]);
        J.upv[k] = float(u[k]);
        J.fwd_d[k] = f[k];
        J.right_d[k] = r[k];
        J.upv_d[k] = u[k];
    }
    J.sx = float(s * cam->width / cam->height);
    J.sy = float(s);
    J.sx_d = s * cam->width / cam->height;
    J.sy_d = s;
    J.inv_w2 = float(2.0 / cam->width);
    J.inv_h2 = float(2.0 / cam->height);
    J.width = cam->width;
    J.height = cam->height;
    J.tiles_x = (cam->width + frt::kTile - 1) / frt::kTile;
    J.tiles_y = (cam->height + frt::kTile - 1) / frt::kTile;
    // fractal
    J.kind = fr->kind;
    J.max_iter = fr->max_iter;
    J.bailout2 = fr->bailout2;
    for (int k = 0; k < 4; ++k) J.c[k] = fr->kind == FRT_JULIA ? fr->c[k] : 0.0f;
    double R;
    if (fr->kind == FRT_JULIA) {
        // degree p: the escape radius is the root R >= 1 of R^p - R - |c|
        const int p = int_power_of(fr);
        J.power = float(p);
        J.int_power = p;
        const double cn = std::sqrt(double(fr->c[0]) * fr->c[0] + double(fr->c[1]) * fr->c[1] +
                                    double(fr->c[2]) * fr->c[2] + double(fr->c[3]) * fr->c[3]);
        if (p == 2) {
            R = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * cn));
        } else {
            // Newton from the right of the root: the polynomial is convex and
            // increasing there, so the iterates decrease monotonically onto it
            R = 2.0 + cn;
            for (int it = 0; it < 100; ++it) {
                const double rp1 = std::pow(R, p - 1);
                const double step = (rp1 * R - R - cn) / (p * rp1 - 1.0);
                if (!(step > 0.0)) break;
                R -= step;
            }
        }
    } else {
        J.power = fr->power;
        R = std::pow(2.0, 1.0 / (double(fr->power) - 1.0));
        J.int_power = int_power_of(fr);
    }
    R = std::max(R, double(fr->bound_radius));
    J.radius = float(R);
    J.n_rev = float(double(J.power) / (2.0 * M_PI));
    // planes
    J.n_planes = n_planes;
    for (int k = 0; k < n_planes; ++k) {
        const double l = norm3(planes[k].n);
        for (int e = 0; e < 3; ++e) J.pn[k][e] = float(planes[k].n[e] / l);
        J.pd[k] = planes[k].d;
    }
    // march / shading
    J.max_steps = mc->max_steps;
    J.normal_mode = mc->normal_mode;
    J.refine_iters = mc->refine_iters;
    J.shadow = mc->shadow;
    J.eps_abs = mc->eps_abs;
    J.eps_rel = mc->eps_rel;
    J.clamp = mc->step_clamp;
    J.t_max = mc->t_max;
    const double ll = norm3(mc->light_dir);
    for (int k = 0; k < 3; ++k) {
        J.light[k] = float(mc->light_dir[k] / ll);
        J.albedo[k] = mc->albedo[k];
    }
    J.k_a = mc->k_ambient;
    J.k_d = mc->k_diffuse;
    J.shading = mc->shading;
    J.k_s = mc->k_specular;
    J.shininess = mc->shininess;
    J.k_r = mc->k_reflect;
    J.trap_colour = 0;
    if (mc->shading == FRT_SHADING_PHONG) {
        for (int k = 0; k < 4; ++k)
            for (int c = 0; c < 3; ++c) {
                J.trap_pal[k][c] = mc->trap_colour[k][c];
                if (mc->trap_colour[k][c] != 0.0f) J.trap_colour = 1;
            }
    }
    // outputs
    J.depth = out.depth;
    J.normal = out.normal;
    J.colour = out.colour;
    J.status = out.status;
    J.counters = out.counters;
    J.npix = int64_t(cam->width) * cam->height;
    J.ray_begin = ray_begin;
    J.ray_count = ray_count_of(cam);
}

int variant_of(const JobDev& J) {
    if (J.kind == FRT_JULIA) return J.int_power == 2 ? frt::kVarJulia : frt::kVarJuliaDeg;
    if (J.int_power == 8) return frt::kVarBulb8;
    return J.int_power > 0 ? frt::kVarBulbInt : frt::kVarBulbReal;
}

// ----------------------------------------------------- staging and graphs
// Pinned host buffers for the job-table uploads, used in turn: a call waits
// only when the upload of the call kStageSlots calls before it (which used
// the same buffer) has not been copied yet.
struct Staging {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;   // recorded after the last upload from `host`
    bool pending = false;
};
constexpr int kStageSlots = 8;
// first size of a staging buffer: the header and a few dozen jobs with their
// adjoint entries
constexpr size_t kStageMinBytes = size_t(64) << 10;
std::mutex g_stage_mu;
Staging g_stage[kStageSlots];
int g_stage_next = 0;

struct GraphEntry {
    void* workspace;
    std::vector<frt::TraceGroup> groups;
    int device;
    hipGraphExec_t exec;
};

bool same_groups(const std::vector<frt::TraceGroup>& a, const std::vector<frt::TraceGroup>& b) {
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i) {
        const LaunchCfg &x = a[i].cfg, &y = b[i].cfg;
        if (a[i].variant != b[i].variant || a[i].any_shadow != b[i].any_shadow || x.grid != y.grid ||
            x.normal_grid != y.normal_grid || x.block != y.block || x.chunk != y.chunk ||
            x.orbit_lanes != y.orbit_lanes || x.rare_lanes != y.rare_lanes)
            return false;
    }
    return true;
}
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;
hipStream_t g_capture_stream = nullptr;

// Copy consecutive host blocks into the start of the workspace through the
// next pinned staging buffer of the ring.
frt_status upload_parts(const void* const* parts, const size_t* sizes, int n_parts, void* workspace,
                        hipStream_t stream) {
    size_t bytes = 0;
    for (int i = 0; i < n_parts; ++i) bytes += sizes[i];
    std::lock_guard<std::mutex> lk(g_stage_mu);
    Staging& sg = g_stage[g_stage_next];
    g_stage_next = (g_stage_next + 1) % kStageSlots;
    hipError_t e;
    if (sg.pending) {
        e = hipEventSynchronize(sg.done);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        sg.pending = false;
    }
    if (sg.bytes < bytes) {
        // grow by powers of two from kStageMinBytes: freeing pinned memory
        // waits for the device, so a slot should rarely need it again
        size_t cap = kStageMinBytes;
        while (cap < bytes) cap *= 2;
        if (sg.host) (void)hipHostFree(sg.host);
        sg.host = nullptr;
        sg.bytes = 0;
        e = hipHostMalloc(&sg.host, cap, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
        sg.bytes = cap;
    }
    if (!sg.done) {
        e = hipEventCreateWithFlags(&sg.done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    size_t off = 0;
    for (int i = 0; i < n_parts; ++i) {
        if (sizes[i]) std::memcpy(static_cast<char*>(sg.host) + off, parts[i], sizes[i]);
        off += sizes[i];
    }
    e = hipMemcpyAsync(workspace, sg.host, bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipEventRecord(sg.done, stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    sg.pending = true;
    return FRT_OK;
}

// Header + job table (+ the adjoint's table, if given).
frt_status upload_table(const std::vector<JobDev>& jobs, const WorkspaceHeader& hdr, void* workspace,
                        hipStream_t stream, const std::vector<frt::AdjointJob>* ajobs = nullptr) {
    const void* parts[3] = {&hdr, jobs.data(), ajobs ? static_cast<const void*>(ajobs->data()) : nullptr};
    const size_t sizes[3] = {sizeof(hdr), jobs.size() * sizeof(JobDev),
                             ajobs ? ajobs->size() * sizeof(frt::AdjointJob) : 0};
    return upload_parts(parts, sizes, 3, workspace, stream);
}

frt_status check_workspace(void* workspace, size_t ws_bytes, int32_t n_jobs) {
    if (!workspace) return fail(FRT_EINVAL, "workspace is null");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(FRT_EINVAL, "workspace not 256-byte aligned");
    if (ws_bytes < frt_workspace_bytes(n_jobs)) return fail(FRT_ENOMEM, "workspace too small");
    return FRT_OK;
}

}  // namespace

namespace frt {

namespace {
// side streams and their fork/join events, per device
struct SideSet {
    hipStream_t s[kSideStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSideStreams] = {};
    bool ready = false;
};
std::mutex g_side_mu;
SideSet g_side[64];

hipError_t side_set(SideSet*& out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    SideSet& ss = g_side[dev];
    if (!ss.ready) {
        for (int k = 0; k < kSideStreams; ++k) {
            e = hipStreamCreateWithFlags(&ss.s[k], hipStreamNonBlocking);
            if (e != hipSuccess) return e;
            e = hipEventCreateWithFlags(&ss.join[k], hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        e = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming);
        if (e != hipSuccess) return e;
        ss.ready = true;
    }
    out = &ss;
    return hipSuccess;
}
}  // namespace

hipError_t fork_streams(hipStream_t main, int n, hipStream_t* side) {
    if (n < 1 || n > kSideStreams) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lk(g_side_mu);
    SideSet* ss = nullptr;
    hipError_t e = side_set(ss);
    if (e != hipSuccess) return e;
    e = hipEventRecord(ss->fork, main);
    for (int k = 0; k < n && e == hipSuccess; ++k) {
        e = hipStreamWaitEvent(ss->s[k], ss->fork, 0);
        side[k] = ss->s[k];
    }
    return e;
}

hipError_t join_streams(hipStream_t main, int n) {
    if (n < 1 || n > kSideStreams) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lk(g_side_mu);
    SideSet* ss = nullptr;
    hipError_t e = side_set(ss);
    if (e != hipSuccess) return e;
    for (int k = 0; k < n && e == hipSuccess; ++k) {
        e = hipEventRecord(ss->join[k], ss->s[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(main, ss->join[k], 0);
    }
    return e;
}

void set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }

frt_status record_error(frt_status s, const char* msg) { return fail(s, msg ? msg : ""); }

frt_status batch_validate(const frt_job* jobs, int32_t n_jobs, bool allow_closest_hit) {
    for (int i = 0; i < n_jobs; ++i) {
        std::string why;
        const frt_job& jb = jobs[i];
        if (!validate(&jb.cam, &jb.frac, jb.planes, jb.n_planes, &jb.march, &jb.out, true, why))
            return fail(FRT_EINVAL, "job " + std::to_string(i) + ": " + why);
        if (jb.march.shading != FRT_SHADING_LAMBERT && !allow_closest_hit)
            return fail(FRT_EUNSUPPORTED, "job " + std::to_string(i) +
                                              ": the closest-hit shading model is not served by this entry point");
    }
    return FRT_OK;
}

frt_status batch_layout(const frt_job* jobs, int32_t n_jobs, WorkspaceHeader& hdr, TraceGroup* groups, int& n_groups,
                        bool (*sink)(void* ctx, const JobDev& J), void* ctx, bool closest_hit_elsewhere) {
    n_groups = 0;
    // every job is validated before anything is packed or launched; jobs
    // with the closest-hit shading model are left to the caller
    frt_status vs = batch_validate(jobs, n_jobs, closest_hit_elsewhere);
    if (vs != FRT_OK) return vs;
    int n_table = 0;
    // lay the rays out variant by variant: group v is one contiguous range of
    // the ray index space traced by its own kernels (the table order is
    // internal; outputs travel with each job)
    std::memset(&hdr, 0, sizeof(hdr));
    int64_t begin = 0;
    for (int v = 0; v < kNumVariants; ++v) {
        const int64_t g0 = begin;
        bool shadow = false;
        for (int i = 0; i < n_jobs; ++i) {
            const frt_job& jb = jobs[i];
            if (variant_of_frac(&jb.frac) != v || jb.march.shading != FRT_SHADING_LAMBERT) continue;
            ++n_table;
            JobDev J;
            pack(&jb.cam, &jb.frac, jb.planes, jb.n_planes, &jb.march, jb.out, begin, J);
            begin += J.ray_count;
            shadow = shadow || J.shadow != 0;
            if (!sink(ctx, J)) return fail(FRT_EHIP, "job table upload failed");
        }
        hdr.range[v][0] = static_cast<unsigned long long>(g0);
        hdr.range[v][1] = static_cast<unsigned long long>(begin);
        if (begin == g0) continue;
        TraceGroup& g = groups[n_groups++];
        g.variant = v;
        g.any_shadow = shadow;
        std::string why;
        if (!make_cfg(trace_kernel_symbol(v, true), v, begin - g0, g.cfg, why)) return fail(FRT_EHIP, why);
    }
    hdr.total_rays = static_cast<unsigned long long>(begin);
    hdr.n_jobs = n_table;
    return FRT_OK;
}

// A job with the closest-hit shading model as a one-object scene: the
// object placed by the identity, the job's camera, march and outputs.
void pack_scene_job(const frt_job& jb, SceneObject& S, JobDev& camJ) {
    std::memset(&S, 0, sizeof(S));
    frt_frame none{};
    pack(&jb.cam, &jb.frac, jb.planes, jb.n_planes, &jb.march, none, 0, S.job);
    S.rot[0] = S.rot[4] = S.rot[8] = 1.0f;
    S.scale = 1.0f;
    S.inv_scale = 1.0f;
    S.variant = variant_of(S.job);
    pack(&jb.cam, &jb.frac, jb.planes, jb.n_planes, &jb.march, jb.out, 0, camJ);
}

}  // namespace frt

// ======================================================================
extern "C" {

size_t frt_workspace_bytes(int32_t n_jobs) {
    if (n_jobs < 1) n_jobs = 1;
    const int64_t per_job = int64_t(frt::kWorkspaceBytesPerJob);
    return size_t(round_up(int64_t(sizeof(WorkspaceHeader)) + int64_t(n_jobs) * per_job, 256));
}

size_t frt_scene_workspace_bytes(int32_t n_objects) {
    if (n_objects < 1) n_objects = 1;
    return size_t(round_up(int64_t(sizeof(WorkspaceHeader)) + int64_t(n_objects) * int64_t(sizeof(frt::SceneObject)),
                           256));
}

frt_status frt_render_scene(const frt_camera* cam, const frt_object* objects, int32_t n_objects,
                            const frt_march* march, frt_frame out, int32_t* object_id, float* trap,
                            void* workspace, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    if (!objects || n_objects < 1 || n_objects > frt::kMaxSceneObjects)
        return fail(FRT_EINVAL, "n_objects must be in [1, 16] with a non-null table");
    std::string why;
    const frt_object& o0 = objects[0];
    if (!validate(cam, &o0.frac, o0.planes, o0.n_planes, march, &out, true, why)) return fail(FRT_EINVAL, why);
    if (!workspace) return fail(FRT_EINVAL, "workspace is null");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(FRT_EINVAL, "workspace not 256-byte aligned");
    if (ws_bytes < frt_scene_workspace_bytes(n_objects)) return fail(FRT_ENOMEM, "workspace too small");
    std::vector<frt::SceneObject> table(static_cast<size_t>(n_objects));
    for (int k = 0; k < n_objects; ++k) {
        const frt_object& ob = objects[k];
        const std::string tag = "object " + std::to_string(k) + ": ";
        if (!finite_n(ob.rotation, 9) || !finite_n(ob.translation, 3) || !finite(ob.scale))
            return fail(FRT_EINVAL, tag + "non-finite transform");
        if (!(ob.scale > 0.0f)) return fail(FRT_EINVAL, tag + "scale must be > 0");
        // R must be a rotation: R R^T = I (to float accuracy) and det R = +1
        const float* R = ob.rotation;
        double worst = 0.0;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double d = 0.0;
                for (int i = 0; i < 3; ++i) d += double(R[3 * r + i]) * R[3 * c + i];
                worst = std::max(worst, std::fabs(d - (r == c ? 1.0 : 0.0)));
            }
        const double det = double(R[0]) * (double(R[4]) * R[8] - double(R[5]) * R[7]) -
                           double(R[1]) * (double(R[3]) * R[8] - double(R[5]) * R[6]) +
                           double(R[2]) * (double(R[3]) * R[7] - double(R[4]) * R[6]);
        if (!(worst <= 1e-4 && det > 0.0)) return fail(FRT_EINVAL, tag + "rotation is not a proper rotation");
        const double sc = ob.scale;
        frt_march mo = *march;
        mo.eps_abs = float(double(march->eps_abs) / sc);
        mo.step_clamp = float(double(march->step_clamp) / sc);
        mo.t_max = float(double(march->t_max) / sc);
        if (!validate(cam, &ob.frac, ob.planes, ob.n_planes, &mo, nullptr, false, why))
            return fail(FRT_EINVAL, tag + why);
        frt::SceneObject& S = table[size_t(k)];
        std::memset(&S, 0, sizeof(S));
        frt_frame none{};
        pack(cam, &ob.frac, ob.planes, ob.n_planes, &mo, none, 0, S.job);
        for (int i = 0; i < 9; ++i) S.rot[i] = R[i];
        for (int i = 0; i < 3; ++i) S.trans[i] = ob.translation[i];
        S.scale = ob.scale;
        S.inv_scale = float(1.0 / sc);
        S.variant = variant_of(S.job);
    }
    JobDev camJ;
    pack(cam, &o0.frac, o0.planes, o0.n_planes, march, out, 0, camJ);
    WorkspaceHeader hdr;
    std::memset(&hdr, 0, sizeof(hdr));
    hdr.n_jobs = n_objects;
    const void* parts[2] = {&hdr, table.data()};
    const size_t sizes[2] = {sizeof(hdr), table.size() * sizeof(frt::SceneObject)};
    hipStream_t st = static_cast<hipStream_t>(stream);
    frt_status s = upload_parts(parts, sizes, 2, workspace, st);
    if (s != FRT_OK) return s;
    const auto* objs = reinterpret_cast<const frt::SceneObject*>(static_cast<char*>(workspace) + sizeof(hdr));
    hipError_t e = frt::launch_scene(objs, n_objects, camJ, object_id, trap, st);
    if (e != hipSuccess) return hip_fail(e, "scene launch");
    return FRT_OK;
}

frt_status frt_render(const frt_camera* cam, const frt_fractal* frac, const frt_plane* planes, int32_t n_planes,
                      const frt_march* march, frt_frame out, void* workspace, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    std::string why;
    if (!validate(cam, frac, planes, n_planes, march, &out, true, why)) return fail(FRT_EINVAL, why);
    frt_status s = check_workspace(workspace, ws_bytes, 1);
    if (s != FRT_OK) return s;
    if (march->shading != FRT_SHADING_LAMBERT) {
        // the closest-hit model: a one-object scene with the identity placement
        frt_job jb;
        std::memset(&jb, 0, sizeof(jb));
        jb.cam = *cam;
        jb.frac = *frac;
        for (int k = 0; k < n_planes; ++k) jb.planes[k] = planes[k];
        jb.n_planes = n_planes;
        jb.march = *march;
        jb.out = out;
        frt::SceneObject S;
        JobDev camJ;
        frt::pack_scene_job(jb, S, camJ);
        WorkspaceHeader hdr;
        std::memset(&hdr, 0, sizeof(hdr));
        const void* parts[2] = {&hdr, &S};
        const size_t sizes[2] = {sizeof(hdr), sizeof(S)};
        hipStream_t st = static_cast<hipStream_t>(stream);
        s = upload_parts(parts, sizes, 2, workspace, st);
        if (s != FRT_OK) return s;
        const auto* objs = reinterpret_cast<const frt::SceneObject*>(static_cast<char*>(workspace) + sizeof(hdr));
        hipError_t e = frt::launch_scene(objs, 1, camJ, nullptr, nullptr, st);
        if (e != hipSuccess) return hip_fail(e, "scene launch");
        return FRT_OK;
    }
    JobDev J;
    pack(cam, frac, planes, n_planes, march, out, 0, J);
    frt::TraceGroup g;
    g.variant = variant_of(J);
    g.any_shadow = J.shadow != 0;
    if (!make_cfg(frt::trace_kernel_symbol(g.variant, false), g.variant, J.ray_count, g.cfg, why))
        return fail(FRT_EHIP, why);
    hipError_t e = frt::launch_trace(&g, 1, false, nullptr, J, static_cast<WorkspaceHeader*>(workspace),
                                     static_cast<hipStream_t>(stream), timing_marks());
    if (e != hipSuccess) return hip_fail(e, "trace launch");
    return FRT_OK;
}

frt_status frt_render_batch(const frt_job* jobs, int32_t n_jobs, void* workspace, size_t ws_bytes, int32_t use_graph,
                            void* stream) {
    g_last_error.clear();
    if (!jobs || n_jobs < 1) return fail(FRT_EINVAL, "jobs is null or n_jobs < 1");
    if (use_graph != 0 && use_graph != 1) return fail(FRT_EINVAL, "use_graph must be 0 or 1");
    frt_status s = check_workspace(workspace, ws_bytes, n_jobs);
    if (s != FRT_OK) return s;
    WorkspaceHeader hdr;
    std::vector<JobDev> table;
    table.reserve(size_t(n_jobs));
    frt::TraceGroup group_arr[frt::kNumVariants];
    int ng = 0;
    auto push = [](void* ctx, const JobDev& J) {
        static_cast<std::vector<JobDev>*>(ctx)->push_back(J);
        return true;
    };
    // Lambert jobs go to the persistent trace; jobs with the closest-hit
    // model are traced as one-object scenes, their objects after the table
    s = frt::batch_layout(jobs, n_jobs, hdr, group_arr, ng, push, &table, true);
    if (s != FRT_OK) return s;
    std::vector<frt::SceneObject> sobj;
    std::vector<JobDev> scam;
    for (int i = 0; i < n_jobs; ++i) {
        if (jobs[i].march.shading == FRT_SHADING_LAMBERT) continue;
        sobj.emplace_back();
        scam.emplace_back();
        frt::pack_scene_job(jobs[i], sobj.back(), scam.back());
    }
    std::vector<frt::TraceGroup> groups(group_arr, group_arr + ng);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const void* parts[3] = {&hdr, table.data(), sobj.data()};
    const size_t sizes[3] = {sizeof(hdr), table.size() * sizeof(JobDev), sobj.size() * sizeof(frt::SceneObject)};
    s = upload_parts(parts, sizes, 3, workspace, st);
    if (s != FRT_OK) return s;
    char* base = static_cast<char*>(workspace);
    const JobDev* dev_jobs = reinterpret_cast<const JobDev*>(base + sizeof(WorkspaceHeader));
    const auto* dev_objs =
        reinterpret_cast<const frt::SceneObject*>(base + sizeof(WorkspaceHeader) + table.size() * sizeof(JobDev));
    WorkspaceHeader* dhdr = static_cast<WorkspaceHeader*>(workspace);
    auto scenes = [&]() -> frt_status {
        for (size_t k = 0; k < sobj.size(); ++k) {
            hipError_t e = frt::launch_scene(dev_objs + k, 1, scam[k], nullptr, nullptr, st);
            if (e != hipSuccess) return hip_fail(e, "scene launch");
        }
        return FRT_OK;
    };
    if (ng == 0) return scenes();
    if (!use_graph) {
        hipError_t e = frt::launch_trace(groups.data(), ng, true, dev_jobs, table[0], dhdr, st, timing_marks(), true);
        if (e != hipSuccess) return hip_fail(e, "trace launch");
        return scenes();
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_graph_mu);
    hipGraphExec_t exec = nullptr;
    for (const GraphEntry& g : g_graphs) {
        if (g.workspace == workspace && g.device == dev && same_groups(g.groups, groups)) {
            exec = g.exec;
            break;
        }
    }
    hipError_t e;
    if (!exec) {
        if (!g_capture_stream) {
            e = hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
        }
        e = hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipError_t le = frt::launch_trace(groups.data(), ng, true, dev_jobs, table[0], dhdr, g_capture_stream);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(g_capture_stream, &graph);
        if (le != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(le, "trace launch during capture");
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        g_graphs.push_back(GraphEntry{workspace, groups, dev, exec});
    }
    e = hipGraphLaunch(exec, st);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return scenes();
}

size_t frt_noalloc_scratch_bytes(void) { return frt::noalloc_scratch_bytes(); }

frt_status frt_render_batch_noalloc(const frt_job* jobs, int32_t n_jobs, void* stream) {
    g_last_error.clear();
    if (!jobs || n_jobs < 1) return fail(FRT_EINVAL, "jobs is null or n_jobs < 1");
    if (n_jobs > FRT_NOALLOC_MAX_JOBS) return fail(FRT_EINVAL, "n_jobs exceeds FRT_NOALLOC_MAX_JOBS");
    // every job is checked before the first device call
    frt_status vs = frt::batch_validate(jobs, n_jobs, false);
    if (vs != FRT_OK) return vs;
    hipError_t he = hipSuccess;
    char* ws = static_cast<char*>(frt::noalloc_scratch(he));
    if (!ws) return hip_fail(he, "scratch address");
    if (frt::noalloc_scratch_bytes() < frt_workspace_bytes(n_jobs)) return fail(FRT_ENOMEM, "scratch too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the job table is written into the scratch through argument-carried
    // uploads of a few jobs each, in table order, as the layout packs it
    struct Sink {
        hipStream_t st;
        char* dst;
        hipError_t err;
        int fill;
        JobDev first;
        bool have_first;
        alignas(16) unsigned char buf[frt::kUploadBytes];
        bool flush() {
            if (fill > 0) err = frt::launch_upload(dst, buf, fill, st);
            dst += fill;
            fill = 0;
            return err == hipSuccess;
        }
    } sk;
    sk.st = st;
    sk.dst = ws + sizeof(WorkspaceHeader);
    sk.err = hipSuccess;
    sk.fill = 0;
    sk.have_first = false;
    static_assert(sizeof(JobDev) % 16 == 0 && sizeof(JobDev) <= frt::kUploadBytes, "job upload granularity");
    auto put = [](void* ctx, const JobDev& J) {
        Sink& k = *static_cast<Sink*>(ctx);
        if (!k.have_first) {
            k.first = J;
            k.have_first = true;
        }
        if (k.fill + int(sizeof(JobDev)) > frt::kUploadBytes && !k.flush()) return false;
        std::memcpy(k.buf + k.fill, &J, sizeof(JobDev));
        k.fill += int(sizeof(JobDev));
        return true;
    };
    WorkspaceHeader hdr;
    frt::TraceGroup groups[frt::kNumVariants];
    int ng = 0;
    frt_status s = frt::batch_layout(jobs, n_jobs, hdr, groups, ng, put, &sk, false);
    if (s != FRT_OK) return s;
    if (!sk.flush()) return hip_fail(sk.err, "job table upload");
    // the header's fields (its first KiB; the claim counters after them are
    // zeroed by the trace launch's reset kernel)
    static_assert(offsetof(WorkspaceHeader, queue) == 1024, "header fields fit one KiB");
    hipError_t e = frt::launch_upload(ws, &hdr, 1024, st);
    if (e != hipSuccess) return hip_fail(e, "header upload");
    e = frt::launch_trace(groups, ng, true, reinterpret_cast<const JobDev*>(ws + sizeof(WorkspaceHeader)), sk.first,
                          reinterpret_cast<WorkspaceHeader*>(ws), st, nullptr);
    if (e != hipSuccess) return hip_fail(e, "trace launch");
    return FRT_OK;
}

// Orbit parameters and kernel variant of a fractal for the point queries
// (validated with a placeholder camera and march).
static bool query_params(const frt_fractal* frac, frt::OrbitParams& P, int& variant, std::string& why) {
    frt_camera cam{};
    cam.eye[2] = 1.0f;
    cam.up[1] = 1.0f;
    cam.fov_y_deg = 45.0f;
    cam.width = cam.height = 1;
    frt_march mc{};
    mc.max_steps = 1;
    mc.eps_abs = 1.0f;
    mc.step_clamp = 1.0f;
    mc.t_max = 2.0f;
    mc.light_dir[1] = 1.0f;
    if (!validate(&cam, frac, nullptr, 0, &mc, nullptr, false, why)) return false;
    frt_frame none{};
    JobDev J;
    pack(&cam, frac, nullptr, 0, &mc, none, 0, J);
    P.c0 = J.c[0]; P.c1 = J.c[1]; P.c2 = J.c[2]; P.c3 = J.c[3];
    P.n = J.power;
    P.nm1_half = 0.5f * (J.power - 1.0f);
    P.n_rev = J.n_rev;
    P.ipow = J.int_power;
    P.kind = J.kind;
    P.max_iter = J.max_iter;
    P.bail2 = J.bailout2;
    variant = variant_of(J);
    return true;
}

frt_status frt_distance(const frt_fractal* frac, const float* points, int64_t n, float* d, int32_t* iters,
                        void* stream) {
    g_last_error.clear();
    if (!frac) return fail(FRT_EINVAL, "null fractal");
    if (n < 0) return fail(FRT_EINVAL, "n must be >= 0");
    if (n == 0) return FRT_OK;
    if (!points || !d) return fail(FRT_EINVAL, "null points or output");
    std::string why;
    frt::OrbitParams P;
    int variant = 0;
    if (!query_params(frac, P, variant, why)) return fail(FRT_EINVAL, why);
    hipError_t e = frt::launch_distance(variant, P, points, n, d, iters, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "distance launch");
    return FRT_OK;
}

frt_status frt_normal_at(const frt_fractal* frac, int32_t normal_mode, const float* points, const float* eps,
                         int64_t n, float* normals, void* stream) {
    g_last_error.clear();
    if (!frac) return fail(FRT_EINVAL, "null fractal");
    if (normal_mode != FRT_NORMAL_TETRA && normal_mode != FRT_NORMAL_CENTRAL && normal_mode != FRT_NORMAL_ANALYTIC)
        return fail(FRT_EINVAL, "unknown normal_mode");
    if (n < 0) return fail(FRT_EINVAL, "n must be >= 0");
    if (n == 0) return FRT_OK;
    if (!points || !normals) return fail(FRT_EINVAL, "null points or output");
    if (!eps && normal_mode != FRT_NORMAL_ANALYTIC) return fail(FRT_EINVAL, "the tap modes need eps");
    std::string why;
    frt::OrbitParams P;
    int variant = 0;
    if (!query_params(frac, P, variant, why)) return fail(FRT_EINVAL, why);
    hipError_t e = frt::launch_normal_query(variant, P, normal_mode, points, eps, n, normals,
                                            static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "normal launch");
    return FRT_OK;
}

frt_status frt_math_eval(int32_t func, const float* x, const float* y, float* out, int64_t n, void* stream) {
    g_last_error.clear();
    if (func < 0 || func > 7) return fail(FRT_EINVAL, "func must be in [0, 7]");
    if (n < 0) return fail(FRT_EINVAL, "n must be >= 0");
    if (n == 0) return FRT_OK;
    if (!x || !out || (func == 1 && !y)) return fail(FRT_EINVAL, "null input or output");
    hipError_t e = frt::launch_math(func, x, y, out, n, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "math launch");
    return FRT_OK;
}

frt_status frt_valu_rate(int32_t op, int32_t iters, double* lane_ops_per_s, void* stream) {
    g_last_error.clear();
    if (op < 0 || op >= frt::kNumRateOps) return fail(FRT_EINVAL, "op must be in [0, 10]");
    if (iters < 1 || iters > (1 << 20)) return fail(FRT_EINVAL, "iters must be in [1, 1 << 20]");
    if (!lane_ops_per_s) return fail(FRT_EINVAL, "null output");
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    // 8 workgroups of 4 waves per CU: 8 waves on each of its 4 SIMDs
    const int blocks = 8 * cus;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    float* sink = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    float ms = 0.0f;
    e = hipMalloc(&sink, size_t(blocks) * frt::kRateBlock * sizeof(float));
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) e = frt::launch_rate(op, iters, sink, blocks, s);
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = frt::launch_rate(op, iters, sink, blocks, s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    const hipError_t first = e;
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (sink) {
        const hipError_t ef = hipFree(sink);
        if (e == hipSuccess) e = ef;
    }
    if (first != hipSuccess || e != hipSuccess) return hip_fail(first != hipSuccess ? first : e, "rate probe");
    if (!(ms > 0.0f)) return fail(FRT_EHIP, "rate probe: zero elapsed time");
    const double ops = double(blocks) * frt::kRateBlock * double(iters) * frt::rate_ops_per_iter(op);
    *lane_ops_per_s = ops / (double(ms) * 1e-3);
    return FRT_OK;
}

frt_status frt_render_backward(const frt_job* jobs, int32_t n_jobs, const float* const* g_colour,
                               const float* const* g_depth, const float* const* g_normal,
                               float* const* grad_pixel, float* grad_c,
                               float* grad_power, float* grad_plane, void* workspace, size_t ws_bytes,
                               void* stream) {
    g_last_error.clear();
    if (!jobs || n_jobs < 1) return fail(FRT_EINVAL, "jobs is null or n_jobs < 1");
    if (!grad_c || !grad_power || !grad_plane) return fail(FRT_EINVAL, "null gradient output");
    frt_status s = check_workspace(workspace, ws_bytes, n_jobs);
    if (s != FRT_OK) return s;
    std::vector<JobDev> packed(static_cast<size_t>(n_jobs));
    std::vector<frt::AdjointJob> adj_in(static_cast<size_t>(n_jobs));
    for (int i = 0; i < n_jobs; ++i) {
        std::string why;
        const frt_job& jb = jobs[i];
        if (!validate(&jb.cam, &jb.frac, jb.planes, jb.n_planes, &jb.march, &jb.out, false, why))
            return fail(FRT_EINVAL, "job " + std::to_string(i) + ": " + why);
        if (jb.march.shading != FRT_SHADING_LAMBERT)
            return fail(FRT_EUNSUPPORTED, "job " + std::to_string(i) + ": the adjoint covers the Lambert model only");
        if (!jb.out.depth || !jb.out.status)
            return fail(FRT_EINVAL, "job " + std::to_string(i) + ": null depth or status plane");
        if (jb.march.normal_mode == FRT_NORMAL_ANALYTIC)
            return fail(FRT_EUNSUPPORTED, "job " + std::to_string(i) +
                                              ": the adjoint of analytic normals needs second derivatives");
        pack(&jb.cam, &jb.frac, jb.planes, jb.n_planes, &jb.march, jb.out, 0, packed[size_t(i)]);
        frt::AdjointJob& a = adj_in[size_t(i)];
        std::memset(&a, 0, sizeof(a));
        a.g_colour = g_colour ? g_colour[i] : nullptr;
        a.g_depth = g_depth ? g_depth[i] : nullptr;
        a.g_normal = g_normal ? g_normal[i] : nullptr;
        a.g_pixel = grad_pixel ? grad_pixel[i] : nullptr;
        for (int k = 0; k < 2; ++k)
            for (int e = 0; e < 3; ++e) a.raw_n[k][e] = k < jb.n_planes ? jb.planes[k].n[e] : 0.0f;
        a.out_index = i;
    }
    // the ray index space holds the Julia jobs, then the Mandelbulb jobs, so
    // each kind's kernel drains only its own tiles
    WorkspaceHeader hdr;
    std::memset(&hdr, 0, sizeof(hdr));
    std::vector<JobDev> table;
    std::vector<frt::AdjointJob> adj;
    table.reserve(size_t(n_jobs));
    adj.reserve(size_t(n_jobs));
    int64_t begin = 0;
    for (int kind = 0; kind < 2; ++kind) {
        hdr.range[kind][0] = static_cast<unsigned long long>(begin);
        for (int i = 0; i < n_jobs; ++i) {
            if (packed[size_t(i)].kind != kind) continue;
            JobDev J = packed[size_t(i)];
            J.ray_begin = begin;
            begin += J.ray_count;
            table.push_back(J);
            adj.push_back(adj_in[size_t(i)]);
        }
        hdr.range[kind][1] = static_cast<unsigned long long>(begin);
    }
    hdr.total_rays = static_cast<unsigned long long>(begin);
    hdr.n_jobs = n_jobs;
    hipStream_t st = static_cast<hipStream_t>(stream);
    s = upload_table(table, hdr, workspace, st, &adj);
    if (s != FRT_OK) return s;
    char* base = static_cast<char*>(workspace);
    frt::AdjointArgs a;
    a.jobs = reinterpret_cast<const JobDev*>(base + sizeof(WorkspaceHeader));
    a.ajobs = reinterpret_cast<const frt::AdjointJob*>(base + sizeof(WorkspaceHeader) + size_t(n_jobs) * sizeof(JobDev));
    a.grad_c = grad_c;
    a.grad_power = grad_power;
    a.grad_plane = grad_plane;
    a.n_jobs = n_jobs;
    std::string why;
    for (int kind = 0; kind < 2; ++kind) {
        long long rays = 0;
        for (const JobDev& J : table)
            if (J.kind == kind) rays += J.ray_count;
        a.grid[kind] = 0;
        if (rays == 0) continue;
        int per_cu = 0;
        if (!occupancy(frt::adjoint_kernel_symbol(kind), 256, per_cu, why)) return fail(FRT_EHIP, why);
        const long long wgs_needed = (rays / 64 + 3) / 4;
        a.grid[kind] = static_cast<int>(
            std::max<long long>(1, std::min<long long>(static_cast<long long>(per_cu) * device_cus(), wgs_needed)));
    }
    hipError_t e = frt::launch_adjoint(a, static_cast<WorkspaceHeader*>(workspace), st);
    if (e != hipSuccess) return hip_fail(e, "adjoint launch");
    return FRT_OK;
}

frt_status frt_autotune_set(int32_t kernel_variant, int32_t block, int32_t chunk, int32_t waves_per_simd,
                            int32_t orbit_lanes, int32_t rare_lanes) {
    g_last_error.clear();
    if (kernel_variant < 0 || kernel_variant >= frt::kNumVariants) return fail(FRT_EINVAL, "unknown kernel_variant");
    if (block != 64 && block != 128 && block != 256 && block != 512) return fail(FRT_EINVAL, "block must be 64..512");
    if (chunk < 64 || chunk > 4096 || chunk % 64 != 0) return fail(FRT_EINVAL, "chunk must be a multiple of 64 in [64, 4096]");
    if (waves_per_simd < 0 || waves_per_simd > 8) return fail(FRT_EINVAL, "waves_per_simd must be in [0, 8]");
    if (orbit_lanes < 1 || orbit_lanes > 64) return fail(FRT_EINVAL, "orbit_lanes must be in [1, 64]");
    if (rare_lanes < 1 || rare_lanes > 64) return fail(FRT_EINVAL, "rare_lanes must be in [1, 64]");
    std::lock_guard<std::mutex> lk(g_mu);
    g_tune[kernel_variant] = Tune{block, chunk, waves_per_simd, orbit_lanes, rare_lanes};
    return FRT_OK;
}

frt_status frt_autotune_get(int32_t kernel_variant, int32_t* block, int32_t* chunk, int32_t* waves_per_simd,
                            int32_t* orbit_lanes, int32_t* rare_lanes) {
    g_last_error.clear();
    if (kernel_variant < 0 || kernel_variant >= frt::kNumVariants) return fail(FRT_EINVAL, "unknown kernel_variant");
    if (!block || !chunk || !waves_per_simd || !orbit_lanes || !rare_lanes) {
        return fail(FRT_EINVAL, "null output pointer");
    }
    std::lock_guard<std::mutex> lk(g_mu);
    const Tune& t = g_tune[kernel_variant];
    *block = t.block;
    *chunk = t.chunk;
    *waves_per_simd = t.waves_per_simd;
    *orbit_lanes = t.orbit_lanes;
    *rare_lanes = t.rare_lanes;
    return FRT_OK;
}

frt_status frt_set_stage_timing(int32_t enable) {
    g_last_error.clear();
    if (enable != 0 && enable != 1) return fail(FRT_EINVAL, "enable must be 0 or 1");
    std::lock_guard<std::mutex> lk(g_time_mu);
    g_timing = enable == 1;
    g_marks_recorded = false;
    return FRT_OK;
}

frt_status frt_stage_times(float* ms) {
    g_last_error.clear();
    if (!ms) return fail(FRT_EINVAL, "null output");
    std::lock_guard<std::mutex> lk(g_time_mu);
    if (!g_timing || !g_marks_recorded) return fail(FRT_EINVAL, "stage timing is off or nothing was recorded");
    for (int k = 0; k < 3; ++k) {
        hipError_t e = hipEventSynchronize(g_marks[k + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        e = hipEventElapsedTime(&ms[k], g_marks[k], g_marks[k + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    }
    return FRT_OK;
}

frt_status frt_graph_reset(void) {
    g_last_error.clear();
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (GraphEntry& g : g_graphs) (void)hipGraphExecDestroy(g.exec);
    g_graphs.clear();
    return FRT_OK;
}

const char* frt_status_string(frt_status s) {
    switch (s) {
        case FRT_OK: return "ok";
        case FRT_EINVAL: return "invalid argument";
        case FRT_EHIP: return "HIP runtime error";
        case FRT_ENOMEM: return "workspace too small";
        case FRT_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* frt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
