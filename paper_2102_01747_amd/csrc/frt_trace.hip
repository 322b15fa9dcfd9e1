// frt_trace.hip -- forward sphere-tracing kernels for gfx950.
//
// One lane per ray, FP32.  The per-pixel path of the paper (Listings 2-5 and
// 7) runs as three kernels over the rays of a batch, so that each keeps only
// the state of its own stage in registers (more resident waves per SIMD, which
// this latency-bound loop needs):
//   1. march_kernel<primary>: search interval (bounding sphere and cut
//      planes), cut-face test, sphere-tracing march of Listing 3 and the
//      bisection refinement of the hit; writes depth, status and counters
//      (and the plane normal of cut-face hits, and the miss encoding);
//   2. normal_kernel: normal taps of Eq. 5 / Listing 5 around each refined
//      hit, the normal, and Lambert shading assuming the point is lit;
//   3. march_kernel<shadow>: one shadow ray toward the light from every lit
//      hit; on a hit the pixel is marked shadowed and keeps only ambient light.
// The two march kernels are persistent: each wave runs one loop in which the
// busy lanes advance their orbits (Eq. 3-4) while at least `orbit_lanes` of
// them still iterate, so the wave does not wait for its slowest orbit: lanes
// whose estimate is done take their march / refinement step in place and
// start the next sample, stragglers resume next trip; and when `rare_lanes`
// lanes wait (or none is busy)
// finished rays are written and idle lanes refill from a global ray queue --
// one atomic claims `chunk` ray indices, handed out by ballot + mbcnt.  A wave
// leaves its loop when the ballot of busy lanes is empty and the queue is
// drained.  One launch of each kernel serves all renders of a batch.
//
// The build compiles this file alone with FP32 denormals flushed, the
// hardware's IEEE mode off and no NaN or signed-zero semantics, so that a
// doubling or power-of-two scale folds into the output modifier of the
// instruction producing the value.  No value here that an output depends on
// is a denormal, a NaN or a signed zero; work-item IDs come from the amdgcn
// builtins (device-library code would not inline into this mode).
#include <hip/hip_runtime.h>

#include "frt_fractal.hpp"
#include "frt_internal.hpp"
#include "frt_job.hpp"
#include "frt_normal.hpp"
#include "frt_ray.hpp"

namespace frt {

// FRT_TRIP_COUNTERS: a measurement build that counts, per march stage, the
// wave-level trips, orbit-loop iterations, step paths and claims (summed
// into the workspace header at each wave's exit); off in the product build.
// FRT_WAVE_TIMES (implied by FRT_TRIP_COUNTERS): only stamps of the
// real-time counter at each wave's start, its first finding the queue dry
// and its exit -- a few instructions per wave outside its loop.
#ifdef FRT_TRIP_COUNTERS
#define FRT_TRIP_ADD(k, v) (trip_c[k] += (v))
#ifndef FRT_WAVE_TIMES
#define FRT_WAVE_TIMES
#endif
#else
#define FRT_TRIP_ADD(k, v) ((void)0)
#endif
#ifdef FRT_WAVE_TIMES
#define FRT_TRIP_DRAINED() (wave_stamp[1] = __builtin_amdgcn_s_memrealtime())
#else
#define FRT_TRIP_DRAINED() ((void)0)
#endif

// Real-time counter stamps (FRT_WAVE_TIMES): lane 0 folds a stamp into the
// latest and (complemented) the earliest of slots k and k + 1.  Called only
// outside the wave's loop (a divergent branch inside it changes how the loop
// is compiled); the stamps taken inside wait in LDS, not in registers.
__device__ __forceinline__ void wave_time_mark(unsigned long long* tc, int k, unsigned long long now) {
    if (__lane_id() == 0) {
        atomicMax(&tc[k], now);
        atomicMax(&tc[k + 1], ~now);
    }
}

// Bisection stops once the root bracket is narrower than eps(t) / 32 (then one
// secant step on the final bracket).  A coarser bracket keeps the depth within
// tolerance but moves the normal taps with it; the bisection also picks the
// same root as the oracle's when a step holds several crossings.
constexpr float kRefineTol = 1.0f / 32.0f;
// Upper bound on orbit bodies per loop trip (keeps finished rays flowing).
constexpr int kMaxBodiesPerTrip = 64;

enum MarchPhase : int { kIdle = 0, kCut = 1, kMarch = 2, kRefine = 3, kDone = 4 };

// Results of a finished primary ray (R12's miss encoding; a cut-face hit takes
// the plane's normal, other hits get theirs from the normal kernel).
__device__ __forceinline__ void write_primary(const JobDev& J, int pix, int status, float t, int entry, int steps,
                                              unsigned evals, unsigned bodies, int hit_it) {
    const long long NP = J.npix;
    const int cls = status & 7;
    if (cls == kMissBounds || cls == kMissTmax) {
        J.depth[pix] = -1.0f;
        J.normal[pix] = 0.0f;
        J.normal[NP + pix] = 0.0f;
        J.normal[2 * NP + pix] = 0.0f;
        J.colour[pix] = 0.0f;
        J.colour[NP + pix] = 0.0f;
        J.colour[2 * NP + pix] = 0.0f;
    } else {
        J.depth[pix] = t;
        if (cls == kHitCut) {
            J.normal[pix] = J.pn[entry][0];
            J.normal[NP + pix] = J.pn[entry][1];
            J.normal[2 * NP + pix] = J.pn[entry][2];
        }
    }
    J.status[pix] = static_cast<uint8_t>(status);
    if (J.counters) {
        J.counters[pix] = static_cast<unsigned>(steps);
        J.counters[NP + pix] = evals;
        J.counters[2 * NP + pix] = bodies;
        J.counters[3 * NP + pix] = static_cast<unsigned>(hit_it);
        for (int k = 4; k < kCounterPlanes; ++k) J.counters[k * NP + pix] = 0u;
    }
}

// Results of a finished shadow ray: a shadowed pixel keeps only the ambient
// term of its colour.
__device__ __forceinline__ void write_shadow(const JobDev& J, int pix, int status, unsigned evals, unsigned bodies) {
    const long long NP = J.npix;
    if (status & kFlagShadowed) {
        J.status[pix] = static_cast<uint8_t>(J.status[pix] | kFlagShadowed);
        J.colour[pix] = J.albedo[0] * J.k_a;
        J.colour[NP + pix] = J.albedo[1] * J.k_a;
        J.colour[2 * NP + pix] = J.albedo[2] * J.k_a;
    }
    if (J.counters) {
        J.counters[6 * NP + pix] = evals;
        J.counters[7 * NP + pix] = bodies;
    }
}

// ---------------------------------------------------------------------------
// Persistent march kernel.  SHADOW = false: primary rays (interval, cut face,
// march, refinement).  SHADOW = true: the shadow ray of every lit hit, from
// p* + 4 eps(t*) N toward the light with threshold eps(t*) (the hit is read
// back from depth / normal / status written by the earlier kernels).
// ---------------------------------------------------------------------------
// The primary march of every variant but n = 8 is held to 64 VGPRs (8 waves
// per SIMD): left alone the real-power kernel took 66 and ran its 4K sweep
// about 1.5% slower.  The n = 8 primary march is held to 7 waves per SIMD:
// left alone it took 106 SGPRs, and with those only 6 of its waves per SIMD
// were resident (the workgroups of a seventh started as others left, though
// the occupancy query counts 7); at 94 SGPRs 7 are, and it runs about 2%
// faster.  The shadow marches are left alone: held to 8 waves per SIMD the
// n = 8 one (56 VGPRs) spilled SGPRs and ran about 4% slower.
template <int VAR, bool BATCH, bool SHADOW>
__global__ void __launch_bounds__(512)
    __attribute__((amdgpu_waves_per_eu(SHADOW ? 1 : (VAR == kVarBulb8 ? 7 : 8))))
march_kernel(const JobDev* __restrict__ jobs, const JobDev job1,
                                                    WorkspaceHeader* __restrict__ hdr, int chunk,
                                                    int orbit_lanes, int rare_lanes) {
    using Orbit = typename OrbitOf<VAR>::T;
    // this variant's group of rays and its counter
    unsigned long long* queue = &hdr->queue[(VAR * 2 + (SHADOW ? 1 : 0)) * kQueueSlots][0];
    int n_jobs = 1;
    unsigned long long r_begin = 0, r_end = static_cast<unsigned long long>(job1.ray_count);
    if constexpr (BATCH) {
        n_jobs = hdr->n_jobs;
        r_begin = hdr->range[VAR][0];
        r_end = hdr->range[VAR][1];
    }
    unsigned long long q_next = 0, q_end = 0;   // wave-uniform window of claimed rays
#ifdef FRT_TRIP_COUNTERS
    unsigned long long trip_c[kTripCount] = {};
#endif
#ifdef FRT_WAVE_TIMES
    __shared__ unsigned long long wave_stamps[8][2];   // per wave: start, first dry queue
    unsigned long long* wave_stamp = wave_stamps[thread_x() >> 6];
    wave_stamp[0] = __builtin_amdgcn_s_memrealtime();
    wave_stamp[1] = 0ull;
#endif
    bool drained = false;
    // A wave's first claim is chunk number (its index in the grid), taken
    // without a counter.  The chunks after the grid's first n_waves are
    // dealt to kQueueSlots counters in turn (chunk n_waves + s + j
    // kQueueSlots is the j-th of slot s); a wave claims from its block's
    // slot, and from the others once that share is spent.  All waves
    // claiming through one address would queue on it.
    const unsigned wpb = block_threads() >> 6;
    const unsigned long long n_waves = grid_threads() >> 6;
    const unsigned long long first_chunk =
        static_cast<unsigned long long>(block_x()) * wpb + __builtin_amdgcn_readfirstlane(thread_x() >> 6);
    const unsigned home = block_x() % kQueueSlots;
    unsigned spent = 0u;   // slots whose share is spent (wave-uniform)
    bool first_claim = true;
    auto claim = [&]() -> unsigned long long {   // the chunk's first ray, or r_end
        FRT_TRIP_ADD(kTripClaims, 1);
        if (first_claim) {
            first_claim = false;
            return min(r_begin + first_chunk * static_cast<unsigned long long>(chunk), r_end);
        }
        for (unsigned i = 0; i < static_cast<unsigned>(kQueueSlots); ++i) {
            const unsigned sl = (home + i) % kQueueSlots;
            if (spent & (1u << sl)) continue;
            unsigned long long a = 0;
            if (i > 0) {
                // another slot: most are spent by the time a wave looks, so
                // read the counter first (it only grows, so a stale value can
                // only cost an extra attempt) instead of queueing an update
                if (__lane_id() == 0) a = __hip_atomic_load(queue + 32 * sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                a = bcast_first(a);
                if (r_begin + (n_waves + sl + a * kQueueSlots) * static_cast<unsigned long long>(chunk) >= r_end) {
                    spent |= 1u << sl;
                    continue;
                }
            }
            if (__lane_id() == 0) a = atomicAdd(queue + 32 * sl, 1ull);
            const unsigned long long k = n_waves + sl + bcast_first(a) * kQueueSlots;
            const unsigned long long base = r_begin + k * static_cast<unsigned long long>(chunk);
            if (base < r_end) return base;
            spent |= 1u << sl;
        }
        return r_end;
    };
    JobCursor cur;                               // job of the current claim (wave-uniform)
    // shadow rays: the current tile's first ray index and the mask of its
    // shadow-casting pixels not yet handed to a lane (wave-uniform)
    unsigned long long tile_g = 0, tmask = 0;
    __shared__ uint8_t slots[8][64];   // per wave: lane index of the k-th set bit of tmask
    uint8_t* slot = slots[thread_x() >> 6];
    // per wave: the shadow rays gathered for a refill (ray index within their job)
    __shared__ int gathered_rays[SHADOW ? 8 : 1][64];
    int* gathered = gathered_rays[SHADOW ? (thread_x() >> 6) : 0];

    int phase = kIdle;
    int jb = 0, pix = 0, entry = -1, status = 0, steps = 0, rk = 0, hit_it = 0;
    unsigned evals = 0, bodies = 0;
    float ox = 0.f, oy = 0.f, oz = 0.f, dx = 0.f, dy = 0.f, dz = 1.f;
    float t = 0.f, t1 = 0.f, lt = 0.f, lh = 0.f, gb = 0.f, ea = 0.f, er = 0.f;
    // march settings of the lane's job, copied when the ray is claimed
    float clamp = 0.2f;
    int max_steps = 1, refine_iters = 0;
    // lanes whose orbit is still iterating, as a wave-uniform mask (the orbit
    // loop then needs one ballot and one scalar AND a body); lanes (re)started
    // in divergent code set `rearm`, folded into the mask at uniform points
    unsigned long long live = 0ull;
    bool rearm = false;
    OrbitParams P = orbit_params(job1);
    Orbit orb;

    for (;;) {
        // ------------------------------------------ finished rays + refill
        FRT_TRIP_ADD(kTripLoops, 1);
        const unsigned long long m_busy = __ballot(phase == kCut || phase == kMarch || phase == kRefine);
        const unsigned long long m_done = __ballot(phase == kDone);
        const bool exhausted = drained && tmask == 0ull;
        if (m_busy == 0ull && m_done == 0ull && exhausted) {
            break;
        }
        const int waiting = __popcll(m_done) + (exhausted ? 0 : __popcll(__ballot(phase == kIdle)));
        if (m_busy == 0ull || waiting >= rare_lanes) {
            FRT_TRIP_ADD(kTripRefills, 1);
            const bool one_job = BATCH && __ballot(phase == kDone && jb != cur.j) == 0ull;
            // when the finished lanes all belong to the cursor's job (the
            // usual case) its output pointers come through scalar loads
            if (phase == kDone && !FRT_CHECK(hdr, jb >= 0 && jb < n_jobs && pix >= 0 &&
                                                  pix < job_ref<BATCH>(jobs, job1, jb).npix, kCheckPixel)) {
                phase = kIdle;   // a finished ray whose pixel lies outside its job: not written
            }
            if (phase == kDone) {
                const JobDev& J = job_ref<BATCH>(jobs, job1, jb);
                if constexpr (!SHADOW) {
                    if (one_job) {
                        write_primary(job_ref<BATCH>(jobs, job1, cur.j), pix, status, t, entry, steps, evals, bodies,
                                      hit_it);
                    } else {
                        write_primary(J, pix, status, t, entry, steps, evals, bodies, hit_it);
                    }
                } else {
                    if (one_job) write_shadow(job_ref<BATCH>(jobs, job1, cur.j), pix, status, evals, bodies);
                    else write_shadow(J, pix, status, evals, bodies);
                }
                phase = kIdle;
            }

            unsigned long long idle = __ballot(phase == kIdle);
            if constexpr (!SHADOW) {
            while (idle != 0ull && !drained) {
                if (q_next >= q_end) {
                    const unsigned long long base = claim();
                    if (base >= r_end) {
                        drained = true;
                        FRT_TRIP_DRAINED();
                        continue;
                    }
                    q_next = base;
                    q_end = min(base + static_cast<unsigned long long>(chunk), r_end);
                }
                // this round's rays all lie in the cursor's job
                job_seek<BATCH>(jobs, job1, n_jobs, q_next, cur);
                if (!FRT_CHECK(hdr, cur.j >= 0 && cur.j < n_jobs, kCheckJob) ||
                    !FRT_CHECK(hdr, q_next >= cur.begin && q_next < cur.end && q_end <= r_end, kCheckRay)) {
                    drained = true;
                    break;
                }
                const unsigned rank = lane_rank(idle);
                const unsigned long long avail = min(q_end, cur.end) - q_next;
                const int j = cur.j;
                const JobDev& J = job_ref<BATCH>(jobs, job1, j);
                int px, py;
                if (phase == kIdle && rank < avail &&
                    FRT_CHECK(hdr, static_cast<long long>(q_next + rank - cur.begin) < J.ray_count, kCheckRay) &&
                    tile_pixel(J, static_cast<long long>(q_next + rank - cur.begin), px, py) &&
                    FRT_CHECK(hdr, static_cast<long long>(py) * J.width + px < J.npix, kCheckPixel)) {
                    const int p = py * J.width + px;
                    float lo, hi;
                    bool go = false;
                    {
                        primary_dir(J, px, py, dx, dy, dz);
                        ox = J.eye[0];
                        oy = J.eye[1];
                        oz = J.eye[2];
                        ea = J.eps_abs;
                        er = J.eps_rel;
                        status = 0;
                        go = ray_interval(J, ox, oy, oz, dx, dy, dz, J.eps_abs, lo, hi, entry);
                        if (!go) {
                            // no interval: written as a miss right away
                            const long long NP = J.npix;
                            J.depth[p] = -1.0f;
                            J.normal[p] = 0.0f;
                            J.normal[NP + p] = 0.0f;
                            J.normal[2 * NP + p] = 0.0f;
                            J.colour[p] = 0.0f;
                            J.colour[NP + p] = 0.0f;
                            J.colour[2 * NP + p] = 0.0f;
                            J.status[p] = kMissBounds;
                            if (J.counters) {
                                for (int k = 0; k < kCounterPlanes; ++k) J.counters[k * NP + p] = 0u;
                            }
                        }
                    }
                    if (go) {
                        jb = j;
                        pix = p;
                        if constexpr (BATCH) P = orbit_params(J);
                        clamp = J.clamp;
                        max_steps = J.max_steps;
                        refine_iters = J.refine_iters;
                        t = lo;
                        t1 = hi;
                        steps = 0;
                        hit_it = 0;
                        evals = 0;
                        bodies = 0;
                        phase = entry >= 0 ? kCut : kMarch;
                        orb.init(fmaf(t, dx, ox), fmaf(t, dy, oy), fmaf(t, dz, oz));
                        rearm = true;
                    }
                }
                q_next += min(static_cast<unsigned long long>(__popcll(idle)), avail);
                idle = __ballot(phase == kIdle);
            }
            } else {
            // Shadow rays: claim 64-ray tiles and read the tile's status bytes
            // once (one load per lane); the normal kernel flagged the pixels
            // that cast a shadow ray, so the tile's rays reduce to a 64-bit
            // mask.  The flagged rays of as many tiles of one job as the idle
            // lanes can take are gathered into this wave's table in LDS (ray
            // index within the job), then handed out to the idle lanes in
            // order in one pass, so the per-ray set-up runs once per refill
            // rather than once per tile.
            while (idle != 0ull && (tmask != 0ull || !drained)) {
                const unsigned need = static_cast<unsigned>(__popcll(idle));
                const unsigned lane = __lane_id();
                unsigned got = 0;   // rays gathered (wave-uniform)
                int gj = cur.j;     // their job (wave-uniform)
                while (got < need && (tmask != 0ull || !drained)) {
                    if (tmask == 0ull) {
                        if (q_next >= q_end) {
                            const unsigned long long base = claim();
                            if (base >= r_end) {
                                drained = true;
                                FRT_TRIP_DRAINED();
                                break;
                            }
                            q_next = base;
                            q_end = min(base + static_cast<unsigned long long>(chunk), r_end);
                        }
                        tile_g = q_next;
                        q_next += 64ull;
                        job_seek<BATCH>(jobs, job1, n_jobs, tile_g, cur);
                        if (!FRT_CHECK(hdr, cur.j >= 0 && cur.j < n_jobs, kCheckJob) ||
                            !FRT_CHECK(hdr, tile_g >= cur.begin && tile_g + 64ull <= cur.end && tile_g < r_end,
                                       kCheckRay)) {
                            drained = true;
                            tmask = 0ull;
                            break;
                        }
                        const JobDev& J = job_ref<BATCH>(jobs, job1, cur.j);
                        int px, py;
                        bool cast = false;
                        if (tile_pixel(J, static_cast<long long>(tile_g - cur.begin) + lane, px, py))
                            cast = (J.status[py * J.width + px] & kFlagShadowRay) != 0;
                        tmask = __ballot(cast);
                        // a tile of another job waits for the next refill
                        if (got > 0 && cur.j != gj) break;
                        gj = cur.j;
                        continue;
                    }
                    // the tile's set bits in order: the first `take` join the
                    // table, the rest stay in tmask
                    const unsigned nbits = static_cast<unsigned>(__popcll(tmask));
                    const unsigned take = min(nbits, need - got);
                    if ((tmask >> lane) & 1ull) {
                        const unsigned k = lane_rank(tmask);
                        slot[k] = static_cast<uint8_t>(lane);
                        if (k < take) gathered[got + k] = static_cast<int>(tile_g - cur.begin) + static_cast<int>(lane);
                    }
                    __builtin_amdgcn_wave_barrier();
                    if (take < nbits) {
                        const unsigned cut = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(slot[take]));
                        tmask &= ~((1ull << cut) - 1ull);
                    } else {
                        tmask = 0ull;
                    }
                    got += take;
                    __builtin_amdgcn_wave_barrier();
                }
                if (got == 0) break;
                const unsigned rank = lane_rank(idle);
                if (phase == kIdle && rank < got) {
                    const JobDev& J = job_ref<BATCH>(jobs, job1, gj);
                    int px, py;
                    tile_pixel(J, static_cast<long long>(gathered[rank]), px, py);
                    const int p = py * J.width + px;
                    const long long NP = J.npix;
                    const float nx = J.normal[p], ny = J.normal[NP + p], nz = J.normal[2 * NP + p];
                    float pdx, pdy, pdz;
                    primary_dir(J, px, py, pdx, pdy, pdz);
                    const float ts = J.depth[p];
                    const float eps = fmaf(J.eps_rel, ts, J.eps_abs);
                    const float off = 4.0f * eps;
                    ox = fmaf(off, nx, fmaf(ts, pdx, J.eye[0]));
                    oy = fmaf(off, ny, fmaf(ts, pdy, J.eye[1]));
                    oz = fmaf(off, nz, fmaf(ts, pdz, J.eye[2]));
                    dx = J.light[0];
                    dy = J.light[1];
                    dz = J.light[2];
                    ea = eps;
                    er = 0.0f;
                    status = 0;
                    float lo, hi;
                    if (ray_interval(J, ox, oy, oz, dx, dy, dz, eps, lo, hi, entry)) {
                        jb = gj;
                        pix = p;
                        if constexpr (BATCH) P = orbit_params(J);
                        clamp = J.clamp;
                        max_steps = J.max_steps;
                        refine_iters = J.refine_iters;
                        t = lo;
                        t1 = hi;
                        steps = 0;
                        hit_it = 0;
                        evals = 0;
                        bodies = 0;
                        phase = entry >= 0 ? kCut : kMarch;
                        orb.init(fmaf(t, dx, ox), fmaf(t, dy, oy), fmaf(t, dz, oz));
                        rearm = true;
                    }
                }
                __builtin_amdgcn_wave_barrier();
                idle = __ballot(phase == kIdle);
            }
            }
        }

        // -------------------------------------------------- orbit bodies
        // Iterate while at least `orbit_lanes` lanes still iterate (and at
        // least once); lanes whose orbit ends wait for the step below, the
        // stragglers carry their orbit state into the next trip.  The body
        // runs on every lane with no branch; step() keeps the estimate's
        // inputs only in live lanes (three selects and two compares a body).
        live |= __ballot(rearm);
        rearm = false;
        if (live != 0ull) {
            // Fewer lanes iterating than orbit_lanes happens only once the
            // queue has run dry (otherwise the refill above has run): then
            // every orbit runs to its end before the step, instead of the
            // last rays of a launch paying the step path after every body.
            const int keep = __popcll(live) < orbit_lanes ? 1 : orbit_lanes;
            int b = 0;
            do {
                FRT_TRIP_ADD(kTripBodyIters, 1);
                FRT_TRIP_ADD(kTripLiveLanes, __popcll(live));
                live = orb.step(P, live);
            } while (++b < kMaxBodiesPerTrip && __popcll(live) >= keep);
        }
#ifdef FRT_TRIP_COUNTERS
        {
            const unsigned long long m_step =
                __ballot(!__builtin_amdgcn_inverse_ballot_w64(live) && (phase == kCut || phase == kMarch || phase == kRefine));
            if (m_step != 0ull) {
                FRT_TRIP_ADD(kTripSteps, 1);
                FRT_TRIP_ADD(kTripStepLanes, __popcll(m_step));
            }
        }
#endif
        if (!__builtin_amdgcn_inverse_ballot_w64(live) && (phase == kCut || phase == kMarch || phase == kRefine)) {
            // One pass with no branches: nearly every wave has lanes in
            // each case, so every case's values are computed and each lane
            // selects its own.
            const DEResult de = orb.result(P);
            evals += 1u;
            bodies += static_cast<unsigned>(de.bodies);
            const float d = de.d;
            const float eps_t = fmaf(er, t, ea);
            // g = d - eps(t).  One bracket update serves the march (Listing
            // 3) and the bisection: a sample above the eps-region becomes the
            // bracket's left end lt (g(lt) = lh >= 0), one below it the right
            // end t1 (g(t1) = gb < 0).  A march lane keeps t1 = the
            // interval's end until its first sample below, which ends the
            // march.
            const float g = d - eps_t;
            const bool below = g < 0.0f;
            // cut face: the entry point is inside when its orbit does not
            // escape or the estimate is below eps; otherwise the lane
            // marches on from this sample
            const bool cut_in = phase == kCut && (de.it == P.max_iter || d < eps_t);
            const bool ref = !SHADOW && phase == kRefine;
            const bool mar = phase != kRefine && !cut_in;
            steps += mar ? 1 : 0;
            if constexpr (!SHADOW) {
                hit_it = ref ? hit_it : de.it;
                t1 = below ? t : t1;
                gb = below ? g : gb;
                lt = below ? lt : t;
                lh = below ? lh : g;
            }
            const bool adv = mar && !below;
            const float tn = t + fminf(d, clamp);
            const bool miss = adv && tn > t1;
            const bool exhausted = adv && !miss && steps >= max_steps;
            // shadow rays stop at their first hit; a primary ray whose first
            // sample is inside has no bracket
            const bool first = mar && below && (SHADOW || steps == 1);
            // the bracket [lt, t1] holds a root of g: bisect it down to
            // eps / 32, then one secant step
            const bool bis = !SHADOW && (ref || (mar && below)) && !first;
            rk = ref ? rk + 1 : 0;
            const float w = t1 - lt;
            const bool cont = bis && rk < refine_iters && w > kRefineTol * fmaf(er, t1, ea);
            const float tmid = 0.5f * (lt + t1);
            // (the hardware reciprocal: the secant only has to land inside a
            // bracket already narrower than eps / 32)
            const float tsec = fmaf(-gb, w * hw_rcp(gb - lh), t1);
            t = adv ? tn : (cont ? tmid : (bis ? tsec : t));
            if constexpr (SHADOW) {
                status = (cut_in || exhausted || first) ? kFlagShadowed : (miss ? 0 : status);
            } else {
                status = cut_in ? kHitCut
                       : miss ? kMissTmax
                       : exhausted ? (kHitExhausted | kFlagUnrefined)
                       : first ? (kHit | kFlagUnrefined)
                       : (bis && !ref) ? kHit : status;
            }
            const bool done = cut_in || miss || exhausted || first || (bis && !cont);
            phase = done ? kDone : (cont ? kRefine : kMarch);
            // the next sample's orbit (finished lanes restart one too, unused)
            orb.init(fmaf(t, dx, ox), fmaf(t, dy, oy), fmaf(t, dz, oz));
            rearm = !done;
        }
        live |= __ballot(rearm);
        rearm = false;
    }
#ifdef FRT_TRIP_COUNTERS
    if (__lane_id() == 0) {
        for (int k = 0; k < kTripCount; ++k) atomicAdd(&hdr->trips[(SHADOW ? 16 : 0) + k], trip_c[k]);
    }
#endif
#ifdef FRT_WAVE_TIMES
    {
        unsigned long long* tc = &hdr->trips[SHADOW ? 16 : 0];
        const unsigned long long t_exit = __builtin_amdgcn_s_memrealtime();
        const unsigned long long t_drain = wave_stamp[1];
        wave_time_mark(tc, kTripStartMax, wave_stamp[0]);
        wave_time_mark(tc, kTripDrainMax, t_drain ? t_drain : t_exit);
        wave_time_mark(tc, kTripExitMax, t_exit);
        if (__lane_id() == 0) {
            atomicAdd(&tc[kTripLifeSum], t_exit);
            atomicAdd(&tc[kTripWaves], 1ull);
        }
    }
#endif
}

// ---------------------------------------------------------------------------
// Normal taps (Eq. 5 / Listing 5) and Lambert shading of every hit, one lane
// per ray of the batch.  Tetrahedral: h = 0.5773 eps(t*), N ~ sum nu_i d(p +
// h nu_i); central: h = eps(t*), N_k ~ d(p + h e_k) - d(p - h e_k); analytic:
// N ~ grad d(p) by forward-mode tangents (frt_gradient.hpp).  A zero or
// non-finite gradient falls back to -dir.  Colour assumes the point is lit; the shadow
// kernel darkens shadowed pixels.
// ---------------------------------------------------------------------------
template <int VAR, bool BATCH>
__global__ void __launch_bounds__(256) normal_kernel(const JobDev* __restrict__ jobs, const JobDev job1,
                                                     WorkspaceHeader* __restrict__ hdr) {
    int n_jobs = 1;
    unsigned long long r_begin = 0, r_end = static_cast<unsigned long long>(job1.ray_count);
    if constexpr (BATCH) {
        n_jobs = hdr->n_jobs;
        r_begin = hdr->range[VAR][0];
        r_end = hdr->range[VAR][1];
    }
    const unsigned long long stride = grid_threads();
    JobCursor cur;
    for (unsigned long long g = r_begin + static_cast<unsigned long long>(block_x()) * block_threads() + thread_x();
         g < r_end; g += stride) {
        // a wave covers one 64-ray tile, inside one job
        job_seek<BATCH>(jobs, job1, n_jobs, bcast_first(g - __lane_id()), cur);
        if (!FRT_CHECK(hdr, cur.j >= 0 && cur.j < n_jobs, kCheckJob) ||
            !FRT_CHECK(hdr, g >= cur.begin && g < cur.end, kCheckRay)) continue;
        const int j = cur.j;
        const JobDev& J = job_ref<BATCH>(jobs, job1, j);
        int px, py;
        if (!tile_pixel(J, static_cast<long long>(g - cur.begin), px, py)) continue;
        const int p = py * J.width + px;
        if (!FRT_CHECK(hdr, p >= 0 && p < J.npix, kCheckPixel)) continue;
        const int cls = J.status[p] & 7;
        if (cls < kHit) continue;
        const long long NP = J.npix;
        float nx, ny, nz;
        unsigned evals = 0, bodies = 0;
        if (cls == kHitCut) {
            nx = J.normal[p];
            ny = J.normal[NP + p];
            nz = J.normal[2 * NP + p];
        } else {
            const OrbitParams P = orbit_params(J);
            float dx, dy, dz;
            primary_dir(J, px, py, dx, dy, dz);
            const float ts = J.depth[p];
            const float eps = fmaf(J.eps_rel, ts, J.eps_abs);
            const float sx = fmaf(ts, dx, J.eye[0]), sy = fmaf(ts, dy, J.eye[1]), sz = fmaf(ts, dz, J.eye[2]);
            float gx, gy, gz;
            estimate_normal<VAR>(P, J.normal_mode, sx, sy, sz, eps, gx, gy, gz, evals, bodies);
            if (!unit_normal(gx, gy, gz, nx, ny, nz)) {
                nx = -dx;
                ny = -dy;
                nz = -dz;
            }
            J.normal[p] = nx;
            J.normal[NP + p] = ny;
            J.normal[2 * NP + p] = nz;
        }
        const float ndl = fmaf(nx, J.light[0], fmaf(ny, J.light[1], nz * J.light[2]));
        if (J.shadow && ndl > 0.0f) J.status[p] = static_cast<uint8_t>(J.status[p] | kFlagShadowRay);
        const float lam = fmaf(J.k_d, fmaxf(ndl, 0.0f), J.k_a);
        J.colour[p] = J.albedo[0] * lam;
        J.colour[NP + p] = J.albedo[1] * lam;
        J.colour[2 * NP + p] = J.albedo[2] * lam;
        if (J.counters && evals) {
            J.counters[4 * NP + p] = evals;
            J.counters[5 * NP + p] = bodies;
        }
    }
}

__global__ void reset_queue_kernel(WorkspaceHeader* hdr) {
    if (thread_x() < 2 * kNumVariants * kQueueSlots) hdr->queue[thread_x()][0] = 0ull;
}

static hipError_t mark(hipEvent_t* marks, int k, hipStream_t stream) {
    return marks ? hipEventRecord(marks[k], stream) : hipSuccess;
}

// One stage (0 primary march, 1 normals, 2 shadow march) of one group.
template <int VAR, bool BATCH>
static hipError_t launch_stage(int stage, const LaunchCfg& cfg, const JobDev* jobs, const JobDev& job1,
                               WorkspaceHeader* hdr, hipStream_t stream) {
    if (stage == 0) {
        hipLaunchKernelGGL((march_kernel<VAR, BATCH, false>), dim3(cfg.grid), dim3(cfg.block), 0, stream, jobs,
                           job1, hdr, cfg.chunk, cfg.orbit_lanes, cfg.rare_lanes);
    } else if (stage == 1) {
        hipLaunchKernelGGL((normal_kernel<VAR, BATCH>), dim3(cfg.normal_grid), dim3(256), 0, stream, jobs, job1,
                           hdr);
    } else {
        // a tile holds few shadow rays (only lit hits cast one), so a claim
        // covers twice the primary march's rays to keep the queue traffic down
        hipLaunchKernelGGL((march_kernel<VAR, BATCH, true>), dim3(cfg.grid), dim3(cfg.block), 0, stream, jobs,
                           job1, hdr, 2 * cfg.chunk, cfg.orbit_lanes, cfg.rare_lanes);
    }
    return hipGetLastError();
}

template <bool BATCH>
static hipError_t launch_stage_var(int variant, int stage, const LaunchCfg& cfg, const JobDev* jobs,
                                   const JobDev& job1, WorkspaceHeader* hdr, hipStream_t stream) {
    switch (variant) {
        case kVarJulia: return launch_stage<kVarJulia, BATCH>(stage, cfg, jobs, job1, hdr, stream);
        case kVarBulbReal: return launch_stage<kVarBulbReal, BATCH>(stage, cfg, jobs, job1, hdr, stream);
        case kVarBulbInt: return launch_stage<kVarBulbInt, BATCH>(stage, cfg, jobs, job1, hdr, stream);
        case kVarBulb8: return launch_stage<kVarBulb8, BATCH>(stage, cfg, jobs, job1, hdr, stream);
        default: return launch_stage<kVarJuliaDeg, BATCH>(stage, cfg, jobs, job1, hdr, stream);
    }
}

template <int VAR, bool BATCH>
static const void* kernel_ptr() {
    return reinterpret_cast<const void*>(&march_kernel<VAR, BATCH, false>);
}

const void* trace_kernel_symbol(int variant, bool batch) {
    switch (variant) {
        case kVarJulia: return batch ? kernel_ptr<kVarJulia, true>() : kernel_ptr<kVarJulia, false>();
        case kVarBulbReal: return batch ? kernel_ptr<kVarBulbReal, true>() : kernel_ptr<kVarBulbReal, false>();
        case kVarBulbInt: return batch ? kernel_ptr<kVarBulbInt, true>() : kernel_ptr<kVarBulbInt, false>();
        case kVarBulb8: return batch ? kernel_ptr<kVarBulb8, true>() : kernel_ptr<kVarBulb8, false>();
        default: return batch ? kernel_ptr<kVarJuliaDeg, true>() : kernel_ptr<kVarJuliaDeg, false>();
    }
}

hipError_t launch_trace(const TraceGroup* groups, int n_groups, bool batch, const JobDev* jobs, const JobDev& job1,
                        WorkspaceHeader* hdr, hipStream_t stream, hipEvent_t* marks, bool fork) {
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(2 * kNumVariants * kQueueSlots), 0, stream, hdr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && fork && !marks && n_groups > 1 && n_groups <= 1 + kSideStreams) {
        // group g > 0 on side stream g - 1; each group's stages stay in order
        hipStream_t side[kSideStreams];
        e = fork_streams(stream, n_groups - 1, side);
        for (int g = 0; g < n_groups && e == hipSuccess; ++g) {
            hipStream_t s = g == 0 ? stream : side[g - 1];
            for (int stage = 0; stage < 3 && e == hipSuccess; ++stage) {
                if (stage == 2 && !groups[g].any_shadow) continue;
                e = batch ? launch_stage_var<true>(groups[g].variant, stage, groups[g].cfg, jobs, job1, hdr, s)
                          : launch_stage_var<false>(groups[g].variant, stage, groups[g].cfg, jobs, job1, hdr, s);
            }
        }
        const hipError_t ej = join_streams(stream, n_groups - 1);
        return e != hipSuccess ? e : ej;
    }
    for (int stage = 0; stage < 3 && e == hipSuccess; ++stage) {
        e = mark(marks, stage, stream);
        for (int g = 0; g < n_groups && e == hipSuccess; ++g) {
            if (stage == 2 && !groups[g].any_shadow) continue;
            e = batch ? launch_stage_var<true>(groups[g].variant, stage, groups[g].cfg, jobs, job1, hdr, stream)
                      : launch_stage_var<false>(groups[g].variant, stage, groups[g].cfg, jobs, job1, hdr, stream);
        }
    }
    if (e == hipSuccess) e = mark(marks, 3, stream);
    return e;
}

}  // namespace frt
