/*
 * frt.h -- C ABI of the MI355X fractal sphere tracer.
 *
 * Renders escape-time fractals by per-pixel sphere tracing, after da Silva,
 * Novello, Lopes and Velho, "Real-time rendering of complex fractals"
 * (arXiv 2102.01747):
 *   - the quaternion Julia set z^p + c (Sec. 1.1 at p = 2, Eq. 3-4 and the
 *     cubic of Listing 4 for higher integer degrees), sliced to 3-D with the
 *     fourth quaternion component zero and optionally cut by planes (Fig. 1
 *     and the text around Listing 3);
 *   - the White-Nylander power-n Mandelbulb (Sec. 1.2, Eq. 1, Listing 7).
 * Both are driven by the orbit-derivative distance estimate
 * d = 0.5 |z| ln|z| / |z'| (Sec. 2, Eq. 2-4; Listings 4 and 7), marched as in
 * Listing 3, with normals from distance taps (Eq. 5, Listing 5) and Lambert
 * shading with an optional shadow ray.
 *
 * Conventions shared by every entry point
 *   - All device buffers are owned by the caller.  The library keeps no
 *     pointer after a call returns, except that a captured batch graph
 *     (frt_render_batch with use_graph=1) keeps the workspace pointer until
 *     frt_graph_reset() or the next capture.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL is the
 *     default stream).  Device faults surface at the caller's next sync.
 *   - Parameter structs are read by value during the call.
 *   - Invalid arguments return FRT_EINVAL before anything is launched, so
 *     no output is written; frt_last_error() then names the argument.
 *   - No C++ exception crosses this interface.
 *
 * Framebuffer layout (frt_frame): structure of arrays over P = width*height
 * pixels, linear index j*width + i with row j = 0 at the top of the image.
 *   depth    float[P]      ray parameter t* of the hit along the unit ray
 *                          direction (Euclidean distance from the eye),
 *                          -1 on a miss
 *   normal   float[3][P]   unit normal planes x, y, z (0 on a miss)
 *   colour   float[3][P]   shaded colour planes r, g, b (0 on a miss)
 *   status   uint8[P]      bits 0-2: 0 miss (no bounding interval),
 *                          1 miss (left the interval), 2 hit, 3 hit on a cut
 *                          face, 4 hit by running out of steps;
 *                          bit 3: shadowed (the shadow ray hit);
 *                          bit 4: depth not refined (first sample or
 *                          running out of steps);
 *                          bit 6: a shadow ray was traced from this hit
 *   counters uint32[8][P]  optional (NULL to skip), per pixel:
 *                          0 primary march samples,
 *                          1 distance evaluations of the primary ray (cut
 *                            face, march, refinement), 2 their orbit bodies,
 *                          3 escape count at the last primary march sample,
 *                          4 normal-tap evaluations, 5 their orbit bodies,
 *                          6 shadow-ray evaluations, 7 their orbit bodies
 */
#ifndef FRT_H
#define FRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FRT_OK = 0,
    FRT_EINVAL = -1,        /* invalid argument; nothing launched            */
    FRT_EHIP = -2,          /* a HIP runtime call failed                     */
    FRT_ENOMEM = -3,        /* workspace too small                           */
    FRT_EUNSUPPORTED = -4   /* valid request this build cannot serve         */
} frt_status;

enum { FRT_JULIA = 0, FRT_MANDELBULB = 1 };
enum { FRT_NORMAL_TETRA = 0, FRT_NORMAL_CENTRAL = 1, FRT_NORMAL_ANALYTIC = 2 };
enum { FRT_SHADING_LAMBERT = 0, FRT_SHADING_PHONG = 1 };

/* Pinhole camera: vertical field of view, pixel centres, row 0 at the top.
 * Ray through pixel (i, j): dir = normalize(f + x r + y u) with
 * f = normalize(target - eye), r = normalize(f x up), u = r x f,
 * s = tan(fov_y/2), x = (2(i+1/2)/W - 1) s W/H, y = (1 - 2(j+1/2)/H) s.     */
typedef struct {
    float eye[3], target[3], up[3];
    float fov_y_deg;            /* (0, 180)                                  */
    int32_t width, height;      /* >= 1 each                                 */
} frt_camera;

/* Fractal (Sec. 1.1, 1.2).  Julia: z0 = (x, y, z, 0) with component 0 the
 * real part, z <- z^p + c (Eq. 3) for an integer degree p in [2, 16] given
 * in `power` (Listing 4 is p = 3), with the squared derivative gaining
 * p^2 |z|^(2(p-1)) per body (Eq. 4 in norm); bailout2^p must be below 2^120
 * so that the escaping body's |z|^2 stays finite in float32.  Mandelbulb: w0 = p, w <- w^n + p with the
 * power map of Eq. 1 in Listing 7's axes (y polar, azimuth atan2(x, z)),
 * any real n >= 2.  An orbit stops after max_iter bodies or when |z|^2
 * exceeds bailout2.  The march is confined to a sphere whose radius is the
 * larger of the provable escape radius (the root R >= 1 of R^p - R - |c|
 * for Julia, (1 + sqrt(1 + 4|c|))/2 at p = 2,
 * 2^(1/(n-1)) for the Mandelbulb) and bound_radius (0 for automatic).      */
typedef struct {
    int32_t kind;               /* FRT_JULIA or FRT_MANDELBULB               */
    float c[4];                 /* Julia constant; ignored for Mandelbulb    */
    float power;                /* Mandelbulb n >= 2; Julia degree p         */
    int32_t max_iter;           /* [1, 4096]                                 */
    float bailout2;             /* > 0                                       */
    float bound_radius;         /* >= 0                                      */
} frt_fractal;

/* Cut plane: the kept half-space is { x : (n/|n|) . x <= d }.  n need not be
 * unit length (it must be non-zero); gradients are taken w.r.t. raw n.     */
typedef struct {
    float n[3];
    float d;
} frt_plane;

/* March and shading (Listing 3, Eq. 5, Listing 5).
 * eps(t) = eps_abs + eps_rel t is the stop threshold; steps are
 * min(d, step_clamp); the search interval starts at eps_abs and ends at
 * t_max, cut by the bounding sphere and the planes.  A hit is refined to the
 * root of d - eps(t) between the last two samples by bisection (at most
 * refine_iters halvings, stopping once the bracket is narrower than
 * eps(t)/32) and one secant step on the final bracket; bisection picks the
 * same root as the FP64 reference when the bracket holds several (the
 * estimate jumps where the escape count changes).  Normals: tetrahedral taps with
 * h = 0.5773 eps(t*), central differences with h = eps(t*), or the analytic
 * normal: the exact gradient of the estimate at p* by forward-mode
 * differentiation of the orbit (Sec. 2: on the set it is grad G / |grad G|),
 * one orbit evaluation with three tangents and no tap spacing.
 * colour = albedo (k_ambient + k_diffuse max(0, N.L) V), L = light_dir
 * normalised, V = 0 when the shadow ray (from p* + 4 eps(t*) N toward L,
 * threshold eps(t*)) hits, else 1; V is traced only when shadow != 0 and
 * N.L > 0.
 * FRT_SHADING_PHONG, the closest-hit shading of the paper's shaders, is
 * served by frt_render_scene, frt_render and frt_render_batch (the latter
 * two trace such a job as a one-object scene with the identity placement;
 * the adjoint and frt_render_batch_noalloc return FRT_EUNSUPPORTED): the
 * colour above plus a white highlight
 * k_specular max(0, R.V)^shininess V (R = 2 (N.L) N - L, V = -dir, zero when
 * N.L <= 0), plus k_reflect F c_r, where c_r is the colour of the first hit
 * of the reflection ray (from p* + 4 eps(t*) N along dir - 2 (dir.N) N,
 * threshold eps(t*) + eps_rel s at distance s, against every object; its
 * own Lambert and highlight terms, no shadow ray; 0 on a miss) and
 * F = albedo + (1 - albedo)(1 - max(0, -dir.N))^5 (Schlick, per channel).
 * With this model the albedo of a hit (and of the reflection ray's hit) is
 * coloured by the orbit trap T of its point (the colour parameters of the
 * Mandelbulb distance listing: the minima of |x|, |y|, |z| and |w|^2 over
 * the orbit): albedo_c + sum_k trap_colour[k][c] T_k, clamped to [0, 1]
 * per channel; a zero trap_colour leaves the albedo as given.               */
typedef struct {
    int32_t max_steps;          /* [1, 65536]                                */
    float eps_abs, eps_rel;     /* >= 0, not both 0                          */
    float step_clamp;           /* > 0                                       */
    float t_max;                /* > eps_abs                                 */
    int32_t normal_mode;        /* FRT_NORMAL_TETRA, _CENTRAL or _ANALYTIC   */
    int32_t refine_iters;       /* [0, 32]                                   */
    int32_t shadow;             /* 0 or 1                                    */
    float light_dir[3];         /* non-zero                                  */
    float albedo[3];
    float k_ambient, k_diffuse;
    int32_t shading;            /* FRT_SHADING_LAMBERT, or _PHONG (scenes)   */
    float k_specular;           /* >= 0 (Phong highlight weight)             */
    float shininess;            /* [1, 10000] (Phong exponent)               */
    float k_reflect;            /* [0, 1] (reflection weight); these three   */
                                /* are read only with FRT_SHADING_PHONG      */
    float trap_colour[4][3];    /* finite; albedo change per unit of each    */
                                /* trap component (read with _PHONG only)    */
} frt_march;

/* Output planes (device pointers, see the layout above).  depth, normal,
 * colour and status are required; counters may be NULL.                   */
typedef struct {
    float* depth;
    float* normal;
    float* colour;
    uint8_t* status;
    uint32_t* counters;
} frt_frame;

/* One render of a batch. */
typedef struct {
    frt_camera cam;
    frt_fractal frac;
    frt_plane planes[2];
    int32_t n_planes;           /* [0, 2]                                    */
    frt_march march;
    frt_frame out;
} frt_job;

/* Device workspace needed by a call over n_jobs renders (work-queue
 * counters, the job table and the adjoint's table of upstream-gradient
 * pointers, or the object table of jobs traced as one-object scenes).  Any
 * device allocation of at least this many bytes, 256-byte aligned, serves. */
size_t frt_workspace_bytes(int32_t n_jobs);

/* Render one view (the per-pixel path of Listings 2-5 and 7).
 * workspace: device memory of frt_workspace_bytes(1) bytes (ws_bytes).
 * Returns FRT_EINVAL (nothing launched) for invalid parameters, FRT_ENOMEM
 * when the workspace is too small, FRT_EHIP when a launch fails.           */
frt_status frt_render(const frt_camera* cam, const frt_fractal* frac, const frt_plane* planes,
                      int32_t n_planes, const frt_march* march, frt_frame out,
                      void* workspace, size_t ws_bytes, void* stream);

/* Render n_jobs independent views in one persistent launch per kernel
 * variant present (Julia of degree 2 or of higher degree, Mandelbulb with
 * real, integer or n = 8 power): the
 * rays of a variant's jobs form one index space that its waves drain through
 * a shared queue.
 * jobs: host array of n_jobs (>= 1) entries; workspace: device memory of
 * frt_workspace_bytes(n_jobs) bytes.  use_graph = 1 replays a HIP graph of
 * the launches captured on the first call with the same (workspace,
 * variants present, launch settings); the job table is re-uploaded before
 * every replay, so
 * parameters and output pointers may change between calls.  Without a
 * graph, the variants after the first run on the library's side streams of
 * the current device, forked from `stream` after the queue reset and joined
 * back into it before the call returns: the work is still ordered on
 * `stream` as a whole.
 * Errors as frt_render; a job's index appears in frt_last_error().         */
frt_status frt_render_batch(const frt_job* jobs, int32_t n_jobs, void* workspace, size_t ws_bytes,
                            int32_t use_graph, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * render as frt_render_batch with use_graph = 0 (same kernels, bit-identical
 * output), but its workspace is the library's own device scratch, a
 * file-scope device array of frt_noalloc_scratch_bytes() bytes (about
 * 140 KiB) that each GPU the library runs on holds until the process ends.
 * The call allocates nothing: no hipMalloc/hipFree, no pinned staging (the
 * job table travels in the arguments of small upload kernels), no events, no
 * graphs; it records no stage timing.  The caller still owns the output
 * planes named in jobs[i].out.
 * jobs: host array of n_jobs entries, 1 <= n_jobs <= FRT_NOALLOC_MAX_JOBS.
 * Every call on one GPU shares that GPU's scratch, which keeps the last
 * call's contents (the claim counters are cleared by each call's own
 * kernels): calls that overlap on one GPU -- on different streams, or from
 * different host threads without ordering -- race and must not be issued.
 * Errors as frt_render_batch; FRT_EINVAL also for n_jobs above the maximum. */
#define FRT_NOALLOC_MAX_JOBS 256
frt_status frt_render_batch_noalloc(const frt_job* jobs, int32_t n_jobs, void* stream);
size_t frt_noalloc_scratch_bytes(void);

/* Adjoint of a batch render (the gradient the renderer is differentiated
 * for, by implicit differentiation at the hit points; Sec. 2 gives the
 * orbit-derivative estimate d whose root the depth is):
 * for a refined hit, t* solves d(o + t dir) = eps_abs + eps_rel t, so
 *   d t* / d theta = -(dd/dtheta) / (grad d . dir - eps_rel);
 * normal (Eq. 5 / Listing 5 taps) and colour follow by the chain rule
 * through the taps, whose orbit tangents are recomputed (nothing from the
 * forward orbit is stored).  Cut-face hits use t* = (d - n_hat.o)/(n_hat.dir)
 * and normal n_hat, n_hat = n / |n|.  Exhausted and unrefined hits, misses
 * and the shadow visibility contribute nothing.
 * The result is, per job, the gradient of
 *   sum_p g_colour . colour + g_depth depth + g_normal . normal
 * with respect to theta = (c0..c3 | power | plane 0 raw n xyz, d |
 * plane 1 raw n xyz, d); slots a job does not use come out zero (power for
 * Julia jobs, whose degree is discrete; c for the Mandelbulb).
 * jobs: the forward jobs, with out.depth and out.status holding the forward
 *       results (the other out pointers are not read);
 * g_colour / g_depth / g_normal: host arrays of n_jobs device pointers to
 *       float[3][P] / float[P] / float[3][P] upstream gradients; an array
 *       or any entry may be NULL (zero);
 * grad_pixel: host array of n_jobs device pointers to float[13][P], or NULL
 *       (as may any entry): receives each pixel's contribution (zeros where
 *       none), for checking against a per-pixel reference;
 * grad_c [n_jobs][4], grad_power [n_jobs], grad_plane [n_jobs][2][4]:
 *       device outputs, overwritten (zeroed by the call, then accumulated
 *       with float atomics, so the last bits vary from run to run);
 * workspace: frt_workspace_bytes(n_jobs) bytes, not shared with a call in
 *       flight on another stream.
 * Errors: as frt_render_batch (validation before any launch, no writes);
 * FRT_EINVAL also for a null gradient output or a null depth / status;
 * FRT_EUNSUPPORTED for a job with analytic normals (their parameter
 * derivative needs second derivatives of the estimate, not provided).      */
frt_status frt_render_backward(const frt_job* jobs, int32_t n_jobs, const float* const* g_colour,
                               const float* const* g_depth, const float* const* g_normal,
                               float* const* grad_pixel, float* grad_c, float* grad_power, float* grad_plane,
                               void* workspace, size_t ws_bytes, void* stream);

/* One object of a scene (Sec. 3: every procedural object sits in its own
 * box with a transform from world space to its local space).  The map from
 * world to object space is the similarity x_obj = R^T (x - T) / s with
 * R = rotation (object-to-world, row-major, a proper rotation: R R^T = I to
 * 1e-4 and det R > 0), T = translation and s = scale > 0.  Distances scale
 * by s, so the estimate stays a distance bound (a general affine map would
 * not keep it one).  frac and planes are in object space; the fractal's
 * bounding sphere plays the role of the paper's box.                       */
typedef struct {
    frt_fractal frac;
    frt_plane planes[2];
    int32_t n_planes;           /* [0, 2]                                    */
    float rotation[9];
    float translation[3];
    float scale;
} frt_object;

/* Device workspace of frt_render_scene over n_objects objects (the
 * workspace header and the object table), 256-byte aligned.                 */
size_t frt_scene_workspace_bytes(int32_t n_objects);

/* Render one view of a scene of n_objects (1..16) objects in one launch.
 * Every primary ray is marched through each object in its own frame (the
 * world ray mapped by the object's similarity, with eps_abs, step_clamp and
 * t_max divided by its scale and eps_rel unchanged, so eps(t) stays a world
 * quantity) and the closest hit is kept, ties going to the lower index (the
 * closest-hit rule of the paper's intersection shaders).  The hit's normal
 * is computed in object space and mapped to world space by R; shading is
 * done in world space and the shadow ray of a lit hit is blocked by a hit
 * on any object.  march and out as in frt_render (depth in world units).
 * Counter planes 0-3 describe the primary march of the object hit (zero on
 * a miss), 4-5 its normal, 6-7 the shadow ray over all objects.  A miss is
 * a t_max miss when the ray entered any object's interval, else a bounds
 * miss.  object_id: int32[H*W] (device, may be NULL) receives the index of
 * the object hit, -1 on a miss.  trap: float[4][H*W] (device, may be NULL)
 * receives the orbit trap at the hit point in the object's frame (the
 * colour parameters of the Mandelbulb distance listing, defined here as the
 * minima of |x|, |y|, |z| and |w|^2 over the start point and every body of
 * the estimate's orbit; Julia: the first three quaternion components), 0 on
 * a miss.  With FRT_SHADING_PHONG, status bit 7 (128) marks pixels whose
 * reflection ray hit an object, and counter planes 6-7 count the shadow and
 * reflection rays together.
 * Errors: FRT_EINVAL (nothing launched) for invalid parameters, naming the
 * object; FRT_ENOMEM for a small workspace; FRT_EHIP for a failed launch. */
frt_status frt_render_scene(const frt_camera* cam, const frt_object* objects, int32_t n_objects,
                            const frt_march* march, frt_frame out, int32_t* object_id, float* trap,
                            void* workspace, size_t ws_bytes, void* stream);

/* Distance estimate (Sec. 2, Eq. 2-4) at n points, the same orbit code the
 * renderer marches with: points float[n][3] (device), d float[n] (device),
 * iters int32[n] (device, may be NULL) receives the escape count (max_iter:
 * no escape).  frac is validated as for frt_render.                        */
frt_status frt_distance(const frt_fractal* frac, const float* points, int64_t n, float* d, int32_t* iters,
                        void* stream);

/* Normal at n points by the renderer's rule for normal_mode (the normal
 * stage of Eq. 5 / Listing 5, or the analytic gradient of Sec. 2's remark,
 * without the march): points float[n][3] (device); eps float[n] (device)
 * the tap scale eps(t*) as in frt_march, ignored by FRT_NORMAL_ANALYTIC and
 * then allowed to be NULL; normals float[n][3] (device) receives unit
 * normals, (0, 0, 0) where the gradient is zero or not finite.  frac is
 * validated as for frt_render; FRT_EINVAL for an unknown mode or a NULL eps
 * with a tap mode.                                                          */
frt_status frt_normal_at(const frt_fractal* frac, int32_t normal_mode, const float* points, const float* eps,
                         int64_t n, float* normals, void* stream);

/* Evaluate one of the library's fast float32 functions on n device values,
 * for accuracy checks: func 0 acos(x) (x clamped to [-1, 1]), 1 atan2(x, y),
 * 2 sin(2 pi x), 3 cos(2 pi x), 4 log2(x), 5 exp2(x), 6 1/sqrt(x), 7 1/x.
 * y is read only by func 1.                                                 */
frt_status frt_math_eval(int32_t func, const float* x, const float* y, float* out, int64_t n, void* stream);

/* Measurement utility, not a step of the method: the sustained device-wide
 * issue rate of one FP32 vector operation, for the ceilings the march
 * kernels are measured against (the kernels are bound by the vector unit).
 * op: 0 FMA, 1 exp2, 2 log2, 3 1/sqrt, 4 1/x, 5 sqrt, 6 sin(2 pi x),
 * 7 a mix of four dependent FMAs per exp2 (whether transcendentals overlap
 * FMAs), 8 FP32 add, 9 FP32 multiply, 10 an integer shift and add (the
 * rate of non-FP32 vector instructions).  Each lane of 8 workgroups of 256
 * threads per compute unit runs eight independent chains for iters rounds,
 * iters in [1, 1 << 20]; op 7 counts five operations per chain and round,
 * op 10 two.  *lane_ops_per_s receives
 * the lane operations per second of one timed launch (after one untimed
 * launch); an FMA is one operation (two FLOP).  Allocates and frees a
 * device buffer of 1 KiB per workgroup and waits for the launches on
 * stream.  FRT_EINVAL for an unknown op, iters out of range or a null
 * output; FRT_EHIP for a failed HIP call.                                   */
frt_status frt_valu_rate(int32_t op, int32_t iters, double* lane_ops_per_s, void* stream);

/* Launch configuration of the persistent kernels, chosen by the autotuner.
 * kernel_variant: 0 Julia z^2 + c, 1 Mandelbulb (real n), 2 Mandelbulb
 * (integer n), 3 Mandelbulb with n = 8 (the power the paper renders),
 * 4 Julia z^p + c with p >= 3.  A batch is traced
 * as one group of rays per variant present, each with its own setting.
 * block: 64, 128, 256 or 512 threads; chunk: rays taken from the queue per
 * refill, a multiple of 64 in [64, 4096]; waves_per_simd: resident waves per
 * SIMD the grid is sized for, [1, 8] (0 = occupancy limit);
 * orbit_lanes: the wave keeps advancing orbits while at least this many
 * of its lanes still iterate, then lanes whose estimate is done take their
 * next step (1: every orbit runs to its end first), [1, 64];
 * rare_lanes: number of waiting lanes that triggers shading, output writes
 * and refill, [1, 64].  The setting is process-wide and applies to launches
 * that start after the call.                                               */
frt_status frt_autotune_set(int32_t kernel_variant, int32_t block, int32_t chunk, int32_t waves_per_simd,
                            int32_t orbit_lanes, int32_t rare_lanes);
frt_status frt_autotune_get(int32_t kernel_variant, int32_t* block, int32_t* chunk, int32_t* waves_per_simd,
                            int32_t* orbit_lanes, int32_t* rare_lanes);

/* Per-stage timing of the forward pass.  While enabled (enable = 1), each
 * frt_render / non-graph frt_render_batch call records HIP events on its
 * stream around its three kernels; frt_stage_times() waits for the last
 * call's events and writes the durations in ms of the primary march, the
 * normal kernel and the shadow march (0 when no shadow rays) to ms[0..2].
 * Process-wide; meant for benchmarking, not for concurrent streams.        */
frt_status frt_set_stage_timing(int32_t enable);
frt_status frt_stage_times(float* ms);

/* Drop every captured batch graph; the next graph call captures again.     */
frt_status frt_graph_reset(void);

/* Static description of a status code.                                     */
const char* frt_status_string(frt_status s);

/* Message of the last failed call on this thread (empty if none); valid
 * until the next frt_* call on the same thread.                            */
const char* frt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FRT_H */
