/*
 * ugp.h -- C ABI of libugp: Monte Carlo path tracing of scenes made entirely of
 * linear-transmittance Gaussian primitives on AMD Instinct MI355X (gfx950).
 *
 * Method: "Unified Gaussian Primitives for Scene Representation and Rendering"
 * (arXiv 2406.09733).  The entry points are the scene operations a path tracer
 * needs (Sec. 5, table tab:highlevel, right column): free-flight (primitive)
 * sampling, transmittance evaluation, and a full path tracer with next-event
 * estimation built on them.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers (e.g. torch tensor storage on the
 *    context's device) unless marked [host].  The caller owns them.
 *  - Work is enqueued on the context's stream and the call returns without
 *    waiting, except where stated.  Inputs must stay alive until the stream
 *    has consumed them (torch's caching allocator on the same stream does this).
 *  - Rays are float32 [n][8] = (origin.xyz, direction.xyz, t0, t1), direction of
 *    unit length, t1 may be +inf.  The ray is x(t) = origin + t * direction,
 *    t in [t0, t1] (Sec. 4.1 "Ray Integral").  The per-ray queries validate
 *    each ray on the device (the host never reads the data): a non-finite
 *    origin, direction or t0, a NaN t1, or a direction whose length differs
 *    from 1 by more than 1e-3 makes that ray's outputs NaN (primitive -1)
 *    without tracing it, leaves every other ray's results unchanged, and is
 *    reported once by the next ugp_sync as UGP_ERR_INVALID_ARGUMENT.
 *  - Primitive indices in and out are the caller's original indices
 *    (0 .. n-1 in the order the scene was given); -1 means "none".
 *  - Problems a host check can see (NULL required pointer, bad sizes, eps
 *    outside (0,1), no scene) return UGP_ERR_INVALID_ARGUMENT / UGP_ERR_NO_SCENE
 *    and enqueue nothing.  Device failures return UGP_ERR_DEVICE.  No C++
 *    exception crosses this boundary and nothing aborts.
 *  - One host thread uses a context at a time.
 */
#ifndef UGP_H
#define UGP_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ugp_ctx_s *ugp_ctx;

typedef enum {
    UGP_OK = 0,
    UGP_ERR_INVALID_ARGUMENT = 1,
    UGP_ERR_OUT_OF_MEMORY = 2,
    UGP_ERR_DEVICE = 3,
    UGP_ERR_NO_SCENE = 4,
    UGP_ERR_UNSUPPORTED = 5,
    UGP_ERR_OVERFLOW = 6
} ugp_status;

/* [host] struct of DEVICE pointers describing n primitives (Sec. 3.1, Sec. 4,
 * Sec. 6).  All float32 unless noted.
 *   mean[n][3]      mean mu
 *   scale[n][3]     per-axis scale s (> 0); Sigma = (R S)(R S)^T (eq. covariance_decomposition)
 *   rotation[n][4]  quaternion (w, x, y, z) of R, any non-zero norm (normalised here)
 *   density[n]      peak value d = G(mu) >= 0 (the paper's magnitude c equals
 *                   d (2 pi)^(3/2) s_x s_y s_z)
 *   albedo[n][3]    base colour: Lambert albedo, or GGX F0
 *   roughness[n]    GGX roughness in (0, 1]; alpha = roughness^2
 *   emission[n][3]  emitted radiance (0 = not an emitter)
 *   material[n]     int32: 0 = diffuse (Lambert), 1 = glossy (GGX): the delta-NDF
 *                   limit of eq. phase_function with the facet normal along the
 *                   axis of the smallest scale; 2 / 3 = SGGX microflakes (Sec.
 *                   4.2, eq. vndf and eq. phase_function: stochastic evaluation
 *                   with internal MIS, visible-normal sampling, the approximate
 *                   MIS pdf of App. B) with a Lambertian base BSDF (2) or a
 *                   Disney-style base (3): a diffuse lobe with retro-reflection,
 *                   weight 1 - metallic, and a GGX specular lobe (alpha =
 *                   roughness^2) with Schlick F0 = 0.04 (1 - metallic) +
 *                   albedo metallic
 *   sggx[n][6]      SGGX matrix S per primitive (xx, yy, zz, xy, xz, yz), world
 *                   frame, symmetric positive definite; may be NULL when no
 *                   primitive has material 2 or 3.  When given, every row is
 *                   checked (leading minors > 0, finite) and a bad row fails the
 *                   build with UGP_ERR_INVALID_ARGUMENT, as do materials 2 and 3
 *                   with NULL
 *   metallic[n]     metallic of material 3 in [0, 1] (checked); NULL = 0       */
typedef struct {
    int64_t n;
    const float *mean, *scale, *rotation, *density, *albedo, *roughness, *emission;
    const int32_t *material;
    const float *sggx;
    const float *metallic;
} ugp_scene;

/* [host] pinhole camera: pixel (i, j), j = 0 at the top, jitter (jx, jy) in
 * [0,1)^2 maps to direction normalize(f + sx*right + sy*up) with
 * sx = (2 (i + jx) / width - 1) tan(vfov/2) width/height,
 * sy = (1 - 2 (j + jy) / height) tan(vfov/2),
 * f = normalize(target - origin), right = normalize(f x up_hint), up = right x f. */
typedef struct {
    float origin[3], target[3], up[3];
    float vfov_deg;
    int32_t width, height;
} ugp_camera;

/* [host] render settings.
 *   spp            samples per pixel of this call (>= 1)
 *   max_depth      number of scattering events per path (>= 0); emission is
 *                  still picked up at collision max_depth + 1
 *   seed           key of the Philox4x32-10 generator; counters are
 *                  (pixel, sample_offset + s, vertex, group)
 *   sample_offset  first sample index, so progressive calls resume exactly
 *   env_radiance   constant environment radiance (0 = black background)
 *   mis_mode       0 balance heuristic, 1 phase sampling only, 2 light sampling only
 *   nrc_mode       neural radiance cache (the learned cache that ends paths early):
 *                  0 off (plain tracer);
 *                  1 infer and train: a path is a training path with probability
 *                    f (Philox vertex 0, group 2); other paths end at collision
 *                    nrc_terminate_after + 1 (if <= max_depth) where, after
 *                    the emission pick-up, throughput x max(0, cache) is
 *                    added; training paths run to max_depth and record every
 *                    scattering vertex; after each sample pass the records'
 *                    targets (path radiance - radiance so far) / throughput
 *                    drive nrc_train_steps Adam steps (as ugp_nrc_train_step)
 *                    after every chunk of samples (see ugp_render) and f is
 *                    rescaled toward nrc_train_records records per chunk.
 *                    Up to 4 x nrc_train_records records of a chunk are
 *                    kept and ordered by path (a fixed shuffle of the paths,
 *                    each path's records in vertex order), and the first
 *                    nrc_train_records of them are trained on, so the
 *                    training and every later image repeat exactly from
 *                    run to run (as long as no chunk attempts more than
 *                    that: ugp_render_stats.nrc_records);
 *                  2 infer only (every path ends in the cache);
 *                  3 end paths at nrc_terminate_after + 1 and add nothing
 *   nrc_terminate_after  scattering events before a cached path ends (>= 1)
 *   nrc_train_records    records used per training step, 1 .. 1 << 20 (mode 1);
 *                  f starts at min(1, nrc_train_records / (8 paths of a chunk))
 *   nrc_lr         Adam learning rate of the cache (0 = 1e-2)
 *   nrc_box        lo[3], hi[3] of the cache's position encoding; hi <= lo on
 *                  any axis = the scene bounds
 *   nrc_train_steps  Adam steps per chunk, on consecutive batches of the
 *                  chunk's records (0 = 1)
 *   nrc_radiance_scale  radiance unit of the network's output (targets are
 *                  divided by it, predictions multiplied); 0 = keep the
 *                  current unit, which the first training after
 *                  ugp_nrc_set_weights sets to the mean of its targets
 *   nrc_target_clamp  training targets (in that unit) are clamped at this
 *                  value in the loss (0 = no clamp)
 *   transport      0 the paper's linear transmittance; 1 its exponential
 *                  variant (App. D, eq. exp_ff; the baseline of the paper's
 *                  comparison of transmittance models): the Gaussians as a
 *                  medium with sigma_t = sum_k G_k, a path's collisions and
 *                  light samples drawn by analog decomposition tracking (the
 *                  uniform of Gaussian k at vertex v: the path's generator
 *                  with group 16 + 2k, or 17 + 2k for the light sample), a
 *                  light sample scoring if its target is hit first along the
 *                  segment to the target's chord exit, environment samples
 *                  weighted by exp(-sum_k I_k), and no primitive skipped after
 *                  a scatter (it happens inside the Gaussian).  Requires
 *                  nrc_mode 0; no adjoint entry point takes it (UGP_ERR_UNSUPPORTED). */
typedef struct {
    int32_t spp, max_depth;
    uint64_t seed;
    int64_t sample_offset;
    float env_radiance[3];
    int32_t mis_mode;
    int32_t nrc_mode, nrc_terminate_after, nrc_train_records;
    float nrc_lr;
    float nrc_box[6];
    int32_t nrc_train_steps;
    float nrc_radiance_scale;
    float nrc_target_clamp;
    int32_t transport;
} ugp_render_params;

/* Create a context on `device` that enqueues on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  Allocates nothing on the device until a scene is
 * built.  Returns UGP_ERR_DEVICE if the device is not a usable gfx950. */
ugp_status ugp_create(int device, void *hip_stream, ugp_ctx *out);
ugp_status ugp_destroy(ugp_ctx ctx);
ugp_status ugp_set_stream(ugp_ctx ctx, void *hip_stream);

/* Build the scene: pack the primitives (normalise rotations, form the
 * world-to-unit-Gaussian map M = S^-1 R^T, the facet normal and the box of the
 * cut-off ellipsoid |M (x - mu)| = sqrt(-2 ln eps), eq. cutoff_threshold) and
 * build a bounding volume hierarchy over those boxes on the GPU.  The scene is
 * copied into library-owned memory (leaf order), so the input arrays may be
 * freed once the stream passes this call.  eps in (0, 1); the paper uses 0.01.
 * Synchronises the stream once (to size the tree).  n >= 1. */
ugp_status ugp_build_bvh(ugp_ctx ctx, const ugp_scene *scene, float cutoff_eps);

/* New parameters for the same n primitives without a new hierarchy: the
 * records are packed again and every box of the built hierarchy is refitted
 * bottom-up, keeping its topology and the slab layout of each primitive (cut
 * primitives keep their slab count and axis, which still cover the new
 * ellipsoid).  Queries and renders then give the new scene's results; only
 * the hierarchy's quality (node visits per ray) can degrade as primitives
 * move, so a caller rebuilds from time to time.  For optimisation loops that
 * move primitives a little per step (Sec. 7.2 rebuilds its structure every
 * iteration).  scene->n must equal the built scene's n
 * (UGP_ERR_INVALID_ARGUMENT); invalid parameters (as ugp_build_bvh) return
 * UGP_ERR_INVALID_ARGUMENT and leave the scene unchanged; UGP_ERR_NO_SCENE
 * before a build.  The emitter list and the scene bounds are updated.
 * Synchronises the stream (validation, emitter count). */
ugp_status ugp_refit_bvh(ugp_ctx ctx, const ugp_scene *scene);

/* Transmittance along each ray (Sec. 4 eq. transmittance, Sec. 5.3):
 * F = 1/2 sum_k I_k(a_k, b_k) over every primitive k != exclude[i] whose
 * cut-off ellipsoid meets [t0, t1] in the chord [a_k, b_k], with I_k the
 * closed-form ray integral (App. A); T = max(0, 1 - F).
 *   exclude  int32 [n] original indices, or NULL (none)
 *   T_out    float [n]
 *   F_out    float [n] or NULL.  If given, F is the full sum (no early exit at
 *            F >= 1); if NULL the traversal stops once F reaches 1 (T = 0). */
ugp_status ugp_transmittance(ugp_ctx ctx, int64_t n_rays, const float *rays,
                             const int32_t *exclude, float *T_out, float *F_out);

/* Primitive-level free-flight sampling (Sec. 5.2, Sec. 4.1 eq.
 * sampling_overlaps): with the saturating distance t_sat (smallest t with
 * F(t) = 1, or t1 if F never reaches 1) each primitive k is selected with
 * probability W_k = 1/2 I_k(a_k, min(b_k, t_sat)) and the ray escapes with
 * probability max(0, 1 - F(t1)).  One uniform u[i] in [0,1) picks the outcome
 * deterministically: primitives are ordered by exit key (min(b_k, t_sat), k)
 * and the first k whose running sum of W exceeds u is returned.
 *   u         float [n]
 *   prim_out  int32 [n] selected original index, -1 = escape
 *   t_out     float [n] scatter distance 1/2 (a_k + b_k), the centre of the
 *             clipped chord (Sec. 6 "Importance Sampling"); NaN on escape.
 * Returns UGP_ERR_OVERFLOW (and leaves those outputs at -1 / NaN) if more than
 * 64 primitives overlap a single point of a ray. */
ugp_status ugp_sample_collision(ugp_ctx ctx, int64_t n_rays, const float *rays,
                                const int32_t *exclude, const float *u, int32_t *prim_out,
                                float *t_out);

/* Allocation-free variant of ugp_sample_collision, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Arguments, results and errors as
 * ugp_sample_collision, except:
 *  - n_rays at most UGP_NOALLOC_MAX_RAYS; a larger n_rays returns
 *    UGP_ERR_INVALID_ARGUMENT and enqueues nothing.
 *  - The call allocates nothing (no hipMalloc, hipFree, stream-ordered or
 *    library allocation; no memset node).  Its working memory (the list of
 *    rays that overflow the 16-entry buffer and the saved states they resume
 *    from) is one fixed 32 MiB buffer per GPU, a device array of the library
 *    that each GPU it runs on holds until the process ends; its address is
 *    taken in ugp_create.  Overflowing rays beyond the first ones whose saved
 *    states fit (at least 58,000) restart in the 64-entry pass instead of
 *    resuming (the same result up to float rounding of t).  UGP_ERR_DEVICE if
 *    the buffer is unavailable.
 *  - Every call on one GPU shares that buffer and the previous call's
 *    contents remain in it (each call clears what must start at zero): calls
 *    that overlap on one GPU -- other streams, contexts or threads -- race, and
 *    the caller serialises them. */
#define UGP_NOALLOC_MAX_RAYS 4194304
ugp_status ugp_sample_collision_noalloc(ugp_ctx ctx, int64_t n_rays, const float *rays,
                                        const int32_t *exclude, const float *u, int32_t *prim_out,
                                        float *t_out);

/* Saturating distance per ray: smallest t in [t0, t1] with F(t) = 1 (Sec. 4,
 * below eq. free_flight_pdf), or t1 when F(t1) < 1.  tsat_out float [n]. */
ugp_status ugp_saturation(ugp_ctx ctx, int64_t n_rays, const float *rays,
                          const int32_t *exclude, float *tsat_out);

/* Emission factor of primitive target[i] along each ray: emission rides on the
 * free-flight pdf (eq. rte), so target k contributes L_e,k times
 *   out = 1/2 I_k(a_k, min(b_k, t_sat))
 * where the ray is clipped to [t0, b_k] and t_sat is taken over every primitive
 * except exclude[i] (k included); 0 if the ray misses k or k == exclude[i].
 * This is the light-sampling query of next-event estimation. */
ugp_status ugp_emitter_query(ugp_ctx ctx, int64_t n_rays, const float *rays,
                             const int32_t *exclude, const int32_t *target, float *out);

/* Test hook of the ray integral (Sec. 4.1 eq. ray_integral; App. A closed
 * form): for each ray i and primitive prim[i] (original index), the integral
 * of that primitive's cut-off kernel over the part of its chord inside
 * [t0, t1], I = d sqrt(pi/(2A)) exp(-rho^2/2) [erf tau_b - erf tau_a]
 * (erfc differences in the tails); 0 where the ray misses it.  Computed by the
 * same device code as the queries above.  I_out float [n].  A prim[i] outside
 * [0, n) gives NaN and is reported by ugp_sync as an invalid argument. */
ugp_status ugp_ray_integral(ugp_ctx ctx, int64_t n_rays, const float *rays, const int32_t *prim,
                            float *I_out);

/* Test hook of the counter-based generator every random number of the path
 * tracer is drawn from: Philox4x32-10 (Salmon et al., SC'11) of counters
 * uint32 [n][4] under key (key low 32 bits, key high 32 bits); out uint32
 * [n][4].  No scene is needed. */
ugp_status ugp_philox(ugp_ctx ctx, int64_t n, const uint32_t *counters, uint64_t key, uint32_t *out);

/* ---- Exponential variant (App. D; eq. exp_ff) ----------------------------
 * The same Gaussians read as a heterogeneous exponential medium, sigma_t =
 * sum_k G_k (the comparison variant of the paper's linear-vs-exponential
 * study).  Rays and exclude as the queries above.
 *
 * Transmittance exp(-sum_k I_k(a_k, b_k)) over the clipped chords (the full
 * ray integrals).  T_out float [n]. */
ugp_status ugp_exp_transmittance(ugp_ctx ctx, int64_t n_rays, const float *rays, const int32_t *exclude,
                                 float *T_out);

/* Free-flight sampling by analog decomposition tracking (App. D): every
 * Gaussian k the ray meets draws u_k -- Philox4x32-10, counter (ray index
 * low, ray index high, k, 0), key (seed low, seed high), the top 24 bits of
 * the first word over 2^24 -- and would collide where its optical depth from
 * the chord entry reaches -ln(1 - u_k), if that happens before the chord
 * exit; the ray collides at the nearest such point.  prim_out int32 [n]
 * (original index, -1 = escape), t_out float [n] (NaN on escape). */
ugp_status ugp_exp_sample_collision(ugp_ctx ctx, int64_t n_rays, const float *rays, const int32_t *exclude,
                                    uint64_t seed, int32_t *prim_out, float *t_out);

/* ---- Differentiation: the transmittance optimisation of Sec. 7.2 ---------
 *
 * Accumulated free-flight CDF of each ray (Sec. 7.2, eq. accum_cdf):
 *   C = sum_k 1/2 I_k(a_k, min(b_k, t_sat)),
 * the clipped chords of every primitive except exclude[i], t_sat the ray's
 * saturating distance (as ugp_saturation; t1 when the ray never saturates).
 *   C_out     float [n] or NULL
 * With target (float [n], e.g. one minus a reference transmittance image):
 *   loss_out  [device] float, += loss_scale * sum_i (C_i - target_i)^2, or NULL
 *   grad      float [scene->n][11], += the gradient of that loss with respect
 *             to (mean[3], scale[3], rotation[4] (w,x,y,z, unnormalised as
 *             given), density) of every primitive, or NULL.  As in Sec. 7.2,
 *             each primitive's term is differentiated with t_sat held fixed.
 * scene: the parameters the hierarchy was built from (read for the rotation
 * and scale chain rule); required with grad.  All arrays are device memory,
 * owned by the caller; NULL outputs are skipped.  Enqueued on the stream;
 * temporary buffers are stream-ordered allocations. */
ugp_status ugp_accum_cdf(ugp_ctx ctx, const ugp_scene *scene, int64_t n_rays, const float *rays,
                         const int32_t *exclude, const float *target, float loss_scale, float *C_out,
                         float *loss_out, float *grad);

/* Radiance-field mode (Sec. 8, eq. rf): with emission and absorption only,
 * the radiance along each ray is
 *   L = sum_k 1/2 I_k(a_k, min(b_k, t_sat)) L_e,k,
 * the primitives' free-flight probabilities up to the saturating distance
 * times their emission (the scene's emission, view-independent as in Sec. 8),
 * with no Monte Carlo.  Arguments as ugp_accum_cdf, but per ray three
 * channels: L_out float [n][3] or NULL; target float [n][3]; loss_out +=
 * loss_scale * sum_i |L_i - target_i|^2; grad float [scene->n][14] += its
 * gradient with respect to (mean[3], scale[3], rotation[4], density,
 * emission[3]), t_sat held fixed. */
ugp_status ugp_rf_render(ugp_ctx ctx, const ugp_scene *scene, int64_t n_rays, const float *rays,
                         const int32_t *exclude, const float *target, float loss_scale, float *L_out,
                         float *loss_out, float *grad);

/* Vector-Jacobian products of the two images above, for a caller's own loss
 * (e.g. an autograd engine): with dC = dLoss/dC given per ray,
 *   grad += sum_i dC_i dC_i/d(parameters),
 * the same derivative as the fused loss gradient (Sec. 7.2: each primitive's
 * term with t_sat held fixed), in the same layouts.
 *   dC    float [n] (ugp_accum_cdf_backward) or dL float [n][3]
 *         (ugp_rf_render_backward)
 *   grad  float [scene->n][11] (mean, scale, rotation, density) or [n][14]
 *         (+ emission), added to
 * scene: the parameters the current hierarchy was built from.  Device memory
 * owned by the caller; dC and grad are required (UGP_ERR_INVALID_ARGUMENT,
 * as is a scene whose n differs from the built one); UGP_ERR_NO_SCENE before
 * a build.  Enqueued on the stream; temporaries are stream-ordered. */
ugp_status ugp_accum_cdf_backward(ugp_ctx ctx, const ugp_scene *scene, int64_t n_rays, const float *rays,
                                  const int32_t *exclude, const float *dC, float *grad);
ugp_status ugp_rf_render_backward(ugp_ctx ctx, const ugp_scene *scene, int64_t n_rays, const float *rays,
                                  const int32_t *exclude, const float *dL, float *grad);

/* One jittered pinhole ray per pixel of cam (row-major, rays [w*h][8] as the
 * queries take them, t in [0, inf)); the sub-pixel jitter is the renderer's
 * camera jitter of sample `sample` (counter-based generator keyed on seed,
 * pixel, sample).  Sec. 7.2: one jittered ray per pixel per view. */
ugp_status ugp_camera_rays(ugp_ctx ctx, const ugp_camera *cam, uint64_t seed, int64_t sample, float *rays);

/* One Adam step (Kingma and Ba; beta = (0.9, 0.999), eps = 1e-8) on the
 * primitive parameters.  emission NULL: gradient grad [n][11] (the layout of
 * ugp_accum_cdf); emission [n][3]: grad [n][14] (the layout of ugp_rf_render).
 * Moments m and v have the gradient's layout (zero before step 1); step >= 1.
 * lr [host] float[5]: the rates of the means, of the scales, of the
 * rotations, of the densities and of the emissions (ignored without).
 * Scales step on log s (moments of s dL/ds; s is multiplied by exp(-step)),
 * so their rate is relative to each primitive's extent; the others step
 * linearly.  Then, as in Sec. 7.2, scales are clamped to at least min_scale
 * (> 0), densities and emissions to at least 0, rotations renormalised.
 * Arrays are device memory, updated in place. */
ugp_status ugp_fit_adam(ugp_ctx ctx, int64_t n, float *mean, float *scale, float *rotation, float *density,
                        float *emission, const float *grad, float *m, float *v, int32_t step, const float lr[5],
                        float min_scale);

/* Instrumentation: runs the ordered sweep of ugp_sample_collision (mode 0),
 * ugp_saturation (mode 1) or ugp_emitter_query (mode 2) and writes, per ray,
 * counts int32 [n][4] = (BVH nodes fetched, primitive records chord-tested,
 * primitive records re-read for partial integrals, traversal rounds).  Other
 * arguments as in those calls; results are discarded. */
ugp_status ugp_trace_counts(ugp_ctx ctx, int mode, int64_t n_rays, const float *rays,
                            const int32_t *exclude, const float *u, const int32_t *target,
                            int32_t *counts);

/* Path tracing (Sec. 5 table tab:highlevel, eq. rte) with next-event
 * estimation to emissive primitives and to the environment and the balance
 * heuristic against phase sampling.  A light sample picks an emissive
 * primitive uniformly and aims at a point drawn from its untruncated Gaussian
 * (the solid-angle pdf in closed form; none is taken from inside the emitter's
 * cut-off ellipsoid).  Adds, per pixel, the sum over this call's
 * samples of the path radiance to sum_rgb [height][width][3] and of its square
 * to sumsq_rgb (or NULL).  The samples are traced in chunks of
 * max(1, min(spp, 2^25 / pixels)) samples of every pixel, all paths of a
 * chunk in flight together (about 230 B of device memory per path, 7.6 GB at
 * 2^25 paths, held by the context until ugp_destroy).  The sums do not depend
 * on that scheduling.  Synchronises the stream once
 * per bounce iteration (to read two queue counters). */
ugp_status ugp_render(ugp_ctx ctx, const ugp_camera *cam, const ugp_render_params *p,
                      float *sum_rgb, float *sumsq_rgb);

/* Gradient of a loss of the rendered image with respect to every primitive's
 * albedo (the shading adjoint of the path tracer of eq. rte), by path
 * replay: each chunk of paths is traced as ugp_render traces it, then again
 * with the same random numbers, and at every scattering vertex the radiance
 * that passes through it is weighted by the derivative of its phase function
 * (Sec. 4.2; linear in the albedo: albedo/pi cos for the diffuse lobe, the
 * Schlick term albedo + (1 - albedo) m of the glossy one).  No sampling
 * decision depends on the albedo, so this is the exact derivative of the
 * estimate that ugp_render returns for the same arguments.
 *   d_image      [device] float [height][width][3]: dLoss / d(image), the
 *                image being the per-pixel mean over the spp samples (sum / spp)
 *   grad_albedo  [device] float [scene n][3] by original index, added to
 *   sum_rgb      [device] float [height][width][3] or NULL: the forward pass's
 *                per-pixel sum is added to it (as ugp_render's)
 * p->nrc_mode and p->transport must be 0 and the scene may hold no material 3
 * (UGP_ERR_UNSUPPORTED otherwise); other arguments and errors as ugp_render.
 * A diffuse channel of zero albedo reports a zero gradient (the replay
 * divides the albedo out).
 * Temporaries (three float4 per radiance slot) are stream-ordered. */
ugp_status ugp_render_albedo_grad(ugp_ctx ctx, const ugp_camera *cam, const ugp_render_params *p,
                                  const float *d_image, float *grad_albedo, float *sum_rgb);

/* Roughness adjoint of a render by the same path replay: at every scattering
 * vertex the radiance that passes through it is weighted by d log f / d
 * roughness of its phase function at the direction taken there (the glossy
 * delta-NDF lobe of Sec. 4.2: GGX D and Smith G2 with alpha = roughness^2;
 * 0 for Lambert and SGGX-Lambert vertices and for roughness <= 0.01, where
 * alpha is clamped).  Sampling pdfs and MIS weights are held at their values;
 * the phase sample is an importance sample of f and the MIS weights sum to
 * one for every roughness, so this is an unbiased estimate of the derivative
 * of the expected image (the sampled directions themselves move with the
 * roughness, so it is not the derivative of one estimate).
 *   grad_roughness [device] float [scene n] by original index, added to
 * other arguments, errors and restrictions as ugp_render_albedo_grad. */
ugp_status ugp_render_roughness_grad(ugp_ctx ctx, const ugp_camera *cam, const ugp_render_params *p,
                                     const float *d_image, float *grad_roughness, float *sum_rgb);

/* Density adjoint of a render (the derivative of the expected image with
 * respect to every primitive's peak density d), by the same path replay.
 * Densities enter only through the free-flight distribution (Sec. 4.1 eq.
 * sampling_overlaps: a collision selects primitive k with probability
 * W_k = 1/2 I_k(a_k, min(b_k, t_sat)) and escapes with probability
 * T = 1 - F) and through the weights of light samples (the emitter factor
 * W_k, eq. rte) and environment samples (T); scatter points, directions,
 * throughputs and MIS weights do not depend on them.  So each collision adds
 * the radiance its path collects from there on times d log W_k / d d_j (or
 * d log T / d d_j on an escape), and each light or environment sample adds
 * its contribution's derivative: I_j is linear in d_j, and t_sat moves by
 * -(W_j(t_sat) / d_j) / F'(t_sat) with F' = 1/2 sum G (eq. free_flight_pdf).
 * The result is an unbiased estimate of the derivative of the expected image
 * (a score-function estimate: not the derivative of one estimate, whose
 * discrete choices do not move with d).  Each collision and sample is traced
 * again, up to three times (t_sat, F', the terms).
 *   grad_density [device] float [scene n] by original index, added to (no
 *                gradient for primitives of zero density)
 * p->nrc_mode and p->transport must be 0 (UGP_ERR_UNSUPPORTED); other
 * arguments and errors as ugp_render_albedo_grad; every material is
 * supported. */
ugp_status ugp_render_density_grad(ugp_ctx ctx, const ugp_camera *cam, const ugp_render_params *p,
                                   const float *d_image, float *grad_density, float *sum_rgb);

/* The albedo, roughness and density adjoints above from one forward pass and
 * one replay of the same paths (the three calls each trace and replay the
 * paths again): each gradient pointer is a [device] buffer laid out as in its
 * own call, added to, or NULL when that gradient is not wanted; at least one
 * must be given (else UGP_ERR_INVALID_ARGUMENT).  The restrictions of every
 * requested adjoint apply (UGP_ERR_UNSUPPORTED); the results equal the
 * separate calls' on the same parameters up to the order of floating-point
 * atomic additions. */
ugp_status ugp_render_grads(ugp_ctx ctx, const ugp_camera *cam, const ugp_render_params *p, const float *d_image,
                            float *grad_albedo, float *grad_roughness, float *grad_density, float *sum_rgb);

/* Test hook of the SGGX phase functions (materials 2 and 3; Sec. 4.2 and
 * App. B) for n independent queries (DEVICE arrays, float32):
 *   sggx[n][6]  S (xx, yy, zz, xy, xz, yz), positive definite
 *   base[n][5]  albedo (rgb), roughness, metallic of a Disney-style base
 *               (material 3); NULL = Lambertian base of unit albedo (material 2)
 *   dirs[n][6]  w_o (unit, pointing away from the primitive), w_i (unit)
 *   u[n][12]    uniforms in [0,1): u0..u5 drive the evaluation (u0,u1 the
 *               visible normal; material 2: u2,u3 a normal cosine-distributed
 *               about w_i; material 3: u2,u3 a GGX normal about the half
 *               vector, u4,u5 a normal cosine-distributed about w_i); u6,u7 the
 *               sample's visible normal, u8..u10 its base-BSDF sample
 *               (material 2: cosine from u8,u9; material 3: lobe u8, direction
 *               u9,u10); u11 unused
 *   out[n][12]  f_p estimate (rgb), approximate MIS pdf at (w_i, w_o), sampled
 *               direction (3), its weight f/pdf (rgb), its approximate pdf,
 *               1 if a direction was sampled else 0
 * A query whose S is not positive definite gets NaN in every output.
 * Enqueued on the context's stream; no scene is needed. */
ugp_status ugp_sggx_phase(ugp_ctx ctx, int64_t n, const float *sggx, const float *base, const float *dirs,
                          const float *u, float *out);

/* Waits for the context's stream and reports deferred device-side errors,
 * clearing them: UGP_ERR_INVALID_ARGUMENT if a query since the last sync was
 * given a ray that failed the device's validation (see the ray convention
 * above), else UGP_ERR_OVERFLOW after a queue, stack or event-buffer
 * overflow. */
ugp_status ugp_sync(ugp_ctx ctx);

/* [host] statistics of the last ugp_render call.  A "ray" is one traversal
 * query: a free-flight (collision) query, a light-sample emitter query or an
 * environment transmittance query. */
typedef struct {
    int64_t paths;           /* camera paths (pixels x samples) */
    int64_t collision_rays;  /* free-flight sampling queries */
    int64_t light_rays;      /* emitter queries of next-event estimation */
    int64_t env_rays;        /* environment transmittance queries */
    int64_t node_visits;     /* BVH nodes fetched by all queries (profiling level 2, else -1) */
    int64_t prim_tests;      /* primitive records fetched and chord-tested (level 2, else -1) */
    int64_t prim_reloads;    /* primitive records re-read for partial integrals (level 2, else -1) */
    double ms_collide;       /* summed duration of the main collision kernel launches (level >= 1, else -1) */
    double ms_collide_wide;  /* ... of the overflow collision launches */
    double ms_light;         /* ... of the light-sample kernels (main + overflow) */
    double ms_env;           /* ... of the environment kernels */
    double ms_shade;         /* ... of the shading / path-compaction kernels */
    double ms_sort;          /* ... of the ray-sorting kernels */
    int32_t launches_collide, launches_light, launches_env;
    /* the three traversal counters split by kernel: [0] collision, [1] collision
       overflow pass and tail kernel, [2] light samples, [3] environment samples
       (level 2, else -1) */
    int64_t cat_nodes[4], cat_prims[4], cat_reloads[4];
    int64_t nrc_queries;     /* paths that ended in the radiance cache */
    int64_t nrc_records;     /* training records attempted, summed over chunks (before the caps) */
    double ms_nrc_infer;     /* duration of the cache inference launches (level >= 1, else -1) */
    double ms_nrc_train;     /* ... of the cache training steps */
    float nrc_loss;          /* loss of the last training step (NaN if none) */
    double ms_tail;          /* duration of the tail kernel launches (level >= 1, else -1) */
} ugp_render_stats;

/* Profiling level of later ugp_render calls: 0 off; 1 every kernel launch is
 * bracketed by HIP events on the context's stream and the durations summed;
 * 2 additionally counts BVH node visits and primitive tests (algorithmic
 * traffic).  [host] call, no device work. */
ugp_status ugp_set_profiling(ugp_ctx ctx, int level);

/* Path slots of later ugp_render calls: 0 (the default) keeps every path of
 * a chunk in flight (up to 2^25); a smaller pool (>= 64) bounds the render
 * buffers to about 230 B per slot and refills slots with new camera paths as
 * paths end, at some cost in throughput.  Results do not depend on it.
 * Buffers already allocated are kept.  [host] call, no device work. */
ugp_status ugp_set_path_pool(ugp_ctx ctx, int64_t slots);

/* Live paths at or below which ugp_render runs the remaining bounces of a
 * chunk (once no path is left to generate, from the second bounce on) in one
 * kernel, one lane following its path to the end, instead of one wavefront
 * launch per bounce; 0 disables it.  Default 65536.  Results do not depend on
 * it.  [host] call, no device work. */
ugp_status ugp_set_tail_paths(ugp_ctx ctx, int64_t paths);

/* Statistics of the last ugp_render call (synchronises the stream). */
ugp_status ugp_get_render_stats(ugp_ctx ctx, ugp_render_stats *out);

const char *ugp_status_string(ugp_status s);

/* ------------------------------------------------------------------------
 * Neural radiance cache: a network that predicts the radiance scattered from a
 * path vertex toward the previous vertex, so that paths can end early
 * (ugp_render_params.nrc_mode).  Not part of the paper's method: it follows
 * the rendering workload of the cache configuration (a fully fused MLP
 * 96 -> 64 -> 64 -> 64 -> 64 -> 3, ReLU, no biases).
 *
 * Inputs per query: float32 [16] = position[3], outgoing direction[3] (unit),
 * facet normal[3], roughness, albedo[3], 3 unused.  Encoding (96 features):
 * for each axis the position normalised to the box, x_hat = (x - lo) / (hi -
 * lo), as sin(2^j pi x_hat), cos(2^j pi x_hat) for j = 0..11 (72); the real
 * spherical harmonics of the direction, bands 0..3 (16); normal, roughness,
 * albedo (7); one zero.  Weights: float32 [ugp_nrc_num_params()] = 18624,
 * per layer [n_out][n_in], layers in order.  Arithmetic: bf16 weights and
 * activations on the matrix cores, float32 accumulation, float32 master
 * weights for Adam.  Loss: mean over records and channels of
 * (y - t)^2 / (y^2 + 0.01), the denominator held constant.
 * `box` is [host] lo[3], hi[3], or NULL for the scene bounds (then a scene
 * must have been built: UGP_ERR_NO_SCENE otherwise).
 * ------------------------------------------------------------------------ */
int32_t ugp_nrc_num_params(void);
/* Set the float32 master weights (device [P]) and reset the Adam moments and
 * step count, the radiance unit (the next training sets it) and the
 * training-path probability of nrc_mode 1 (the next such render starts it
 * afresh), so that renders from the same weights repeat exactly.  The first
 * call allocates the cache state. */
ugp_status ugp_nrc_set_weights(ugp_ctx ctx, const float *weights);
/* Copy the float32 master weights to weights_out (device [P]).
 * UGP_ERR_INVALID_ARGUMENT if the cache has no state yet. */
ugp_status ugp_nrc_get_weights(ugp_ctx ctx, float *weights_out);
/* Encoded features: inputs float [n][16] -> feat_out float [n][96]. */
ugp_status ugp_nrc_encode(ugp_ctx ctx, int64_t n, const float *inputs, const float *box,
                          float *feat_out);
/* Network prediction y_out float [n][3].  x_kind 0: x = inputs [n][16]
 * (encoded inside the kernel); 1: x = features [n][96].  Uses the bf16 copy
 * of the current weights. */
ugp_status ugp_nrc_forward(ugp_ctx ctx, int64_t n, const float *x, int32_t x_kind, const float *box,
                           float *y_out);
/* One optimisation step on n records: forward, loss, back-propagation,
 * weight gradient (per-slice partials summed in a fixed order), Adam (lr,
 * beta1 0.9, beta2 0.99, eps 1e-8, bias-corrected) on the master weights, new
 * bf16 copies.  targets float [n][3]; loss_out float [1] and grad_out float
 * [P] (device, or NULL) receive this step's loss and gradient.  1 <= n <= 1 << 22. */
ugp_status ugp_nrc_train_step(ugp_ctx ctx, int64_t n, const float *x, int32_t x_kind, const float *box,
                              const float *targets, float lr, float *loss_out, float *grad_out);
/* The training records of the last sample pass of the last ugp_render call
 * with nrc_mode 1: records_out float [cap][24] (inputs[16], throughput[3],
 * path index as int32 bits, radiance before the vertex's scattered light[3],
 * vertex index) and targets_out float [cap][3] (or NULL), in the order
 * they were trained on (by path, see nrc_mode 1); *count_out [host] =
 * records written (<= cap).  The path index is
 * pixel + pixels x (sample - first sample of its chunk), see ugp_render.
 * Synchronises. */
ugp_status ugp_nrc_records(ugp_ctx ctx, int64_t cap, float *records_out, float *targets_out,
                           int64_t *count_out);

#ifdef __cplusplus
}
#endif
#endif
