// ugp_internal.hpp -- library-private declarations shared by the HIP sources of
// libugp: the context, the device-side scene layout and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ugp.h"

namespace ugp {

// Device-side scene.  A primitive has one or more references (leaves of the
// hierarchy): long primitives are cut into slabs along their long axis, each
// slab a reference with its own box.
//   hot   [n_refs][4] float4, leaf (Morton) order: (mu.xyz, density),
//         (M00 M01 M02 M10), (M11 M12 M20 M21), (M22, orig id bits, 1/min(s),
//         slab bits) with M = S^-1 R^T rounded to float; slab bits = slab index
//         | slab count << 8 | long axis << 16
//   cold  [n][3] float4, original order: (facet normal.xyz, material),
//         (albedo.rgb, roughness), (emission.rgb, bounding-sphere radius)
//   nodes [n_nodes4][8] float4: 4-wide nodes holding the boxes of up to four
//         children as lo.x[4], lo.y[4], lo.z[4], hi.x[4], hi.y[4], hi.z[4],
//         ref[4], pad; a ref >= 0 is a node, < 0 is the leaf ~ref,
//         kEmptySlot marks an unused slot
//   inv   [n] original index -> leaf of its first slab
//   emit  [n_emit] original indices of emissive primitives, ascending
struct SceneDev {
    int64_t n = 0;
    int64_t n_refs = 0;    // leaves (references) of the hierarchy
    int32_t root = 0;      // ref of the root (a leaf ref when n == 1)
    float r2 = 0.f;        // squared Mahalanobis radius of the cut-off ellipsoid
    double r_cut = 0.0;    // that radius in full precision (for a refit)
    float4 *hot = nullptr;
    float4 *cold = nullptr;
    float4 *sggx = nullptr;  // [8 n] SGGX records (materials 2, 3) in original order; null without SGGX input
    bool has_mat3 = false;   // some primitive has material 3 (no albedo adjoint for it)
    float4 *nodes = nullptr;
    int32_t *inv = nullptr;
    int32_t *emit = nullptr;
    int32_t n_emit = 0;
    int32_t depth = 0;     // depth of the 4-wide hierarchy (root = 1)
    int64_t n_nodes4 = 0;
    unsigned long long *count = nullptr;  // [3] node visits, primitive tests, reloads (profiling)
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // bounds of the primitive boxes
};

// Device error word bits (deferred errors reported by ugp_sync): buffer
// overflows, and a caller's ray that failed validation (ray_ok)
enum : uint32_t { kErrStack = 1u, kErrEvents = 2u, kErrQueue = 4u, kErrRay = 8u };

// Sweep modes of the ordered traversal
enum SweepMode : int { kModeCollide = 0, kModeSaturate = 1, kModeEmitter = 2 };

constexpr int kStackSize = 32;   // traversal stack entries per lane in LDS
constexpr int kStackSpill = 160; // further entries per lane in private memory
constexpr int32_t kEmptySlot = 0x7fffffff;
constexpr int kEventsMain = 16;  // event buffer of the main sweep (registers)
constexpr int kEventsWide = 64;  // event buffer of the overflow sweep

struct RenderBuffers;
struct NrcState;

}  // namespace ugp

#include <vector>

struct ugp_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    ugp::SceneDev scene;
    uint32_t *err = nullptr;        // device error word
    // scratch for queries (grown on demand)
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    ugp::RenderBuffers *rb = nullptr;
    ugp::NrcState *nrc = nullptr;
    int64_t last_paths = 0;
    int64_t nrc_frac_pixels = 0;    // image size the training-path probability was set for
    int64_t last_nrc_counts = -1;   // offset of the cache counters of the last mode-1 render in the count buffer
    int64_t last_nrc_cap = 0;       // records cap of that render
    int64_t *stats = nullptr;       // device counters of the last render: [collision, light, env,
                                    //  cache queries, cache training records, -, -, -]
    unsigned long long *counters = nullptr;  // [3] traversal counters (profiling level 2)
    int profiling = 0;
    int64_t path_pool = 0;  // path slots of ugp_render (0: every path of a chunk)
    int64_t tail_paths = 65536;  // live paths at or below which a chunk's last bounces run in one kernel
    // event pairs of the last render, by category: 0 collide main, 1 collide wide, 2 light, 3 env,
    // 4 shade, 5 ray sort
    std::vector<int32_t> node_levels;  // 4-wide nodes of level L: [node_levels[L], node_levels[L + 1])
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> ev_used;  // (category, index of the start event)
    bool ev_cat_valid = false;
};

namespace ugp {

// build.hip
hipError_t build_scene(ugp_ctx ctx, const ugp_scene *s, float eps);
// new parameters for the same n primitives in the built hierarchy's topology
hipError_t refit_scene(ugp_ctx ctx, const ugp_scene *s);
// device-wide exclusive scan of int32, and a stable LSD radix sort of
// (uint32 key, int32 value) pairs (4 passes of 8 bits; result in keys / vals,
// tk / tv are scratch of the same size)
hipError_t exclusive_scan(const int *in, int *out, int64_t n, hipStream_t st);
hipError_t radix_sort(uint32_t *keys, int32_t *vals, uint32_t *tk, int32_t *tv, int64_t n, hipStream_t st);
void free_scene(SceneDev &sc);

// trace.hip
hipError_t launch_transmittance(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *excl,
                                float *T, float *F);
hipError_t launch_sweep(ugp_ctx ctx, int mode, int64_t n, const float *rays, const int32_t *excl,
                        const float *u, const int32_t *target, int32_t *prim_out, float *f_out,
                        int32_t *counts = nullptr, double *td_out = nullptr);

// allocation-free sweep: the working memory is a fixed per-GPU device array
// (at most kNoAllocMaxRays rays per call); noalloc_init takes its address once
// per device, with that device current
constexpr int64_t kNoAllocMaxRays = int64_t(1) << 22;
hipError_t noalloc_init(int device);
hipError_t launch_sweep_noalloc(ugp_ctx ctx, int mode, int64_t n, const float *rays, const int32_t *excl,
                                const float *u, const int32_t *target, int32_t *prim_out, float *f_out);

// test hooks: the ray integral of given primitives, Philox4x32-10 of given counters
hipError_t launch_ray_integral(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *prim, float *I);
hipError_t launch_philox(ugp_ctx ctx, int64_t n, const uint32_t *ctr, uint64_t key, uint32_t *out);

// exponential variant: T = exp(-sum I_k) (sample = false) or decomposition-tracking samples
hipError_t launch_exp(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *excl, bool sample, uint64_t seed,
                      float *T, int32_t *prim_out, float *t_out);

// render.hip
// Albedo adjoint of a render (path replay): d_image = dLoss/d(mean image)
// [h][w][3]; grad [n][3] += dLoss/dalbedo by original index.
struct RenderAdjoint {
    const float *d_image;
    float *grad_albedo = nullptr;     // [n][3], or null: not wanted
    float *grad_roughness = nullptr;  // [n], or null
    float *grad_density = nullptr;    // [n], or null
};
hipError_t render(ugp_ctx ctx, const ugp_camera *cam, const ugp_render_params *p, float *sum, float *sumsq,
                  const RenderAdjoint *adj = nullptr);
// SGGX phase-function test hook (queries laid out as in ugp_sggx_phase)
hipError_t sggx_phase(ugp_ctx ctx, int64_t n, const float *sggx, const float *base, const float *dirs,
                      const float *u, float *out);
struct CamDev;
// the device camera (origin, forward, right and up scaled to the field of view)
void make_cam_dev(const ugp_camera *cam, CamDev *out);
void free_render(ugp_ctx ctx);
// device float: loss of the last radiance-cache training step of a render (or NULL)
const float *render_nrc_loss(ugp_ctx ctx);
// copy the training records (and targets) of the last pass; synchronises
hipError_t render_nrc_records(ugp_ctx ctx, int64_t cap, float *rec_out, float *tgt_out, int64_t *count);

// nrc.hip -- the neural radiance cache.  Record layout shared with the
// renderer (kNrcRecordFloats floats per record): [0..15] network inputs
// (position, outgoing direction, normal, roughness, albedo, 3 unused),
// [16..18] throughput at the vertex, [19] path index bits (the path's slot in
// the wavefront; bit 30 free for the renderer's flags), [20..22] path radiance before the vertex's
// scattered light, [23] vertex index.
constexpr int kNrcRecordFloats = 24;
int nrc_num_params();
hipError_t nrc_ensure(ugp_ctx ctx);
void nrc_free(ugp_ctx ctx);
bool nrc_ready(ugp_ctx ctx);
hipError_t nrc_set_weights(ugp_ctx ctx, const float *w);
hipError_t nrc_get_weights(ugp_ctx ctx, float *w);
// box: [host] lo[3], hi[3] of the position normalisation, or NULL for the scene bounds
hipError_t nrc_encode(ugp_ctx ctx, int64_t n, const float *inputs, int stride, const float *box, float *feat);
// src_kind 0: raw inputs (stride floats per record) -> y; 1: features [n][96]
// -> y; 2: records (kNrcRecordFloats) -> L[pixel] += throughput * max(0, y)
hipError_t nrc_forward(ugp_ctx ctx, int64_t n, const int32_t *n_dev, const float *src, int stride, int src_kind,
                       const float *box, float *y, float4 *L, const float *scale = nullptr);
hipError_t nrc_train_step(ugp_ctx ctx, int64_t n, const int32_t *n_dev, const float *src, int stride, int src_kind,
                          const float *box, const float *targets, float lr, float *loss_out, float *grad_out);
hipError_t nrc_targets(ugp_ctx ctx, int64_t cap, const int32_t *n_dev, const float *rec, const float4 *L,
                       float *targets);
// the training of a render: radiance unit from the first batch (unless set),
// then `steps` Adam steps on consecutive batches of the records
hipError_t nrc_train_render(ugp_ctx ctx, int64_t cap, const int32_t *n_dev, const float *rec, const float *box,
                            const float *targets, float lr, int steps, float tclamp, float *loss_out);
// radiance unit of the network's output: value > 0 sets it, 0 keeps the current one
hipError_t nrc_set_scale(ugp_ctx ctx, float value);
const float *nrc_scale_ptr(ugp_ctx ctx);
hipError_t nrc_adapt(ugp_ctx ctx, const int32_t *attempted, int32_t cap, float *frac);

// diff.hip -- accumulated free-flight CDF, its loss and gradient; camera rays; Adam with clamps
// rgb: the radiance-field mode (outputs, targets [n][3]; gradient rows of 14 with the emission)
hipError_t accum_cdf(ugp_ctx ctx, const ugp_scene *scene, int64_t n, const float *rays, const int32_t *excl,
                     const float *target, float loss_scale, const float *dout, bool rgb, float *out, float *loss,
                     float *grad);
hipError_t camera_rays(ugp_ctx ctx, const ugp_camera *cam, uint64_t seed, uint32_t sample, float *rays);
// lr: mean, log scale, rotation, density, emission (emis may be NULL: rows of 11, else 14)
hipError_t fit_adam(ugp_ctx ctx, int64_t n, float *mean, float *scale, float *rot, float *dens, float *emis,
                    const float *grad, float *m, float *v, int t, const float lr[5], float b1, float b2, float eps,
                    float s_min);

// device scratch of the context: returns a buffer of at least `bytes`
void *ctx_scratch(ugp_ctx ctx, size_t bytes);

}  // namespace ugp
