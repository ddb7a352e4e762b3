// render.hip -- wavefront path tracer over Gaussian primitives (Sec. 5, table
// tab:highlevel right column, eq. rte) with next-event estimation to emissive
// primitives and to a constant environment, balance-heuristic MIS.
//
// Paths live in a pool of queue slots (about 2M).  The samples of a call are
// traced in chunks of several samples of every pixel; within a chunk each
// iteration first refills the free slots with new camera paths of the chunk
// (path g traces pixel g % pixels, sample chunk start + g / pixels), then:
//   collide : primitive-level free-flight sampling of every live path, each
//             at its own vertex; emission pick-up (MIS-weighted against the
//             light pdf of the previous vertex); light / environment samples
//             appended to their queues; phase sampling; surviving paths
//             compacted into the next queue (wave ballot + one atomic per wave)
//   light   : emitter query per light sample (emission rides on the
//             free-flight pdf, so emitter k contributes L_e,k I_k(a, min(b,
//             t_sat))/2 along the sampled direction)
//   env     : transmittance per environment sample
// until the chunk's paths are all done; the host reads two counters per
// iteration.  Each path's radiance has its own slot, so the final
// accumulation into sum / sum of squares runs pixel by pixel in sample order
// and the image does not depend on how paths were scheduled.
// Random numbers: Philox4x32-10 keyed by the seed, counter (pixel, sample,
// vertex, group): group 0 = (collision, emitter pick, -, -), group 1 =
// (phase u, phase v, environment u, environment v), group 7 = the light
// sample's point (three normals by Box-Muller); the camera jitter uses
// vertex 0, group 0, the choice of radiance-cache training paths vertex 0,
// group 2.  At SGGX vertices: groups 3 and 4 drive the stochastic phase
// evaluations of the light and environment samples (group 6 adds material
// 3's third normal to each), group 5 the base BSDF's sample after the
// visible normal.
//
// With the radiance cache, a path that is not a training path ends at
// collision nrc_terminate_after + 1: after its emission pick-up, its
// throughput times the cache's prediction at that vertex is added.  Training
// paths run to max_depth and record, at every scattering vertex, the cache
// inputs, the throughput and the radiance gathered so far; after the chunk the
// record's target is (path radiance - radiance so far) / throughput, and the
// optimisation steps are taken on the chunk's records, ordered by path (a
// fixed shuffle of the path slots) so that training, and with it every later
// image, is the same from run to run.
#include <algorithm>

#include "trace_device.hpp"

namespace ugp {

struct Queue {        // path (ray) queue, structure of arrays
    float4 *a;        // origin.xyz, pdf of the previous phase sample (0 = camera ray)
    float4 *b;        // direction.xyz, excluded primitive (original index bits)
    float4 *c;        // throughput.rgb, path index bits (bit 30: radiance-cache training path)
    int32_t *v;       // vertex index of the path's next collision (1 = camera ray)
};
struct LightQueue {   // light-sample queue
    float4 *a;        // origin.xyz, target primitive bits
    float4 *b;        // direction.xyz, excluded primitive bits
    float4 *c;        // weight.rgb, path index bits
};

struct RenderBuffers {
    int64_t cap = 0;         // path slots of the pool
    int64_t lcap = 0;        // paths of a chunk (radiance slots)
    Queue q[2];
    LightQueue nee, env;
    float4 *L = nullptr;     // radiance per path of the chunk
    int32_t *ovf = nullptr;  // overflow index list (cap entries)
    int2 *hits = nullptr;    // collision result per queue slot (prim, t bits)
    uint32_t *skey = nullptr, *skey2 = nullptr;  // ray-sort keys (and scratch)
    int32_t *sval = nullptr, *sval2 = nullptr;   // ray-sort permutation (and scratch)
    int32_t *counts = nullptr;  // iteration counters (two blocks) and chunk counters
    int32_t *host = nullptr;    // pinned: [paths left in the next queue, paths generated]
    float *qry = nullptr;       // radiance-cache queries (kNrcRecordFloats per path)
    void *block = nullptr;
    // radiance-cache training state (grown on demand): records are appended
    // to `staged` (kRecStage x rec_cap of them) in whatever order the waves
    // reach them, then ordered by path into `rec` (rec_cap)
    int64_t rec_cap = 0;
    float *staged = nullptr, *rec = nullptr, *targets = nullptr, *frac = nullptr, *loss = nullptr;
    uint32_t *rkey = nullptr, *rkey2 = nullptr;  // record-sort keys (and scratch), kRecStage x rec_cap
    int32_t *rval = nullptr, *rval2 = nullptr;   // record-sort permutation (and scratch)
    void *nrc_block = nullptr;
};

namespace {

constexpr int kPersistBlocks = 4096;
// training records staged per chunk, in multiples of the records a chunk
// trains on: the training set does not depend on the order of appends as long
// as a chunk attempts at most this many (the training-path probability is
// adapted toward one multiple and starts at an eighth of a path's worth)
constexpr int64_t kRecStage = 4;
constexpr int64_t kPoolPaths = int64_t(1) << 25;   // path slots of the pool
constexpr int64_t kChunkPaths = int64_t(1) << 25;  // paths of a chunk (radiance slots)
// iteration counters, two blocks used alternately (input / output queue):
// [0] paths in the queue, [1] light samples, [2] environment samples,
// [3] overflow, [4] collision work, [5] light work, [6] cache queries;
// then the chunk block: [0] paths generated, [1] training records appended
// Queue counters, each on a 256-B line of its own: the shading kernel appends
// to three of them once per wave, and atomics on one line serialise (with the
// eight counters of both blocks sharing a line, k_shade took 80% longer).
constexpr int kCtrSpread = 64;
__host__ __device__ constexpr int ctr(int k) { return k * kCtrSpread; }
constexpr int kCountStride = ctr(8);
constexpr int kChunkBlock = 2 * kCountStride;
constexpr int64_t kSortMin = 16384;  // queues shorter than this are traced unsorted

struct NrcArgs {
    int mode;              // 0 off, 1 infer + train, 2 infer, 3 terminate only
    int term;              // scattering events before a cached path ends
    float *rec;            // staged training records [rec_cap][kNrcRecordFloats]
    int32_t *n_rec;        // records appended (may exceed rec_cap: the excess is dropped)
    int32_t rec_cap;
    float *qry;            // cache queries [paths][kNrcRecordFloats]
    int32_t *n_qry;
    const float *frac;     // probability of a training path
};

// Albedo adjoint by path replay.  A chunk is traced twice with the same
// random numbers: the forward pass leaves each path's radiance in its slot,
// the replay subtracts every contribution as it is collected, so the slot
// holds the radiance still to come.  A path term is linear in the albedo of
// each vertex it scatters at (f is linear in it and no sampling decision
// depends on it), so at a vertex the albedo's adjoint is dLoss/dL times the
// radiance that passes through its scattering times (df/dalbedo)/f: the
// continuation's remainder is known when the next vertex is shaded, the
// light and environment samples' terms when they are collected.
struct AdjArgs {
    const float *dimg = nullptr;  // dLoss / d(mean image) [npix][3]; null: forward pass
    float *grad_alb = nullptr;    // [n_prims][3], original index, added to (null: not wanted)
    float *grad_rough = nullptr;  // [n_prims], channels summed
    float *grad_dens = nullptr;   // [n_prims]
    // per slot, for the albedo [0] and roughness [1] adjoints: (ratio, primitive
    // bits) of the vertex's continuation [.][0], light sample [.][1] and
    // environment sample [.][2]; null where that adjoint is not wanted
    float4 *aux[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    float inv_spp = 0.f;
    uint32_t npix = 1;
};

// the shading adjoint `which` (0 albedo, 1 roughness) of primitive k
__device__ __forceinline__ void adj_grad(const AdjArgs &A, int which, int slot, int k, float x, float y, float z) {
    const float *g = A.dimg + 3 * (int64_t)((uint32_t)slot % A.npix);
    const float gx = g[0] * A.inv_spp * x, gy = g[1] * A.inv_spp * y, gz = g[2] * A.inv_spp * z;
    if (which == 1) {
        const float t = gx + gy + gz;
        if (t != 0.f) atomicAdd(A.grad_rough + k, t);
        return;
    }
    float *dst = A.grad_alb + 3 * (int64_t)k;
    if (gx != 0.f) atomicAdd(dst, gx);
    if (gy != 0.f) atomicAdd(dst + 1, gy);
    if (gz != 0.f) atomicAdd(dst + 2, gz);
}

// the ratio (d f / d parameter) / f of adjoint `which` at a vertex
__device__ __forceinline__ V3 adj_ratio(int which, int mat, V3 alb, float rough, V3 wo, V3 wi) {
    if (which == 1) {
        const float r = phase_rough_ratio(mat, rough, wo, wi);
        return v3(r, r, r);
    }
    return phase_albedo_ratio(mat, alb, wo, wi);
}

// radiance c * f collected by the path of `slot`: added in the forward pass
// (one explicit fma per channel, the same in every kernel that collects, so
// that the per-path sums do not depend on which kernel traced the path); in
// the replay subtracted, and for a light (kind 1) or environment (kind 2)
// sample the shading adjoints added from the collecting vertex's ratios
__device__ __forceinline__ void collect(const AdjArgs &A, float4 *L, int slot, float cx, float cy, float cz,
                                        float f, int kind) {
    float4 l = L[slot];
    if (!A.dimg) {
        l.x = fmaf(cx, f, l.x); l.y = fmaf(cy, f, l.y); l.z = fmaf(cz, f, l.z);
        L[slot] = l;
        return;
    }
    l.x = fmaf(-cx, f, l.x); l.y = fmaf(-cy, f, l.y); l.z = fmaf(-cz, f, l.z);
    L[slot] = l;
    if (kind < 1) return;
    for (int w = 0; w < 2; ++w) {
        if (A.aux[w][kind]) {
            const float4 a = A.aux[w][kind][slot];
            adj_grad(A, w, slot, __float_as_int(a.w), a.x * (cx * f), a.y * (cy * f), a.z * (cz * f));
        }
    }
}

struct PassArgs {
    CamDev cam;
    float blo[3], binv[3];   // scene bounds (origin quantisation for ray sorting)
    uint64_t seed;
    uint32_t sample;         // sample index of the wavefront's first sample
    uint32_t npix;           // path q traces pixel q % npix, sample sample + q / npix
    int max_depth;
    int mis_mode;
    float env[3];
    int has_env;
    int transport;           // 0 linear transmittance, 1 the exponential variant
    NrcArgs nrc;
    AdjArgs adj;
};

constexpr int kPixMask = 0x3fffffff;
constexpr int kTrainBit = 0x40000000;

__device__ __forceinline__ V3 f3(float4 v) { return v3(v.x, v.y, v.z); }

// random numbers of path q (pixel, sample) at vertex v, group g
__device__ __forceinline__ Rng4 path_rng(const PassArgs &P, uint32_t q, uint32_t v, uint32_t g) {
    return rng4(P.seed, q % P.npix, P.sample + q / P.npix, v, g);
}

// Light sampling: an emissive primitive picked uniformly, then a point y of
// its untruncated Gaussian N(mu, Sigma) to aim at.  The direction's
// solid-angle pdf is the density of y integrated along the ray,
// int_0^inf N(x + t w) t^2 dt.  In the primitive's unit frame (x' = M (x -
// mu), w' = M w, a = |w'|) the ray passes the centre at distance rho, at
// signed position s = s0 + a t (s0 = x'.w' / a), so the integral is
//   |det M| exp(-rho^2/2) K(s0) / ((2 pi)^(3/2) a^3),
//   K(s0) = (1 + s0^2) sqrt(pi/2) erfc(s0/sqrt 2) - s0 exp(-s0^2/2),
// evaluated in double from the primitive's record, times the uniform choice.
// From a point inside the emitter's cut-off ellipsoid (|x'| <= r) no light
// sample is taken toward it (pdf 0): the directions that leave a flat
// emitter's plane would get a density far below their share of its emission,
// and phase sampling covers them.
__device__ bool inside_cut(const HotRec &h, double r2, V3 x) {
    const double c[3] = {(double)x.x - h.mx, (double)x.y - h.my, (double)x.z - h.mz};
    double q2 = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double xi = h.m[3 * i] * c[0] + h.m[3 * i + 1] * c[1] + h.m[3 * i + 2] * c[2];
        q2 += xi * xi;
    }
    return q2 <= r2;
}

__device__ double light_pdf(const HotRec &h, int n_emit, double r2, V3 x, V3 w) {
    const double c[3] = {(double)x.x - h.mx, (double)x.y - h.my, (double)x.z - h.mz};
    const double wd[3] = {w.x, w.y, w.z};
    double xp[3], wp[3];
    for (int i = 0; i < 3; ++i) {
        const double m0 = h.m[3 * i], m1 = h.m[3 * i + 1], m2 = h.m[3 * i + 2];
        xp[i] = m0 * c[0] + m1 * c[1] + m2 * c[2];
        wp[i] = m0 * wd[0] + m1 * wd[1] + m2 * wd[2];
    }
    if (xp[0] * xp[0] + xp[1] * xp[1] + xp[2] * xp[2] <= r2) return 0.0;
    const double a2 = wp[0] * wp[0] + wp[1] * wp[1] + wp[2] * wp[2];
    if (!(a2 > 0.0)) return 0.0;
    const double a = sqrt(a2);
    const double s0 = (xp[0] * wp[0] + xp[1] * wp[1] + xp[2] * wp[2]) / a;
    double rho2 = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double q = xp[i] - s0 * wp[i] / a;
        rho2 += q * q;
    }
    const double K = (1.0 + s0 * s0) * 1.2533141373155003 * erfc(s0 * 0.7071067811865476) - s0 * exp(-0.5 * s0 * s0);
    const double det = (double)h.m[0] * ((double)h.m[4] * h.m[8] - (double)h.m[5] * h.m[7]) -
                       (double)h.m[1] * ((double)h.m[3] * h.m[8] - (double)h.m[5] * h.m[6]) +
                       (double)h.m[2] * ((double)h.m[3] * h.m[7] - (double)h.m[4] * h.m[6]);
    return fabs(det) * exp(-0.5 * rho2) * fmax(K, 0.0) / (15.749609945653303 * a2 * a) / (double)n_emit;
}

// The light sample's direction from x toward primitive record h: y = mu + A n
// with A = M^-1 (= R S, by the adjugate in double) and n three standard
// normals from the uniforms u (Box-Muller); false when y coincides with x.
__device__ bool light_dir(const HotRec &h, V3 x, const Rng4 &u, V3 &w) {
    double m[9];
    for (int i = 0; i < 9; ++i) m[i] = h.m[i];
    const double det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                       m[2] * (m[3] * m[7] - m[4] * m[6]);
    if (!(fabs(det) > 0.0)) return false;
    const double id = 1.0 / det;
    const double A[9] = {(m[4] * m[8] - m[5] * m[7]) * id, (m[2] * m[7] - m[1] * m[8]) * id,
                         (m[1] * m[5] - m[2] * m[4]) * id, (m[5] * m[6] - m[3] * m[8]) * id,
                         (m[0] * m[8] - m[2] * m[6]) * id, (m[2] * m[3] - m[0] * m[5]) * id,
                         (m[3] * m[7] - m[4] * m[6]) * id, (m[1] * m[6] - m[0] * m[7]) * id,
                         (m[0] * m[4] - m[1] * m[3]) * id};
    const double r1 = sqrt(-2.0 * log(1.0 - (double)u.u[0])), r2 = sqrt(-2.0 * log(1.0 - (double)u.u[2]));
    double s1, c1, s3, c3;
    sincos(6.283185307179586 * (double)u.u[1], &s1, &c1);
    sincos(6.283185307179586 * (double)u.u[3], &s3, &c3);
    const double n[3] = {r1 * c1, r1 * s1, r2 * c3};
    double d[3];
    const double mu[3] = {h.mx, h.my, h.mz}, xs[3] = {x.x, x.y, x.z};
    for (int i = 0; i < 3; ++i) d[i] = mu[i] + A[3 * i] * n[0] + A[3 * i + 1] * n[1] + A[3 * i + 2] * n[2] - xs[i];
    const double l2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(l2 > 0.0)) return false;
    const double il = 1.0 / sqrt(l2);
    w = v3((float)(d[0] * il), (float)(d[1] * il), (float)(d[2] * il));
    return true;
}

// Refill the free slots of the input queue with new camera paths of the
// chunk: n_new = min(free slots, paths not yet generated); path g = generated
// + j goes to slot n_in + j, its radiance slot is cleared.  k_regen_commit
// then advances both counters and clears this iteration's other counters.
__global__ void k_regen(PassArgs P, int64_t pool, int64_t total, const int32_t *cnt_in, const int32_t *chunk,
                        Queue q, float4 *L) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_in = cnt_in[0], gen = chunk[0];
    const int64_t n_new = pool - n_in < total - gen ? pool - n_in : total - gen;
    if (j >= n_new) return;
    const int64_t g = gen + j, slot = n_in + j;
    const Rng4 r = path_rng(P, (uint32_t)g, 0, 0);
    const int pix = (int)((uint32_t)g % P.npix);
    const int px = pix % P.cam.width, py = pix / P.cam.width;
    const V3 d = camera_dir(P.cam, px, py, r.u[0], r.u[1]);
    int bits = (int)g;
    if (P.nrc.mode == 1 && path_rng(P, (uint32_t)g, 0, 2).u[0] < *P.nrc.frac) bits |= kTrainBit;
    q.a[slot] = make_float4(P.cam.ox, P.cam.oy, P.cam.oz, 0.f);
    q.b[slot] = make_float4(d.x, d.y, d.z, __int_as_float(-1));
    q.c[slot] = make_float4(1.f, 1.f, 1.f, __int_as_float(bits));
    q.v[slot] = 1;
    if (!P.adj.dimg) L[g] = make_float4(0.f, 0.f, 0.f, 0.f);  // the replay keeps the forward radiance
}

__global__ void k_regen_commit(int64_t pool, int64_t total, int32_t *cnt_in, int32_t *cnt_out, int32_t *chunk) {
    const int64_t n_in = cnt_in[0], gen = chunk[0];
    const int64_t n_new = pool - n_in < total - gen ? pool - n_in : total - gen;
    cnt_in[0] = (int32_t)(n_in + n_new);
    chunk[0] = (int32_t)(gen + n_new);
    for (int k = 1; k < 8; ++k) cnt_in[ctr(k)] = 0;
    for (int k = 0; k < 8; ++k) cnt_out[ctr(k)] = 0;
}

__device__ __forceinline__ int wave_append(bool want, int32_t *counter) {
    const uint64_t m = __ballot(want);
    if (m == 0ull) return 0;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    return base + __popcll(m & below);
}

// Paths whose collision overflows the register event buffer are listed in
// `ovf` and redone by the wide instantiation (WIDE = true), which walks that
// list instead of the queue.
struct Overflow {
    int32_t *idx;
    int32_t *count;
};

// Sort key of a queued ray: 6 bits each of its origin (in the scene bounds)
// and of its direction (octahedral map) interleaved into 30 bits, so that a
// wave's rays start near each other and point the same way.  Slots past the
// queue length get the largest key.
__device__ __forceinline__ uint32_t spread5(uint32_t v, int k) {
    uint32_t r = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) r |= ((v >> b) & 1u) << (5 * b + k);
    return r;
}

__global__ void k_sort_keys(PassArgs P, Queue q, const int32_t *n_in, int64_t cap, uint32_t *keys,
                            int32_t *vals) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cap) return;
    vals[j] = (int32_t)j;
    if (j >= *n_in) {
        keys[j] = 0xffffffffu;
        return;
    }
    const float4 A = q.a[j], B = q.b[j];
    uint32_t c[5];
    const float o[3] = {A.x, A.y, A.z};
    for (int k = 0; k < 3; ++k)
        c[k] = (uint32_t)fminf(fmaxf((o[k] - P.blo[k]) * P.binv[k] * 64.f, 0.f), 63.f);
    // octahedral map of the direction to [0,1]^2
    const float l1 = fabsf(B.x) + fabsf(B.y) + fabsf(B.z);
    float u = B.x / l1, v = B.y / l1;
    if (B.z < 0.f) {
        const float uu = (1.f - fabsf(v)) * (u >= 0.f ? 1.f : -1.f);
        const float vv = (1.f - fabsf(u)) * (v >= 0.f ? 1.f : -1.f);
        u = uu;
        v = vv;
    }
    c[3] = (uint32_t)fminf(fmaxf((u * 0.5f + 0.5f) * 64.f, 0.f), 63.f);
    c[4] = (uint32_t)fminf(fmaxf((v * 0.5f + 0.5f) * 64.f, 0.f), 63.f);
    uint32_t key = 0;
    for (int k = 0; k < 5; ++k) key |= spread5(c[k], 4 - k);
    keys[j] = key;
}

// Collision sweep of every live path; the result (selected primitive, scatter
// distance) goes to hits[i].  Paths that overflow the register event buffer
// are listed in `ovf` and redone by the wide instantiation (WIDE = true).
template <int K, bool WIDE>
__global__ __launch_bounds__(kBlock, 2) void k_collide(SceneDev S, PassArgs P, Queue qin,
                                                    const int32_t *n_in, const int32_t *order, int32_t *work,
                                                    int2 *hits, int64_t *stats, Overflow ovf, uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int n = WIDE ? *ovf.count : *n_in;
    if (!WIDE && blockIdx.x == 0 && threadIdx.x == 0)
        atomicAdd((unsigned long long *)&stats[0], (unsigned long long)n);
    TraceCount tc;
    auto process = [&](int64_t i) __attribute__((always_inline)) {
        const float4 A = qin.a[i], B = qin.b[i], C = qin.c[i];
        const int pix = __float_as_int(C.w) & kPixMask;
        const int excl = __float_as_int(B.w);
        const int v = qin.v[i];
        const float u = path_rng(P, (uint32_t)pix, (uint32_t)v, 0).u[0];
        const RayD r = make_ray(A.x, A.y, A.z, B.x, B.y, B.z, 0.f, __builtin_huge_val());
        const SweepOut so = sweep<K>(S, r, excl, kModeCollide, u, -1, stack, err, tc);
        if (so.status != 0) {
            if (WIDE) {
                atomicOr(err, kErrEvents);
                hits[i] = make_int2(-1, __float_as_int(0.f));
            } else {
                const int slot = atomicAdd(ovf.count, 1);
                ovf.idx[slot] = (int32_t)i;
            }
            return;
        }
        hits[i] = make_int2(so.prim, __float_as_int(so.t));
    };
    if (WIDE) {
        for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock)
            process((int64_t)ovf.idx[j]);
    } else {
        // one sweep round (or part of one) per iteration; a lane whose ray is
        // done takes the next ray of the sorted queue at once, and traversals
        // are suspended while many lanes wait, so lanes do not wait for the
        // slowest ray of their wave
        int64_t i = -1;
        bool exhausted = false;
        RayD r = make_ray(0.f, 0.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.0);
        float u = 0.f;
        int excl = -1;
        SweepState<K> st;
        SweepOut so;
        int spill[kStackSpill];
        for (;;) {
            const int64_t j = lane_refill(i < 0 && !exhausted, work);
            if (j >= 0) {
                if (j < n) {
                    i = order ? (int64_t)order[j] : j;
                    const float4 A = qin.a[i], B = qin.b[i], C = qin.c[i];
                    const int pix = __float_as_int(C.w) & kPixMask;
                    excl = __float_as_int(B.w);
                    u = path_rng(P, (uint32_t)pix, (uint32_t)qin.v[i], 0).u[0];
                    r = make_ray(A.x, A.y, A.z, B.x, B.y, B.z, 0.f, __builtin_huge_val());
                    sweep_start(st, so, r, kModeCollide);
                } else {
                    exhausted = true;
                }
            }
            if (!__any(i >= 0)) break;
            const int susp = __any(exhausted) ? 0 : kSuspendAt;
            if (i >= 0 &&
                sweep_round<K>(S, r, excl, kModeCollide, u, -1, -kInf, st, so, stack, spill, susp, err, tc)) {
                if (so.status != 0) {
                    const int slot = atomicAdd(ovf.count, 1);
                    ovf.idx[slot] = (int32_t)i;
                } else {
                    hits[i] = make_int2(so.prim, __float_as_int(so.t));
                }
                i = -1;
            }
        }
    }
    flush_counts(S, tc);
}

// What the shading of one path vertex produces (the wavefront kernel appends
// it to the queues; the tail kernel consumes it at once).
struct ShadeOut {
    bool cont = false, do_nee = false, do_env = false, do_qry = false, do_rec = false;
    float4 ca{}, cb{}, cc{};                  // next collision ray (origin + pdf, direction + excluded, beta + bits)
    float4 na{}, nb{}, nc{};                  // light sample (origin + target, direction + excluded, weight + pixel)
    float4 ea{}, eb{}, ec{};                  // environment sample
    float4 r0{}, r1{}, r2{}, r3{}, r4{}, r5{};  // cache query / training record
};

// Phase function of primitive k at a path vertex for the direction wl
// (world frame): f (rgb) and the pdf of phase sampling used by MIS.  The
// SGGX microflakes (material 2) take the stochastic estimate from the four
// uniforms of gs and the approximate pdf; the delta-NDF materials are exact.
__device__ __forceinline__ V3 vertex_phase(int mat, const Sggx &sg, const Sggx &sgr, const Facet &F, V3 wo, V3 wol,
                                           V3 alb, float rough, V3 wl, const float u[6], float &pdf) {
    if (mat == 3) {
        pdf = sggx_disney_pdf_approx(sgr, sg.ps, wo, wl);
        return sggx_disney_est(sg, alb, rough, wo, wl, u);
    }
    if (mat == 2) {
        pdf = sggx_pdf_approx(wo, wl);
        return sggx_phase_est(sg, wo, wl, u[0], u[1], u[2], u[3]) * alb;
    }
    return phase_eval_local(mat, alb, rough, wol, to_local(F, wl), pdf);
}

// uniforms of an SGGX evaluation at vertex v: group g (four), and for
// material 3 two more from group 6 (its first pair for the light sample,
// g = 3, its second for the environment sample)
__device__ __forceinline__ void eval_uniforms(const PassArgs &P, uint32_t q, uint32_t v, uint32_t g, int mat,
                                              float u[6]) {
    u[4] = u[5] = 0.f;
    if (mat < 2) {
        u[0] = u[1] = u[2] = u[3] = 0.f;
        return;
    }
    const Rng4 a = path_rng(P, q, v, g);
    u[0] = a.u[0]; u[1] = a.u[1]; u[2] = a.u[2]; u[3] = a.u[3];
    if (mat == 3) {
        const Rng4 b = path_rng(P, q, v, 6);
        u[4] = g == 3 ? b.u[0] : b.u[2];
        u[5] = g == 3 ? b.u[1] : b.u[3];
    }
}

// Shading of one path vertex after its collision `hit` (prim, t bits):
// emission pick-up (MIS against the light pdf of the previous vertex),
// environment on escape, one light sample and one environment sample, phase
// sampling; the picked-up radiance is added to the path's slot L[pixel].
__device__ __forceinline__ void shade_one(const SceneDev &S, const PassArgs &P, const float4 A, const float4 B,
                                          const float4 C, const int v, const int2 hit, float4 *L, ShadeOut &out) {
    const int pbits = __float_as_int(C.w);
    const int pix = pbits & kPixMask;
    const bool train = (pbits & kTrainBit) != 0;
    const float p_prev = A.w;
    const V3 o = f3(A), d = f3(B);
    V3 beta = f3(C);
    const Rng4 g0 = path_rng(P, (uint32_t)pix, (uint32_t)v, 0);
    const Rng4 g1 = path_rng(P, (uint32_t)pix, (uint32_t)v, 1);
    if (P.adj.dimg && v >= 2) {
        // replay: what is left to collect went through the previous vertex's continuation
        const float4 R = L[pix];
        for (int w = 0; w < 2; ++w) {
            if (P.adj.aux[w][0]) {
                const float4 a = P.adj.aux[w][0][pix];
                adj_grad(P.adj, w, pix, __float_as_int(a.w), a.x * R.x, a.y * R.y, a.z * R.z);
            }
        }
    }
    V3 Lc = v3(0.f, 0.f, 0.f);  // radiance picked up here: Lw * Lc
    float Lw = 0.f;
    if (hit.x < 0) {
        if (P.has_env) {
            float w = 1.f;
            if (v > 1) {
                if (P.mis_mode == 2) w = 0.f;
                else if (P.mis_mode == 0) w = p_prev / (p_prev + 0.25f * kInvPi);
            }
            Lc = mul(beta, v3(P.env[0], P.env[1], P.env[2]));
            Lw = w;
        }
    } else {
        const int k = hit.x;
        const float4 c0 = S.cold[3 * k], c1 = S.cold[3 * k + 1], c2 = S.cold[3 * k + 2];
        const V3 x = o + __int_as_float(hit.y) * d;
        const V3 Le = f3(c2);
        if (nonzero(Le)) {
            float w = 1.f;
            if (v > 1) {
                const float pn = (float)light_pdf(load_hot(S.hot, S.inv[k]), S.n_emit, S.r_cut * S.r_cut, o, d);
                if (P.mis_mode == 2) w = pn > 0.f ? 0.f : 1.f;
                else if (P.mis_mode == 0) w = p_prev / (p_prev + pn);
            }
            Lc = mul(beta, Le);
            Lw = w;
        }
        bool stop = false;
        if (v <= P.max_depth && P.nrc.mode != 0) {
            // radiance cache: inputs of this vertex (position, outgoing
            // direction, facet normal turned toward it, roughness, albedo)
            const V3 wo = -d;
            const V3 nf = dot(f3(c0), wo) >= 0.f ? f3(c0) : -f3(c0);
            out.r0 = make_float4(x.x, x.y, x.z, wo.x);
            out.r1 = make_float4(wo.y, wo.z, nf.x, nf.y);
            out.r2 = make_float4(nf.z, c1.w, c1.x, c1.y);
            out.r3 = make_float4(c1.z, 0.f, 0.f, 0.f);
            out.r4 = make_float4(beta.x, beta.y, beta.z, __int_as_float(pix));
            if (!train && v == P.nrc.term + 1) {
                stop = true;
                out.do_qry = P.nrc.mode != 3;
            } else if (train) {
                const float4 l = L[pix];
                out.r5 = make_float4(fmaf(Lc.x, Lw, l.x), fmaf(Lc.y, Lw, l.y), fmaf(Lc.z, Lw, l.z), (float)v);
                out.do_rec = true;
            }
        }
        if (v <= P.max_depth && !stop) {
            const V3 wo = -d;
            const Facet F = facet(f3(c0), wo);
            const V3 wol = to_local(F, wo);
            const int mat = __float_as_int(c0.w);
            const V3 alb = f3(c1);
            const float rough = c1.w;
            // SGGX microflakes: their record, and the uniforms of the light and
            // environment estimates (groups 3, 4) and of the cosine sample about
            // the visible normal (group 5)
            Sggx sg{}, sgr{};
            if (mat >= 2) sg = sggx_load(S.sggx + 8 * (int64_t)k);
            if (mat == 3) sgr = sggx_load(S.sggx + 8 * (int64_t)k + 4);
            // light sample: one emitter picked uniformly, aimed at a point of its
            // Gaussian (uniforms of group 7)
            if (S.n_emit > 0 && P.mis_mode != 1) {
                // floor(u * n_emit) in exact integer arithmetic (u has 24 bits)
                int j = (int)(((uint64_t)(g0.u[1] * 16777216.f) * (uint64_t)S.n_emit) >> 24);
                j = min(j, S.n_emit - 1);
                const int e = S.emit[j];
                const HotRec eh = load_hot(S.hot, S.inv[e]);
                V3 wl;
                const double r2 = S.r_cut * S.r_cut;
                if (e != k && !inside_cut(eh, r2, x) && light_dir(eh, x, path_rng(P, (uint32_t)pix, (uint32_t)v, 7), wl)) {
                    float pph;
                    float ue[6];
                    eval_uniforms(P, (uint32_t)pix, (uint32_t)v, 3, mat, ue);
                    const V3 f = vertex_phase(mat, sg, sgr, F, wo, wol, alb, rough, wl, ue, pph);
                    Chord tc;
                    const RayD lr = make_ray(x.x, x.y, x.z, wl.x, wl.y, wl.z, 0.f, __builtin_huge_val());
                    const float pn =
                        nonzero(f) && chord(eh, lr, S.r2, tc) ? (float)light_pdf(eh, S.n_emit, r2, x, wl) : 0.f;
                    if (pn > 0.f) {
                        const float w = P.mis_mode == 2 ? 1.f : pn / (pn + pph);
                        const float4 eL = S.cold[3 * e + 2];
                        const V3 wt = (w / pn) * mul(mul(beta, f), f3(eL));
                        out.do_nee = true;
                        for (int aw = 0; aw < 2; ++aw) {
                            if (P.adj.aux[aw][1]) {
                                const V3 q = adj_ratio(aw, mat, alb, rough, wol, to_local(F, wl));
                                P.adj.aux[aw][1][pix] = make_float4(q.x, q.y, q.z, __int_as_float(k));
                            }
                        }
                        out.na = make_float4(x.x, x.y, x.z, __int_as_float(e));
                        // the linear model skips k on the light ray; the exponential
                        // variant skips nothing and keys the ray's draws by the vertex
                        out.nb = make_float4(wl.x, wl.y, wl.z, __int_as_float(P.transport ? v : k));
                        out.nc = make_float4(wt.x, wt.y, wt.z, __int_as_float(pix));
                    }
                }
            }
            // environment sample: uniform direction
            if (P.has_env && P.mis_mode != 1) {
                const float z = 1.f - 2.f * g1.u[2];
                const float rr = sqrtf(fmaxf(0.f, 1.f - z * z));
                float sp, cp;
                sincosf(2.f * kPi * g1.u[3], &sp, &cp);
                const V3 wl = v3(rr * cp, rr * sp, z);
                float pph;
                float ue[6];
                eval_uniforms(P, (uint32_t)pix, (uint32_t)v, 4, mat, ue);
                const V3 f = vertex_phase(mat, sg, sgr, F, wo, wol, alb, rough, wl, ue, pph);
                if (nonzero(f)) {
                    const float pe = 0.25f * kInvPi;
                    const float w = P.mis_mode == 2 ? 1.f : pe / (pe + pph);
                    const V3 wt = (w / pe) * mul(mul(beta, f), v3(P.env[0], P.env[1], P.env[2]));
                    out.do_env = true;
                    for (int aw = 0; aw < 2; ++aw) {
                        if (P.adj.aux[aw][2]) {
                            const V3 q = adj_ratio(aw, mat, alb, rough, wol, to_local(F, wl));
                            P.adj.aux[aw][2][pix] = make_float4(q.x, q.y, q.z, __int_as_float(k));
                        }
                    }
                    out.ea = make_float4(x.x, x.y, x.z, 0.f);
                    out.eb = make_float4(wl.x, wl.y, wl.z, __int_as_float(P.transport ? -1 : k));
                    out.ec = make_float4(wt.x, wt.y, wt.z, __int_as_float(pix));
                }
            }
            // continue by phase sampling from the collision point, skipping k in
            // the linear model (an exponential medium scatters inside the
            // Gaussian, whose rest still attenuates)
            V3 wgt, wil, wi;
            float pdf;
            if (mat == 2) {
                const Rng4 g5 = path_rng(P, (uint32_t)pix, (uint32_t)v, 5);
                wi = sggx_sample(sg, wo, g1.u[0], g1.u[1], g5.u[0], g5.u[1]);
                wil = wol;  // (the albedo ratio of material 2 does not depend on directions)
                wgt = alb;
                pdf = sggx_pdf_approx(wo, wi);
            } else if (mat == 3) {  // (no albedo adjoint for material 3: the entry point refuses it)
                const Rng4 g5 = path_rng(P, (uint32_t)pix, (uint32_t)v, 5);
                wil = wol;
                pdf = sggx_disney_sample(sg, alb, rough, wo, g1.u[0], g1.u[1], g5.u[0], g5.u[1], g5.u[2], wi, wgt)
                          ? sggx_disney_pdf_approx(sgr, sg.ps, wo, wi)
                          : 0.f;
            } else {
                wil = phase_sample_local(mat, alb, rough, wol, g1.u[0], g1.u[1], wgt, pdf);
                wi = to_world(F, wil);
            }
            if (pdf > 0.f) {
                beta = mul(beta, wgt);
                if (nonzero(beta)) {
                    out.cont = true;
                    for (int aw = 0; aw < 2; ++aw) {
                        if (P.adj.aux[aw][0]) {
                            const V3 q = adj_ratio(aw, mat, alb, rough, wol, wil);
                            P.adj.aux[aw][0][pix] = make_float4(q.x, q.y, q.z, __int_as_float(k));
                        }
                    }
                    out.ca = make_float4(x.x, x.y, x.z, pdf);
                    out.cb = make_float4(wi.x, wi.y, wi.z, __int_as_float(P.transport ? -1 : k));
                    out.cc = make_float4(beta.x, beta.y, beta.z, __int_as_float(pbits));
                }
            }
        }
    }
    if (Lw != 0.f && (Lc.x != 0.f || Lc.y != 0.f || Lc.z != 0.f)) collect(P.adj, L, pix, Lc.x, Lc.y, Lc.z, Lw, 0);
}

// Shading of every live path after its collision: emission pick-up (MIS
// against the light pdf of the previous vertex), environment on escape, one
// light sample and one environment sample appended to their queues, phase
// sampling, and compaction of the surviving paths into the next queue.
__global__ __launch_bounds__(kBlock) void k_shade(SceneDev S, PassArgs P, Queue qin, const int32_t *n_in,
                                                  const int2 *hits, Queue qout, int32_t *n_out, LightQueue nee,
                                                  int32_t *n_nee, LightQueue env, int32_t *n_env, float4 *L) {
    const int n = *n_in;
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += (int64_t)gridDim.x * kBlock) {
        const int64_t i = base + threadIdx.x;
        ShadeOut o;
        int v = 0;
        if (i < n) {
            v = qin.v[i];
            shade_one(S, P, qin.a[i], qin.b[i], qin.c[i], v, hits[i], L, o);
        }
        const int pc = wave_append(o.cont, n_out);
        if (o.cont) { qout.a[pc] = o.ca; qout.b[pc] = o.cb; qout.c[pc] = o.cc; qout.v[pc] = v + 1; }
        const int pn = wave_append(o.do_nee, n_nee);
        if (o.do_nee) { nee.a[pn] = o.na; nee.b[pn] = o.nb; nee.c[pn] = o.nc; }
        const int pe = wave_append(o.do_env, n_env);
        if (o.do_env) { env.a[pe] = o.ea; env.b[pe] = o.eb; env.c[pe] = o.ec; }
        if (P.nrc.mode != 0) {
            const int pq = wave_append(o.do_qry, P.nrc.n_qry);
            if (o.do_qry) {
                float4 *q = reinterpret_cast<float4 *>(P.nrc.qry + (int64_t)kNrcRecordFloats * pq);
                q[0] = o.r0; q[1] = o.r1; q[2] = o.r2; q[3] = o.r3; q[4] = o.r4;
            }
            const int pr = wave_append(o.do_rec, P.nrc.n_rec);
            if (o.do_rec && pr < P.nrc.rec_cap) {
                float4 *q = reinterpret_cast<float4 *>(P.nrc.rec + (int64_t)kNrcRecordFloats * pr);
                q[0] = o.r0; q[1] = o.r1; q[2] = o.r2; q[3] = o.r3; q[4] = o.r4; q[5] = o.r5;
            }
        }
    }
}

template <int K, bool WIDE>
__global__ __launch_bounds__(kBlock, 2) void k_light(SceneDev S, LightQueue q, const int32_t *n_in,
                                                  const int32_t *order, int32_t *work, float4 *L, int64_t *stats,
                                                  Overflow ovf, AdjArgs adj, uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int n = WIDE ? *ovf.count : *n_in;
    if (!WIDE && blockIdx.x == 0 && threadIdx.x == 0)
        atomicAdd((unsigned long long *)&stats[1], (unsigned long long)n);
    TraceCount tc;
    auto process = [&](int64_t i) __attribute__((always_inline)) {
        const float4 A = q.a[i], B = q.b[i], C = q.c[i];
        const int target = __float_as_int(A.w), excl = __float_as_int(B.w), pix = __float_as_int(C.w);
        RayD r = make_ray(A.x, A.y, A.z, B.x, B.y, B.z, 0.f, __builtin_huge_val());
        const HotRec h = load_hot(S.hot, S.inv[target]);
        Chord c;
        if (!chord(h, r, S.r2, c)) return;
        r.t1 = c.bd;
        const SweepOut so = sweep<K>(S, r, excl, kModeEmitter, 0.f, target, stack, err, tc, c.a);
        if (so.status != 0) {
            if (WIDE) {
                atomicOr(err, kErrEvents);
            } else {
                const int slot = atomicAdd(ovf.count, 1);
                ovf.idx[slot] = (int32_t)i;
            }
            return;
        }
        if (so.t > 0.f) collect(adj, L, pix, C.x, C.y, C.z, so.t, 1);
    };
    if (WIDE) {
        for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock)
            process((int64_t)ovf.idx[j]);
    } else {
        // one sweep round per iteration, lanes refilled as their rays finish
        int64_t i = -1;
        bool exhausted = false;
        RayD r = make_ray(0.f, 0.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.0);
        int excl = -1, target = -1;
        float entry = 0.f;
        SweepState<K> st;
        SweepOut so;
        int spill[kStackSpill];
        for (;;) {
            const int64_t j = lane_refill(i < 0 && !exhausted, work);
            if (j >= 0) {
                if (j < n) {
                    const int64_t k = order ? (int64_t)order[j] : j;
                    const float4 A = q.a[k], B = q.b[k];
                    target = __float_as_int(A.w);
                    excl = __float_as_int(B.w);
                    r = make_ray(A.x, A.y, A.z, B.x, B.y, B.z, 0.f, __builtin_huge_val());
                    Chord c;
                    if (chord(load_hot(S.hot, S.inv[target]), r, S.r2, c)) {
                        r.t1 = c.bd;
                        entry = c.a;
                        i = k;
                        sweep_start(st, so, r, kModeEmitter);
                    }
                } else {
                    exhausted = true;
                }
            }
            if (!__any(i >= 0 || (j >= 0 && j < n))) break;
            const int susp = __any(exhausted) ? 0 : kSuspendAt;
            if (i >= 0 && sweep_round<K>(S, r, excl, kModeEmitter, 0.f, target, entry, st, so, stack, spill, susp,
                                         err, tc)) {
                if (so.status != 0) {
                    const int slot = atomicAdd(ovf.count, 1);
                    ovf.idx[slot] = (int32_t)i;
                } else if (so.t > 0.f) {
                    const float4 C = q.c[i];
                    collect(adj, L, __float_as_int(C.w), C.x, C.y, C.z, so.t, 1);
                }
                i = -1;
            }
        }
    }
    flush_counts(S, tc);
}

__global__ __launch_bounds__(kBlock) void k_env(SceneDev S, LightQueue q, const int32_t *n_in, float4 *L,
                                                int64_t *stats, AdjArgs adj, uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int n = *n_in;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd((unsigned long long *)&stats[2], (unsigned long long)n);
    TraceCount tc;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const float4 A = q.a[i], B = q.b[i], C = q.c[i];
        const int excl = __float_as_int(B.w), pix = __float_as_int(C.w);
        const RayD r = make_ray(A.x, A.y, A.z, B.x, B.y, B.z, 0.f, __builtin_huge_val());
        const float F = transmittance_F(S, r, excl, true, stack, err, tc);
        const float T = fmaxf(0.f, 1.f - F);
        if (T > 0.f) collect(adj, L, pix, C.x, C.y, C.z, T, 2);
    }
    flush_counts(S, tc);
}

// ---------------------------------------------------------------------------
// The exponential variant (App. D) as a render mode, for the paper's comparison
// of transmittance models: a path's next collision and its light samples are
// drawn by analog decomposition tracking (exp_track), with the uniform of
// Gaussian k at vertex v from the path's generator, group 16 + 2k (collision)
// or 17 + 2k (light sample); environment samples take T = exp(-depth).  One
// ray per lane (no windowed sweep is needed).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_collide_exp(SceneDev S, PassArgs P, Queue qin, const int32_t *n_in,
                                                        const int32_t *order, int2 *hits, int64_t *stats,
                                                        uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int n = *n_in;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd((unsigned long long *)&stats[0], (unsigned long long)n);
    TraceCount tc;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        const int64_t i = order ? (int64_t)order[j] : j;
        const float4 A = qin.a[i], B = qin.b[i], C = qin.c[i];
        const uint32_t pix = (uint32_t)(__float_as_int(C.w) & kPixMask), v = (uint32_t)qin.v[i];
        const RayD r = make_ray(A.x, A.y, A.z, B.x, B.y, B.z, 0.f, __builtin_huge_val());
        double t;
        const int k = exp_track(
            S, r, __float_as_int(B.w),
            [&](int q) __attribute__((always_inline)) {
                return (double)path_rng(P, pix, v, 16u + 2u * (uint32_t)q).u[0];
            },
            stack, err, tc, t);
        hits[i] = make_int2(k, __float_as_int(k >= 0 ? (float)t : 0.f));
    }
    flush_counts(S, tc);
}

// light samples: one decomposition-tracking draw along the segment to the
// target's chord exit scores the sample if the target is hit first (an
// unbiased estimate of the probability that it is)
__global__ __launch_bounds__(kBlock) void k_light_exp(SceneDev S, PassArgs P, LightQueue q, const int32_t *n_in,
                                                      const int32_t *order, float4 *L, int64_t *stats,
                                                      uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int n = *n_in;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd((unsigned long long *)&stats[1], (unsigned long long)n);
    TraceCount tc;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        const int64_t i = order ? (int64_t)order[j] : j;
        const float4 A = q.a[i], B = q.b[i];
        const int target = __float_as_int(A.w);
        RayD r = make_ray(A.x, A.y, A.z, B.x, B.y, B.z, 0.f, __builtin_huge_val());
        Chord c;
        if (!chord(load_hot(S.hot, S.inv[target]), r, S.r2, c)) continue;
        r.t1 = c.bd;
        const float4 C = q.c[i];
        const uint32_t pix = (uint32_t)__float_as_int(C.w), v = (uint32_t)__float_as_int(B.w);
        double t;
        const int k = exp_track(
            S, r, -1,
            [&](int p) __attribute__((always_inline)) {
                return (double)path_rng(P, pix, v, 17u + 2u * (uint32_t)p).u[0];
            },
            stack, err, tc, t);
        if (k == target) collect(P.adj, L, (int)pix, C.x, C.y, C.z, 1.f, 1);
    }
    flush_counts(S, tc);
}

__global__ __launch_bounds__(kBlock) void k_env_exp(SceneDev S, PassArgs P, LightQueue q, const int32_t *n_in,
                                                    float4 *L, int64_t *stats, uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int n = *n_in;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd((unsigned long long *)&stats[2], (unsigned long long)n);
    TraceCount tc;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const float4 A = q.a[i], B = q.b[i], C = q.c[i];
        const RayD r = make_ray(A.x, A.y, A.z, B.x, B.y, B.z, 0.f, __builtin_huge_val());
        const float T = expf(-exp_depth(S, r, __float_as_int(B.w), stack, err, tc));
        if (T > 0.f) collect(P.adj, L, __float_as_int(C.w), C.x, C.y, C.z, T, 2);
    }
    flush_counts(S, tc);
}

// per pixel, the wavefront's samples in sample order (the same float sums
// as one sample per wavefront)
__global__ void k_accum(int64_t npix, int nsamp, const float4 *L, float *sum, float *sumsq) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    float s0 = sum[3 * p], s1 = sum[3 * p + 1], s2 = sum[3 * p + 2];
    float q0 = 0.f, q1 = 0.f, q2 = 0.f;
    if (sumsq) { q0 = sumsq[3 * p]; q1 = sumsq[3 * p + 1]; q2 = sumsq[3 * p + 2]; }
    for (int s = 0; s < nsamp; ++s) {
        const float4 l = L[p + (int64_t)s * npix];
        s0 += l.x; s1 += l.y; s2 += l.z;
        q0 += l.x * l.x; q1 += l.y * l.y; q2 += l.z * l.z;
    }
    sum[3 * p] = s0; sum[3 * p + 1] = s1; sum[3 * p + 2] = s2;
    if (sumsq) { sumsq[3 * p] = q0; sumsq[3 * p + 1] = q1; sumsq[3 * p + 2] = q2; }
}

// Sweeps of the tail kernel, called rather than inlined (it runs few rays; one
// copy of each serves every call site).
__device__ __noinline__ SweepOut tail_sweep_main(const SceneDev &S, const RayD &r, int excl, int mode, float u,
                                                  int target, float stop_a, int *stack, uint32_t *err,
                                                  TraceCount &tc) {
    return sweep<kEventsMain>(S, r, excl, mode, u, target, stack, err, tc, stop_a);
}

__device__ __noinline__ SweepOut tail_sweep_wide(const SceneDev &S, const RayD &r, int excl, int mode, float u,
                                                  int target, float stop_a, int *stack, uint32_t *err,
                                                  TraceCount &tc) {
    return sweep<kEventsWide>(S, r, excl, mode, u, target, stack, err, tc, stop_a);
}

__device__ __forceinline__ SweepOut tail_sweep(const SceneDev &S, const RayD &r, int excl, int mode, float u,
                                               int target, float stop_a, int *stack, uint32_t *err,
                                               TraceCount &tc) {
    SweepOut so = tail_sweep_main(S, r, excl, mode, u, target, stop_a, stack, err, tc);
    if (so.status != 0) so = tail_sweep_wide(S, r, excl, mode, u, target, stop_a, stack, err, tc);
    if (so.status != 0) atomicOr(err, kErrEvents);
    return so;
}

// ---------------------------------------------------------------------------
// Density adjoint of the path tracer (score function).  The densities change
// no sampling decision's inputs other than the free-flight distribution: a
// collision selects primitive k with probability W_k = 1/2 I_k(a_k, min(b_k,
// t_sat)) or escapes with probability T = 1 - F (eq. sampling_overlaps), while
// throughputs, emission pick-ups, directions, scatter points (chord centres)
// and light-sampling densities do not depend on them.  So the derivative of
// the expected image is the expectation, per path, of
//   sum over collisions v: L_v * d log P_v / d d_j
// (P_v the probability of the outcome drawn at v, L_v the radiance the path
// collects from v on), plus the derivatives of the two estimator weights
// that do depend on densities: the emitter factor W_k of a light sample
// (emission rides on the free-flight probability, eq. rte) and the
// transmittance of an environment sample.  I_j is linear in d_j, so at a
// fixed t_sat d W_j / d d_j = W_j / d_j; t_sat moves by
// d t_sat / d d_j = -(W_j(t_sat) / d_j) / F'(t_sat), F' = 1/2 sum G.  The MIS
// weights do not depend on densities.  In the replay the path's slot holds
// L_v when its collision v is processed (nothing of v is collected yet).
// Primitives of zero density get no gradient (W_j / d_j is not formed).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float dens_weight(const AdjArgs &A, int slot, float x, float y, float z) {
    const float *g = A.dimg + 3 * (int64_t)((uint32_t)slot % A.npix);
    return A.inv_spp * (g[0] * x + g[1] * y + g[2] * z);
}

// every primitive j != excl whose clipped chord starts before hi: fn(record, chord)
template <class Fn>
__device__ __forceinline__ void dens_chords(const SceneDev &S, const RayD &r, int excl, float hi, int *stack,
                                            uint32_t *err, TraceCount &tc, Fn &&fn) {
    int spill[kStackSpill];
    TravState ts;
    trav_begin(ts, S);
    traverse(S, r, r.t0, [&]() __attribute__((always_inline)) { return hi; }, stack, spill, ts, 0, err, tc,
             [&](int p) __attribute__((always_inline)) {
                 const HotRec h = load_hot(S.hot, p);
                 return h.orig != excl && !surely_missed(h, r, S.r2);
             },
             [&](int p) __attribute__((always_inline)) {
                 const HotRec h = load_hot(S.hot, p);
                 Chord c;
                 if (chord(h, r, S.r2, c, true) && c.own) fn(h, c);
                 return false;
             });
}

// the t_sat terms of a primitive k straddling t_sat whose weight (or
// factor) enters with coefficient w: grad[j] -= w (1/2 G_k(t_sat)) / F'(t_sat)
// * W_j(t_sat) / d_j for every j entering before t_sat (k included)
__device__ __forceinline__ void dens_tsat_terms(const SceneDev &S, const RayD &r, int excl, double tsat, float gk,
                                                float w, float *grad, int *stack, uint32_t *err, TraceCount &tc) {
    const float hi = (float)tsat * (1.f + 1e-6f) + 1e-30f;
    float Fp = 0.f;
    dens_chords(S, r, excl, hi, stack, err, tc, [&](const HotRec &, const Chord &c) { Fp += half_kernel_at(c, tsat); });
    if (!(Fp > 0.f) || gk == 0.f) return;
    const float coef = w * gk / Fp;
    dens_chords(S, r, excl, hi, stack, err, tc, [&](const HotRec &h, const Chord &c) {
        const float wj = half_integral_to(c, tsat);
        if (wj > 0.f && h.d > 0.f) atomicAdd(grad + h.orig, -coef * wj / h.d);
    });
}

// escape (or an environment sample's transmittance T = 1 - F over the whole
// ray): grad[j] -= w W_j / d_j for every j on the ray, w already divided by T
// for an escape (d log T / d d_j = -(W_j / d_j) / T)
__device__ __forceinline__ void dens_all(const SceneDev &S, const RayD &r, int excl, float w, bool log_T,
                                         float *grad, int *stack, uint32_t *err, TraceCount &tc) {
    if (log_T) {
        float F = 0.f;
        dens_chords(S, r, excl, kInf, stack, err, tc, [&](const HotRec &, const Chord &c) { F += c.W; });
        const float T = 1.f - F;
        if (!(T > 0.f)) return;
        w /= T;
    }
    dens_chords(S, r, excl, kInf, stack, err, tc, [&](const HotRec &h, const Chord &c) {
        if (c.W > 0.f && h.d > 0.f) atomicAdd(grad + h.orig, -w * c.W / h.d);
    });
}

// The rays of the collisions whose t_sat the density adjoint needs (a primitive
// was selected and the pixel's loss weight is not zero), in the queue's traced
// order j, for the saturation query; the others get an empty range.
__global__ void k_dens_rays(PassArgs P, Queue q, const int32_t *n_in, int64_t n, const int32_t *order,
                            const int2 *hits, const float4 *L, float *rays, int32_t *excl) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float *r = rays + 8 * j;
    bool need = false;
    float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = make_float4(0.f, 0.f, 1.f, __int_as_float(-1));
    if (j < *n_in) {
        const int64_t i = order ? (int64_t)order[j] : j;
        A = q.a[i];
        B = q.b[i];
        const int slot = __float_as_int(q.c[i].w) & kPixMask;
        const float4 Rv = L[slot];
        need = hits[i].x >= 0 && dens_weight(P.adj, slot, Rv.x, Rv.y, Rv.z) != 0.f;
    }
    if (!need) {
        A = make_float4(0.f, 0.f, 0.f, 0.f);
        B = make_float4(0.f, 0.f, 1.f, B.w);
    }
    r[0] = A.x; r[1] = A.y; r[2] = A.z;
    r[3] = B.x; r[4] = B.y; r[5] = B.z;
    r[6] = 0.f;
    r[7] = need ? __builtin_huge_valf() : 0.f;
    excl[j] = __float_as_int(B.w);
}

// collisions of the path queue (before their shading collects anything);
// tsat[j] is the saturation query's t_sat of the entry traced j-th
__global__ __launch_bounds__(kBlock) void k_dens_collide(SceneDev S, PassArgs P, Queue q, const int32_t *n_in,
                                                         const int32_t *order, const int2 *hits, const float4 *L,
                                                         const double *tsat, uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int n = *n_in;
    TraceCount tc;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        const int64_t i = order ? (int64_t)order[j] : j;
        const float4 A = q.a[i], B = q.b[i], C = q.c[i];
        const int slot = __float_as_int(C.w) & kPixMask;
        const float4 Rv = L[slot];
        const float w = dens_weight(P.adj, slot, Rv.x, Rv.y, Rv.z);
        if (w == 0.f) continue;
        const int excl = __float_as_int(B.w), k = hits[i].x;
        const RayD r = make_ray(A.x, A.y, A.z, B.x, B.y, B.z, 0.f, __builtin_huge_val());
        if (k < 0) {
            dens_all(S, r, excl, w, true, P.adj.grad_dens, stack, err, tc);
            continue;
        }
        const HotRec hk = load_hot(S.hot, S.inv[k]);
        Chord ck;
        if (!chord(hk, r, S.r2, ck) || !(hk.d > 0.f)) continue;
        atomicAdd(P.adj.grad_dens + k, w / hk.d);
        const double td = tsat[j];  // NaN where the query overflowed (reported by ugp_sync)
        if (td < ck.bd) {  // k straddles t_sat
            const float wk = half_integral_to(ck, td);
            if (wk > 0.f)
                dens_tsat_terms(S, r, excl, td, half_kernel_at(ck, td), w / wk, P.adj.grad_dens, stack, err, tc);
        }
    }
}

// The light samples' rays clipped at their target's exit, in traced order,
// for the density adjoint's saturation query (an empty range where the
// pixel's loss weight is zero or the ray misses its target)
__global__ void k_dens_light_rays(SceneDev S, LightQueue q, const int32_t *n_in, int64_t n, const int32_t *order,
                                  AdjArgs adj, float *rays, int32_t *excl) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float *r = rays + 8 * j;
    float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = make_float4(0.f, 0.f, 1.f, __int_as_float(-1));
    float t1 = 0.f;
    if (j < *n_in) {
        const int64_t i = order ? (int64_t)order[j] : j;
        const float4 C = q.c[i];
        A = q.a[i];
        B = q.b[i];
        const HotRec hk = load_hot(S.hot, S.inv[__float_as_int(A.w)]);
        Chord ck;
        if (dens_weight(adj, __float_as_int(C.w), C.x, C.y, C.z) != 0.f && hk.d > 0.f &&
            chord(hk, make_ray(A.x, A.y, A.z, B.x, B.y, B.z, 0.f, __builtin_huge_val()), S.r2, ck))
            t1 = (float)ck.bd;
    }
    if (!(t1 > 0.f)) {
        A = make_float4(0.f, 0.f, 0.f, 0.f);
        B = make_float4(0.f, 0.f, 1.f, B.w);
        t1 = 0.f;
    }
    r[0] = A.x; r[1] = A.y; r[2] = A.z;
    r[3] = B.x; r[4] = B.y; r[5] = B.z;
    r[6] = 0.f;
    r[7] = t1;
    excl[j] = __float_as_int(B.w);
}

// light samples: the emitter factor W_k of target k along the ray clipped at
// its exit, times the sample's weight; tsat[j] is the saturation query's
// t_sat of the sample traced j-th (its range's end, rounded to float, when
// the ray does not saturate before the exit)
__global__ __launch_bounds__(kBlock) void k_dens_light(SceneDev S, LightQueue q, const int32_t *n_in,
                                                       const int32_t *order, AdjArgs adj, const double *tsat,
                                                       uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int n = *n_in;
    TraceCount tc;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        const int64_t i = order ? (int64_t)order[j] : j;
        const float4 A = q.a[i], B = q.b[i], C = q.c[i];
        const float w = dens_weight(adj, __float_as_int(C.w), C.x, C.y, C.z);
        if (w == 0.f) continue;
        const int target = __float_as_int(A.w), excl = __float_as_int(B.w);
        RayD r = make_ray(A.x, A.y, A.z, B.x, B.y, B.z, 0.f, __builtin_huge_val());
        const HotRec hk = load_hot(S.hot, S.inv[target]);
        Chord ck;
        if (!chord(hk, r, S.r2, ck) || !(hk.d > 0.f)) continue;
        r.t1 = ck.bd;
        double td = tsat[j];
        if (!(td == td)) continue;  // the query overflowed (reported by ugp_sync)
        const bool sat = td < (double)(float)ck.bd;  // saturates before the target's exit
        if (!sat) td = ck.bd;
        const float wk = half_integral_to(ck, td);
        if (!(wk > 0.f)) continue;  // hidden by primitives in front: factor 0
        atomicAdd(adj.grad_dens + target, w * wk / hk.d);
        if (sat) dens_tsat_terms(S, r, excl, td, half_kernel_at(ck, td), w, adj.grad_dens, stack, err, tc);
    }
}

// environment samples: T = 1 - F along the whole ray, times the sample's weight
__global__ __launch_bounds__(kBlock) void k_dens_env(SceneDev S, LightQueue q, const int32_t *n_in, AdjArgs adj,
                                                     uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int n = *n_in;
    TraceCount tc;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const float4 A = q.a[i], B = q.b[i], C = q.c[i];
        const float w = dens_weight(adj, __float_as_int(C.w), C.x, C.y, C.z);
        if (w == 0.f) continue;
        const RayD r = make_ray(A.x, A.y, A.z, B.x, B.y, B.z, 0.f, __builtin_huge_val());
        float F = 0.f;
        dens_chords(S, r, __float_as_int(B.w), kInf, stack, err, tc, [&](const HotRec &, const Chord &c) { F += c.W; });
        if (!(F < 1.f)) continue;  // T = 0: the sample added nothing, and nothing nearby
        dens_all(S, r, __float_as_int(B.w), w, false, adj.grad_dens, stack, err, tc);
    }
}

__device__ __forceinline__ void add_radiance(float4 *L, int pix, float x, float y, float z, float f) {
    float4 l = L[pix];
    l.x = fmaf(x, f, l.x); l.y = fmaf(y, f, l.y); l.z = fmaf(z, f, l.z);  // as collect()
    L[pix] = l;
}

// The last bounces of a chunk, once few paths are left and none is still to
// be generated: the paths run to their end in one launch (each wavefront
// launch would last as long as the slowest of a few thousand rays).  A path
// has two lanes of a wave: lane j < 32 traces its collisions and shades, lane
// j + 32 traces the light sample of the previous vertex meanwhile (the two
// queries start at the same vertex and are independent).  The radiance is
// added in the wavefront's order per path -- emission at vertex v, its light
// sample, its environment sample, then vertex v + 1 -- so it is the same
// float sum.
__global__ __launch_bounds__(kBlock) void k_tail(SceneDev S, PassArgs P, Queue q, const int32_t *n_in, float4 *L,
                                                 int64_t *stats, uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int n = *n_in;
    const int lane = threadIdx.x, jl = lane & 31;
    const bool helper = lane >= 32;
    const int64_t i = (int64_t)blockIdx.x * 32 + jl;
    TraceCount tc;
    unsigned long long n_col = 0, n_light = 0, n_env = 0;
    float4 A{}, B{}, C{};
    int v = 0;
    bool col = !helper && i < n;  // a collision to trace (path lanes)
    if (col) {
        A = q.a[i]; B = q.b[i]; C = q.c[i];
        v = q.v[i];
    }
    bool nee = false, env = false;  // samples of the last shaded vertex still to add (path lanes)
    float4 na{}, nb{}, nc{}, ea{}, eb{}, ec{};
    for (;;) {
        if (!__any(col || nee || env)) break;
        // the light sample of the path's last vertex goes to its helper lane
        const bool hq = __shfl(nee ? 1 : 0, jl) != 0;
        const float4 hna = make_float4(__shfl(na.x, jl), __shfl(na.y, jl), __shfl(na.z, jl), __shfl(na.w, jl));
        const float4 hnb = make_float4(__shfl(nb.x, jl), __shfl(nb.y, jl), __shfl(nb.z, jl), __shfl(nb.w, jl));
        bool query = false;
        RayD r = make_ray(0.f, 0.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.0);
        int excl = -1, mode = kModeCollide, target = -1;
        float u = 0.f, stop_a = -kInf;
        if (!helper && col) {
            const int pix = __float_as_int(C.w) & kPixMask;
            u = path_rng(P, (uint32_t)pix, (uint32_t)v, 0).u[0];
            r = make_ray(A.x, A.y, A.z, B.x, B.y, B.z, 0.f, __builtin_huge_val());
            excl = __float_as_int(B.w);
            query = true;
            ++n_col;
        }
        if (helper && hq) {
            target = __float_as_int(hna.w);
            r = make_ray(hna.x, hna.y, hna.z, hnb.x, hnb.y, hnb.z, 0.f, __builtin_huge_val());
            Chord c;
            if (chord(load_hot(S.hot, S.inv[target]), r, S.r2, c)) {
                r.t1 = c.bd;
                stop_a = c.a;
                excl = __float_as_int(hnb.w);
                mode = kModeEmitter;
                query = true;
            }
        }
        SweepOut so{-1, 0.f, 1};
        if (query) so = tail_sweep(S, r, excl, mode, u, target, stop_a, stack, err, tc);
        const float f = helper && query && so.status == 0 ? so.t : 0.f;
        const float f_nee = __shfl(f, jl + 32);
        if (!helper) {
            if (nee) {
                if (f_nee > 0.f) add_radiance(L, __float_as_int(nc.w), nc.x, nc.y, nc.z, f_nee);
                nee = false;
            }
            if (env) {
                const RayD er = make_ray(ea.x, ea.y, ea.z, eb.x, eb.y, eb.z, 0.f, __builtin_huge_val());
                const float T = fmaxf(0.f, 1.f - transmittance_F(S, er, __float_as_int(eb.w), true, stack, err, tc));
                if (T > 0.f) add_radiance(L, __float_as_int(ec.w), ec.x, ec.y, ec.z, T);
                env = false;
            }
            if (col) {
                const int2 hit = so.status != 0 ? make_int2(-1, __float_as_int(0.f))
                                                : make_int2(so.prim, __float_as_int(so.t));
                ShadeOut o;
                shade_one(S, P, A, B, C, v, hit, L, o);
                nee = o.do_nee;
                na = o.na; nb = o.nb; nc = o.nc;
                env = o.do_env;
                ea = o.ea; eb = o.eb; ec = o.ec;
                n_light += o.do_nee ? 1 : 0;
                n_env += o.do_env ? 1 : 0;
                if (P.nrc.mode != 0) {
                    if (o.do_qry) {
                        const int pq = atomicAdd(P.nrc.n_qry, 1);
                        float4 *w = reinterpret_cast<float4 *>(P.nrc.qry + (int64_t)kNrcRecordFloats * pq);
                        w[0] = o.r0; w[1] = o.r1; w[2] = o.r2; w[3] = o.r3; w[4] = o.r4;
                    }
                    if (o.do_rec) {
                        const int pr = atomicAdd(P.nrc.n_rec, 1);
                        if (pr < P.nrc.rec_cap) {
                            float4 *w = reinterpret_cast<float4 *>(P.nrc.rec + (int64_t)kNrcRecordFloats * pr);
                            w[0] = o.r0; w[1] = o.r1; w[2] = o.r2; w[3] = o.r3; w[4] = o.r4; w[5] = o.r5;
                        }
                    }
                }
                col = o.cont;
                if (col) {
                    A = o.ca; B = o.cb; C = o.cc;
                    ++v;
                }
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        n_col += __shfl_xor(n_col, off);
        n_light += __shfl_xor(n_light, off);
        n_env += __shfl_xor(n_env, off);
    }
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long *)&stats[0], n_col);
        atomicAdd((unsigned long long *)&stats[1], n_light);
        atomicAdd((unsigned long long *)&stats[2], n_env);
    }
    flush_counts(S, tc);
}

__global__ void k_set_count(int32_t *c, int32_t v) { *c = v; }

// running total of a count (radiance-cache queries, training records)
__global__ void k_nrc_count(const int32_t *cnt, int64_t *total) { *total += *cnt; }

// pool buffers for `cap` path slots and radiance slots for `lcap` paths
hipError_t ensure_buffers(ugp_ctx ctx, int64_t cap, int64_t lcap) {
    RenderBuffers *rb = ctx->rb;
    if (rb && rb->cap >= cap && rb->lcap >= lcap) return hipSuccess;
    if (rb) {
        cap = std::max(cap, rb->cap);
        lcap = std::max(lcap, rb->lcap);
    }
    free_render(ctx);
    rb = new RenderBuffers();
    const size_t q = sizeof(float4) * (size_t)cap;
    const size_t counts = sizeof(int32_t) * (kChunkBlock + kCountStride);
    const size_t total = 12 * q + sizeof(float4) * (size_t)lcap + 2 * sizeof(int32_t) * (size_t)cap +
                         sizeof(int32_t) * (size_t)cap + sizeof(int2) * (size_t)cap + counts +
                         4 * sizeof(int32_t) * (size_t)cap + 32 * 256;
    hipError_t e = hipMalloc(&rb->block, total);
    if (e != hipSuccess) {
        delete rb;
        return e;
    }
    e = hipHostMalloc((void **)&rb->host, sizeof(int32_t) * 4, hipHostMallocDefault);
    if (e != hipSuccess) {
        hipFree(rb->block);
        delete rb;
        return e;
    }
    char *p = (char *)rb->block;
    auto take = [&](size_t bytes) {
        void *r = p;
        p += (bytes + 255) & ~(size_t)255;
        return r;
    };
    for (int k = 0; k < 2; ++k) {
        rb->q[k].a = (float4 *)take(q);
        rb->q[k].b = (float4 *)take(q);
        rb->q[k].c = (float4 *)take(q);
        rb->q[k].v = (int32_t *)take(sizeof(int32_t) * (size_t)cap);
    }
    rb->nee.a = (float4 *)take(q); rb->nee.b = (float4 *)take(q); rb->nee.c = (float4 *)take(q);
    rb->env.a = (float4 *)take(q); rb->env.b = (float4 *)take(q); rb->env.c = (float4 *)take(q);
    rb->L = (float4 *)take(sizeof(float4) * (size_t)lcap);
    rb->ovf = (int32_t *)take(sizeof(int32_t) * (size_t)cap);
    rb->hits = (int2 *)take(sizeof(int2) * (size_t)cap);
    rb->skey = (uint32_t *)take(sizeof(uint32_t) * (size_t)cap);
    rb->skey2 = (uint32_t *)take(sizeof(uint32_t) * (size_t)cap);
    rb->sval = (int32_t *)take(sizeof(int32_t) * (size_t)cap);
    rb->sval2 = (int32_t *)take(sizeof(int32_t) * (size_t)cap);
    rb->counts = (int32_t *)take(counts);
    rb->cap = cap;
    rb->lcap = lcap;
    ctx->rb = rb;
    return hipSuccess;
}

}  // namespace

void free_render(ugp_ctx ctx) {
    if (ctx->rb) {
        hipFree(ctx->rb->block);
        hipHostFree(ctx->rb->host);
        hipFree(ctx->rb->qry);
        hipFree(ctx->rb->nrc_block);
        delete ctx->rb;
        ctx->rb = nullptr;
    }
}

namespace {

__global__ void k_set_float(float *p, float v) { *p = v; }

// a bijection of [0, 2^25) (multiplications by odd constants and xor-shifts
// within 25 bits), so that paths of nearby slots scatter over the key range
__device__ __forceinline__ uint32_t slot_mix(uint32_t x) {
    constexpr uint32_t m = (1u << 25) - 1u;
    x = (x * 0x9E3779B1u) & m;
    x ^= x >> 12;
    x = (x * 0x85EBCA77u) & m;
    x ^= x >> 13;
    return x;
}

// sort keys of the staged records: the mixed path slot (radiance slots are
// below 2^25), all ones past the staged count; the values are staging indices
__global__ void k_rec_keys(const int32_t *n_dev, int64_t stage, const float *staged, uint32_t *keys,
                           int32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= stage) return;
    const int64_t n = (int64_t)*n_dev < stage ? (int64_t)*n_dev : stage;
    keys[i] = i < n ? slot_mix((uint32_t)__float_as_int(staged[kNrcRecordFloats * i + 19]) & ((1u << 25) - 1u))
                    : 0xFFFFFFFFu;
    vals[i] = (int32_t)i;
}

// the first min(staged, cap) records in key order.  The sort is stable and a
// path's records are staged in vertex order (each is appended one bounce
// after the last), so the order, and which records fill the cap, depends
// only on which paths were training paths.
__global__ void k_rec_gather(const int32_t *n_dev, int64_t cap, const int32_t *order, const float *staged,
                             float *rec) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)*n_dev < cap ? (int64_t)*n_dev : cap;
    if (j >= n) return;
    const float4 *src = reinterpret_cast<const float4 *>(staged + (int64_t)kNrcRecordFloats * order[j]);
    float4 *dst = reinterpret_cast<float4 *>(rec + (int64_t)kNrcRecordFloats * j);
#pragma unroll
    for (int k = 0; k < kNrcRecordFloats / 4; ++k) dst[k] = src[k];
}

// radiance-cache buffers of a render: queries for every pixel, training
// records and targets for rec_cap records, the training-path probability
hipError_t ensure_nrc_buffers(ugp_ctx ctx, int64_t npix, int64_t rec_cap, bool *fresh) {
    RenderBuffers *rb = ctx->rb;
    *fresh = false;
    if (!rb->qry) {
        hipError_t e = hipMalloc((void **)&rb->qry, sizeof(float) * kNrcRecordFloats * (size_t)rb->cap);
        if (e != hipSuccess) return e;
    }
    if (rb->rec_cap < rec_cap || !rb->nrc_block) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return e;
        hipFree(rb->nrc_block);
        rb->nrc_block = nullptr;
        rb->rec_cap = 0;
        const int64_t cap = rec_cap < 1024 ? 1024 : rec_cap;
        const size_t stage = (size_t)(kRecStage * cap);
        const size_t bytes = sizeof(float) * (stage + (size_t)cap) * kNrcRecordFloats +
                             sizeof(float) * 3 * (size_t)cap + 4 * sizeof(uint32_t) * stage + 2 * 256;
        e = hipMalloc(&rb->nrc_block, bytes);
        if (e != hipSuccess) return e;
        rb->staged = (float *)rb->nrc_block;
        rb->rec = rb->staged + stage * kNrcRecordFloats;
        rb->targets = rb->rec + (size_t)cap * kNrcRecordFloats;
        rb->rkey = (uint32_t *)(rb->targets + 3 * (size_t)cap);
        rb->rkey2 = rb->rkey + stage;
        rb->rval = (int32_t *)(rb->rkey2 + stage);
        rb->rval2 = rb->rval + stage;
        rb->frac = (float *)((char *)rb->nrc_block + bytes - 2 * 256);
        rb->loss = rb->frac + 64;
        rb->rec_cap = cap;
        *fresh = true;
    }
    (void)npix;
    return hipSuccess;
}

}  // namespace

void make_cam_dev(const ugp_camera *cam, CamDev *out) {
    // camera basis (double on the host, float on the device)
    double f[3] = {(double)cam->target[0] - cam->origin[0], (double)cam->target[1] - cam->origin[1],
                   (double)cam->target[2] - cam->origin[2]};
    double fl = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    for (double &x : f) x /= fl;
    const double up[3] = {cam->up[0], cam->up[1], cam->up[2]};
    double rt[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
    const double rl = sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
    for (double &x : rt) x /= rl;
    const double u[3] = {rt[1] * f[2] - rt[2] * f[1], rt[2] * f[0] - rt[0] * f[2], rt[0] * f[1] - rt[1] * f[0]};
    const double th = tan(0.5 * (double)cam->vfov_deg * 3.14159265358979323846 / 180.0);
    const double asp = (double)cam->width / (double)cam->height;
    *out = CamDev{cam->origin[0], cam->origin[1], cam->origin[2], (float)f[0], (float)f[1], (float)f[2],
                  (float)(rt[0] * th * asp), (float)(rt[1] * th * asp), (float)(rt[2] * th * asp),
                  (float)(u[0] * th), (float)(u[1] * th), (float)(u[2] * th), cam->width, cam->height};
}

hipError_t render(ugp_ctx ctx, const ugp_camera *cam, const ugp_render_params *p, float *sum, float *sumsq,
                  const RenderAdjoint *adj) {
    const SceneDev &S0 = ctx->scene;
    const int64_t npix = (int64_t)cam->width * cam->height;
    // chunks of `cs` samples of every pixel share the pool of path slots
    const int cs = (int)std::max<int64_t>(1, std::min<int64_t>(p->spp, kChunkPaths / npix));
    const int64_t lcap = npix * cs;
    const int64_t pool = std::min<int64_t>(ctx->path_pool > 0 ? ctx->path_pool : kPoolPaths, lcap);
    hipError_t e = ensure_buffers(ctx, pool, lcap);
    if (e != hipSuccess) return e;
    RenderBuffers *rb = ctx->rb;
    hipStream_t st = ctx->stream;
    // shading adjoints: the replay's per-slot ratios (three float4 per
    // radiance slot for each of albedo and roughness that is wanted)
    AdjArgs adjA;
    float4 *aux = nullptr;
    struct AuxFree {
        float4 *&p;
        hipStream_t s;
        ~AuxFree() {
            if (p) hipFreeAsync(p, s);
        }
    } aux_free{aux, st};
    char *dens_mem = nullptr;
    struct DensFree {
        char *&p;
        hipStream_t s;
        ~DensFree() {
            if (p) hipFreeAsync(p, s);
        }
    } dens_free{dens_mem, st};
    double *dens_td = nullptr;
    float *dens_rays = nullptr;
    int32_t *dens_excl = nullptr;
    if (adj) {
        const int nsh = (adj->grad_albedo ? 1 : 0) + (adj->grad_roughness ? 1 : 0);
        if (nsh > 0) {
            e = hipMallocAsync((void **)&aux, sizeof(float4) * 3 * (size_t)nsh * (size_t)lcap, st);
            if (e != hipSuccess) return e;
            float4 *next = aux;
            for (int w = 0; w < 2; ++w) {
                if (!(w == 0 ? adj->grad_albedo : adj->grad_roughness)) continue;
                for (int kind = 0; kind < 3; ++kind) adjA.aux[w][kind] = next + (int64_t)kind * lcap;
                next += 3 * lcap;
            }
        }
        if (adj->grad_density) {  // the density adjoint's saturation queries: rays, exclusions, t_sat
            e = hipMallocAsync((void **)&dens_mem, (sizeof(float) * 8 + sizeof(int32_t) + sizeof(double)) * (size_t)pool,
                               st);
            if (e != hipSuccess) return e;
            dens_td = (double *)dens_mem;
            dens_rays = (float *)(dens_td + pool);
            dens_excl = (int32_t *)(dens_rays + 8 * pool);
        }
        adjA.dimg = adj->d_image;
        adjA.grad_alb = adj->grad_albedo;
        adjA.grad_rough = adj->grad_roughness;
        adjA.grad_dens = adj->grad_density;
        adjA.inv_spp = 1.f / (float)p->spp;
        adjA.npix = (uint32_t)npix;
    }
    PassArgs P;
    make_cam_dev(cam, &P.cam);
    for (int k = 0; k < 3; ++k) {
        P.blo[k] = S0.lo[k];
        const float ext = S0.hi[k] - S0.lo[k];
        P.binv[k] = ext > 0.f ? 1.f / ext : 0.f;
    }
    P.seed = p->seed;
    P.npix = (uint32_t)npix;
    P.max_depth = p->max_depth;
    P.mis_mode = p->mis_mode;
    P.env[0] = p->env_radiance[0]; P.env[1] = p->env_radiance[1]; P.env[2] = p->env_radiance[2];
    P.has_env = (P.env[0] > 0.f || P.env[1] > 0.f || P.env[2] > 0.f) ? 1 : 0;
    P.transport = p->transport;
    int32_t *chunk_cnt = rb->counts + kChunkBlock;  // [0] paths generated, [1] records appended
    // radiance cache: modes 1 and 2 need the network; records only in mode 1
    P.nrc = NrcArgs{p->nrc_mode, p->nrc_terminate_after, nullptr, nullptr, 0, nullptr, nullptr, nullptr};
    float nrc_box[6];
    const float *box = nullptr;
    const float *nrc_scale = nullptr;
    if (p->nrc_mode != 0) {
        bool valid = true;
        for (int k = 0; k < 3; ++k) valid = valid && p->nrc_box[3 + k] > p->nrc_box[k];
        if (valid) {
            for (int k = 0; k < 6; ++k) nrc_box[k] = p->nrc_box[k];
            box = nrc_box;
        }
        if (p->nrc_mode != 3) {
            e = nrc_ensure(ctx);
            if (e != hipSuccess) return e;
            e = nrc_set_scale(ctx, p->nrc_radiance_scale);
            if (e != hipSuccess) return e;
            nrc_scale = nrc_scale_ptr(ctx);
        }
        bool fresh = false;
        e = ensure_nrc_buffers(ctx, pool, p->nrc_mode == 1 ? p->nrc_train_records : 0, &fresh);
        if (e != hipSuccess) return e;
        if (p->nrc_mode == 1 && (fresh || ctx->nrc_frac_pixels != lcap)) {
            // a training path is chosen with probability frac; frac starts at
            // records / (8 paths of a chunk) and is adapted after every chunk
            const float f0 = std::min(1.0f, (float)p->nrc_train_records / (8.0f * (float)lcap));
            hipLaunchKernelGGL(k_set_float, dim3(1), dim3(1), 0, st, rb->frac, f0);
            ctx->nrc_frac_pixels = lcap;
        }
        P.nrc.qry = rb->qry;
        P.nrc.frac = rb->frac;
        if (p->nrc_mode == 1) {
            P.nrc.rec = rb->staged;
            P.nrc.n_rec = chunk_cnt + ctr(1);
            P.nrc.rec_cap = (int32_t)(kRecStage * p->nrc_train_records);
        }
    }
    e = hipMemsetAsync(ctx->stats, 0, sizeof(int64_t) * 8, st);
    if (e != hipSuccess) return e;
    // profiling: level 2 counts traversal work, level >= 1 brackets launches with events
    // per kernel category c (0 collide, 1 collide overflow, 2 light, 3 env) the
    // counters live at ctx->counters + 3 c
    SceneDev S = S0, Sc[4] = {S0, S0, S0, S0};
    if (ctx->profiling >= 2) {
        e = hipMemsetAsync(ctx->counters, 0, sizeof(unsigned long long) * 12, st);
        if (e != hipSuccess) return e;
        for (int c = 0; c < 4; ++c) Sc[c].count = ctx->counters + 3 * c;
    }
    ctx->ev_used.clear();
    ctx->ev_cat_valid = ctx->profiling >= 1;
    size_t ev_next = 0;
    auto timed = [&](int cat, auto &&launch) {
        if (ctx->profiling < 1) {
            launch();
            return;
        }
        while (ctx->ev_pool.size() < ev_next + 2) {
            hipEvent_t ev;
            if (hipEventCreate(&ev) != hipSuccess) {
                launch();
                return;
            }
            ctx->ev_pool.push_back(ev);
        }
        hipEventRecord(ctx->ev_pool[ev_next], st);
        launch();
        hipEventRecord(ctx->ev_pool[ev_next + 1], st);
        ctx->ev_used.push_back({cat, (int)ev_next});
        ev_next += 2;
    };
    const unsigned gw = 256;  // the overflow pass: few paths
    for (int s0 = 0; s0 < p->spp; s0 += cs) {
        P.sample = (uint32_t)(p->sample_offset + s0);
        const int ns = std::min(cs, p->spp - s0);
        const int64_t total = npix * ns;
        // with an adjoint the chunk is traced twice: forward, then the replay
        for (int pass = 0; pass < (adj ? 2 : 1); ++pass) {
            P.adj = pass == 1 ? adjA : AdjArgs{};
            e = hipMemsetAsync(rb->counts, 0, sizeof(int32_t) * (kChunkBlock + kCountStride), st);
            if (e != hipSuccess) return e;
            // iterations until every path of the chunk has ended; each path takes
            // at most max_depth + 1 iterations once generated
            const int64_t max_iter = (int64_t)(p->max_depth + 2) * (total / pool + 2);
            int64_t it = 0;
            int64_t left = 0, gen = 0;  // paths carried into this iteration, paths generated (host copies)
            for (;; ++it) {
                if (it > max_iter) return hipErrorUnknown;  // a path outlived its depth: internal error
                int32_t *c = rb->counts + kCountStride * (it & 1);        // input queue's counters
                int32_t *cn = rb->counts + kCountStride * ((it + 1) & 1); // output queue's counters
                Queue qin = rb->q[it & 1], qout = rb->q[(it + 1) & 1];
                Overflow ov{rb->ovf, c + ctr(3)};
                // queue length of this iteration, known on the host: launches are sized to it
                const int64_t n_new = std::min(pool - left, total - gen);
                const int64_t n_it = left + n_new;
                const unsigned gn = (unsigned)std::max<int64_t>(1, (n_it + 255) / 256);
                const unsigned gq = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n_it + kBlock - 1) / kBlock,
                                                                                      kPersistBlocks));
                const bool sorted = n_it >= kSortMin;
                const int32_t *order = sorted ? (const int32_t *)rb->sval : nullptr;
                hipLaunchKernelGGL(k_regen, dim3((unsigned)std::max<int64_t>(1, (n_new + 255) / 256)), dim3(256), 0, st,
                                   P, pool, total, (const int32_t *)c, (const int32_t *)chunk_cnt, qin, rb->L);
                hipLaunchKernelGGL(k_regen_commit, dim3(1), dim3(1), 0, st, pool, total, c, cn, chunk_cnt);
                P.nrc.n_qry = c + ctr(6);
                if (!adj && !P.transport && it > 0 && n_new == 0 && n_it <= ctx->tail_paths) {
                    // few paths left and none to generate: they run to the end in one kernel
                    timed(8, [&] {
                        hipLaunchKernelGGL(k_tail, dim3((unsigned)std::max<int64_t>(1, (n_it + 31) / 32)),
                                           dim3(kBlock), 0, st, Sc[1], P, qin, (const int32_t *)c, rb->L, ctx->stats,
                                           ctx->err);
                    });
                    if (p->nrc_mode == 1 || p->nrc_mode == 2) {
                        timed(6, [&] {
                            e = nrc_forward(ctx, n_it, c + ctr(6), rb->qry, kNrcRecordFloats, 2, box, nullptr, rb->L,
                                            nrc_scale);
                        });
                        if (e != hipSuccess) return e;
                        hipLaunchKernelGGL(k_nrc_count, dim3(1), dim3(1), 0, st, (const int32_t *)(c + ctr(6)),
                                           ctx->stats + 3);
                    }
                    break;
                }
                // order the queue so each wave's rays are coherent
                if (sorted)
                    timed(5, [&] {
                        hipLaunchKernelGGL(k_sort_keys, dim3(gn), dim3(256), 0, st, P, qin, (const int32_t *)c, n_it,
                                           rb->skey, rb->sval);
                        radix_sort(rb->skey, rb->sval, rb->skey2, rb->sval2, n_it, st);
                    });
                if (P.transport) {
                    timed(0, [&] {
                        hipLaunchKernelGGL(k_collide_exp, dim3(gq), dim3(kBlock), 0, st, Sc[0], P, qin,
                                           (const int32_t *)c, order, rb->hits, ctx->stats, ctx->err);
                    });
                } else {
                    timed(0, [&] {
                        hipLaunchKernelGGL((k_collide<kEventsMain, false>), dim3(gq), dim3(kBlock), 0, st, Sc[0], P,
                                           qin, (const int32_t *)c, order, c + ctr(4), rb->hits, ctx->stats, ov,
                                           ctx->err);
                    });
                    timed(1, [&] {
                        hipLaunchKernelGGL((k_collide<kEventsWide, true>), dim3(gw), dim3(kBlock), 0, st, Sc[1], P,
                                           qin, (const int32_t *)c, order, c + ctr(4), rb->hits, ctx->stats, ov,
                                           ctx->err);
                    });
                }
                if (P.adj.dimg && P.adj.grad_dens != nullptr) {
                    // t_sat of the collisions by the persistent saturation query
                    hipLaunchKernelGGL(k_dens_rays, dim3(gn), dim3(256), 0, st, P, qin, (const int32_t *)c, n_it,
                                       order, (const int2 *)rb->hits, (const float4 *)rb->L, dens_rays, dens_excl);
                    e = launch_sweep(ctx, kModeSaturate, n_it, dens_rays, dens_excl, nullptr, nullptr, nullptr,
                                     nullptr, nullptr, dens_td);
                    if (e != hipSuccess) return e;
                    hipLaunchKernelGGL(k_dens_collide, dim3(gq), dim3(kBlock), 0, st, S, P, qin, (const int32_t *)c,
                                       order, (const int2 *)rb->hits, (const float4 *)rb->L, (const double *)dens_td,
                                       ctx->err);
                }
                timed(4, [&] {
                    hipLaunchKernelGGL(k_shade, dim3(gq), dim3(kBlock), 0, st, S, P, qin, (const int32_t *)c,
                                       (const int2 *)rb->hits, qout, cn, rb->nee, c + ctr(1), rb->env, c + ctr(2), rb->L);
                });
                if (S.n_emit > 0 && p->mis_mode != 1) {
                    // light queue (at most n_it records) sorted like the path queue
                    if (sorted)
                        timed(5, [&] {
                            const Queue lq{rb->nee.a, rb->nee.b, rb->nee.c, nullptr};
                            hipLaunchKernelGGL(k_sort_keys, dim3(gn), dim3(256), 0, st, P, lq, (const int32_t *)(c + ctr(1)),
                                               n_it, rb->skey, rb->sval);
                            radix_sort(rb->skey, rb->sval, rb->skey2, rb->sval2, n_it, st);
                        });
                    if (P.transport)
                        timed(2, [&] {
                            hipLaunchKernelGGL(k_light_exp, dim3(gq), dim3(kBlock), 0, st, Sc[2], P, rb->nee,
                                               (const int32_t *)(c + ctr(1)), order, rb->L, ctx->stats, ctx->err);
                        });
                    else
                    timed(2, [&] {
                        hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, st, c + ctr(3), 0);
                        hipLaunchKernelGGL((k_light<kEventsMain, false>), dim3(gq), dim3(kBlock), 0, st, Sc[2], rb->nee,
                                           (const int32_t *)(c + ctr(1)), order, c + ctr(5), rb->L, ctx->stats, ov, P.adj,
                                           ctx->err);
                        hipLaunchKernelGGL((k_light<kEventsWide, true>), dim3(gw), dim3(kBlock), 0, st, Sc[2], rb->nee,
                                           (const int32_t *)(c + ctr(1)), order, c + ctr(5), rb->L, ctx->stats, ov, P.adj,
                                           ctx->err);
                    });
                    if (P.adj.dimg && P.adj.grad_dens != nullptr) {
                        // t_sat of the light samples (at most n_it) by the persistent saturation query
                        hipLaunchKernelGGL(k_dens_light_rays, dim3(gn), dim3(256), 0, st, S, rb->nee,
                                           (const int32_t *)(c + ctr(1)), n_it, order, P.adj, dens_rays, dens_excl);
                        e = launch_sweep(ctx, kModeSaturate, n_it, dens_rays, dens_excl, nullptr, nullptr, nullptr,
                                         nullptr, nullptr, dens_td);
                        if (e != hipSuccess) return e;
                        hipLaunchKernelGGL(k_dens_light, dim3(gq), dim3(kBlock), 0, st, S, rb->nee,
                                           (const int32_t *)(c + ctr(1)), order, P.adj, (const double *)dens_td, ctx->err);
                    }
                }
                if (P.has_env && p->mis_mode != 1)
                    timed(3, [&] {
                        if (P.transport)
                            hipLaunchKernelGGL(k_env_exp, dim3(gq), dim3(kBlock), 0, st, Sc[3], P, rb->env,
                                               (const int32_t *)(c + ctr(2)), rb->L, ctx->stats, ctx->err);
                        else
                            hipLaunchKernelGGL(k_env, dim3(gq), dim3(kBlock), 0, st, Sc[3], rb->env,
                                               (const int32_t *)(c + ctr(2)), rb->L, ctx->stats, P.adj, ctx->err);
                    });
                if (P.has_env && p->mis_mode != 1 && P.adj.dimg && P.adj.grad_dens != nullptr)
                    hipLaunchKernelGGL(k_dens_env, dim3(gq), dim3(kBlock), 0, st, S, rb->env, (const int32_t *)(c + ctr(2)),
                                       P.adj, ctx->err);
                if (p->nrc_mode == 1 || p->nrc_mode == 2) {
                    // cached radiance of the paths that ended in the cache this iteration
                    timed(6, [&] {
                        e = nrc_forward(ctx, n_it, c + ctr(6), rb->qry, kNrcRecordFloats, 2, box, nullptr, rb->L, nrc_scale);
                    });
                    if (e != hipSuccess) return e;
                    hipLaunchKernelGGL(k_nrc_count, dim3(1), dim3(1), 0, st, (const int32_t *)(c + ctr(6)), ctx->stats + 3);
                }
                // continue while paths remain in the next queue or wait to be generated
                e = hipMemcpyAsync(rb->host, cn, sizeof(int32_t), hipMemcpyDeviceToHost, st);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(rb->host + 1, chunk_cnt, sizeof(int32_t), hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e != hipSuccess) return e;
                left = rb->host[0];
                gen = rb->host[1];
                if (left == 0 && gen >= total) break;
            }
            if (pass == 0 && sum)
                hipLaunchKernelGGL(k_accum, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, npix, ns, rb->L,
                                   sum, sumsq);
        }
        if (p->nrc_mode == 1) {
            // this chunk's records in path order, their targets, the optimisation
            // steps, new training-path probability
            timed(7, [&] {
                const int64_t stage = kRecStage * p->nrc_train_records;
                const int32_t *n_att = chunk_cnt + ctr(1);
                hipLaunchKernelGGL(k_rec_keys, dim3((unsigned)((stage + 255) / 256)), dim3(256), 0, st, n_att, stage,
                                   (const float *)rb->staged, rb->rkey, rb->rval);
                e = radix_sort(rb->rkey, rb->rval, rb->rkey2, rb->rval2, stage, st);
                if (e == hipSuccess) {
                    hipLaunchKernelGGL(k_rec_gather,
                                       dim3((unsigned)((p->nrc_train_records + 255) / 256)), dim3(256), 0, st, n_att,
                                       (int64_t)p->nrc_train_records, (const int32_t *)rb->rval,
                                       (const float *)rb->staged, rb->rec);
                    e = hipGetLastError();
                }
                if (e == hipSuccess)
                    e = nrc_targets(ctx, p->nrc_train_records, chunk_cnt + ctr(1), rb->rec, rb->L, rb->targets);
                if (e == hipSuccess)
                    e = nrc_train_render(ctx, p->nrc_train_records, chunk_cnt + ctr(1), rb->rec, box, rb->targets,
                                         p->nrc_lr > 0.f ? p->nrc_lr : 1e-2f, std::max(1, p->nrc_train_steps),
                                         p->nrc_target_clamp, rb->loss);
                if (e == hipSuccess) e = nrc_adapt(ctx, chunk_cnt + ctr(1), p->nrc_train_records, rb->frac);
            });
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_nrc_count, dim3(1), dim3(1), 0, st, (const int32_t *)(chunk_cnt + ctr(1)),
                               ctx->stats + 4);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    ctx->last_paths = npix * p->spp;
    ctx->last_nrc_counts = p->nrc_mode == 1 ? (int64_t)kChunkBlock : -1;
    ctx->last_nrc_cap = p->nrc_mode == 1 ? p->nrc_train_records : 0;
    return hipSuccess;
}

const float *render_nrc_loss(ugp_ctx ctx) { return ctx->rb ? ctx->rb->loss : nullptr; }

hipError_t render_nrc_records(ugp_ctx ctx, int64_t cap, float *rec_out, float *tgt_out, int64_t *count) {
    *count = 0;
    RenderBuffers *rb = ctx->rb;
    if (!rb || !rb->nrc_block || ctx->last_nrc_counts < 0) return hipSuccess;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return e;
    int32_t appended = 0;
    e = hipMemcpy(&appended, rb->counts + ctx->last_nrc_counts + ctr(1), sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    int64_t n = std::min<int64_t>((int64_t)appended, ctx->last_nrc_cap);
    n = std::min<int64_t>(n, cap);
    if (n > 0) {
        e = hipMemcpy(rec_out, rb->rec, sizeof(float) * kNrcRecordFloats * (size_t)n, hipMemcpyDeviceToDevice);
        if (e == hipSuccess && tgt_out)
            e = hipMemcpy(tgt_out, rb->targets, sizeof(float) * 3 * (size_t)n, hipMemcpyDeviceToDevice);
        if (e != hipSuccess) return e;
    }
    *count = n;
    return hipSuccess;
}

// Test hook of the SGGX phase functions: per query the records prepared from
// the inputs as the scene pack does, the stochastic estimate, the approximate
// pdf, and an importance sample with its weight and approximate pdf (layout
// in ugp_sggx_phase).
__global__ __launch_bounds__(256) void k_sggx_phase(int64_t n, const float *sggx, const float *base,
                                                    const float *dirs, const float *u, float *out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double g6[6];
        for (int j = 0; j < 6; ++j) g6[j] = sggx[6 * i + j];
        const float *b = base ? base + 5 * i : nullptr;
        const float alb[3] = {b ? b[0] : 1.f, b ? b[1] : 1.f, b ? b[2] : 1.f};
        const float rough = b ? b[3] : 0.5f, met = b ? b[4] : 0.f;
        float4 rec[8];
        float *o = out + 12 * i;
        if (!sggx_prepare_prim(g6, rough, met, alb, rec)) {
            for (int j = 0; j < 12; ++j) o[j] = __builtin_nanf("");
            continue;
        }
        const Sggx g = sggx_load(rec), gr = sggx_load(rec + 4);
        const float *d = dirs + 6 * i, *r = u + 12 * i;
        const V3 wo = v3(d[0], d[1], d[2]), wi = v3(d[3], d[4], d[5]), c = v3(alb[0], alb[1], alb[2]);
        V3 f, ws, w;
        float pf, pw;
        bool ok;
        if (b) {
            f = sggx_disney_est(g, c, rough, wo, wi, r);
            pf = sggx_disney_pdf_approx(gr, g.ps, wo, wi);
            ok = sggx_disney_sample(g, c, rough, wo, r[6], r[7], r[8], r[9], r[10], ws, w);
            pw = ok ? sggx_disney_pdf_approx(gr, g.ps, wo, ws) : 0.f;
        } else {
            const float e = sggx_phase_est(g, wo, wi, r[0], r[1], r[2], r[3]);
            f = v3(e, e, e);
            pf = sggx_pdf_approx(wo, wi);
            ws = sggx_sample(g, wo, r[6], r[7], r[8], r[9]);
            w = v3(1.f, 1.f, 1.f);
            pw = sggx_pdf_approx(wo, ws);
            ok = true;
        }
        if (!ok) ws = w = v3(0.f, 0.f, 0.f);
        o[0] = f.x; o[1] = f.y; o[2] = f.z; o[3] = pf;
        o[4] = ws.x; o[5] = ws.y; o[6] = ws.z;
        o[7] = w.x; o[8] = w.y; o[9] = w.z; o[10] = pw; o[11] = ok ? 1.f : 0.f;
    }
}

hipError_t sggx_phase(ugp_ctx ctx, int64_t n, const float *sggx, const float *base, const float *dirs,
                      const float *u, float *out) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_sggx_phase, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, sggx, base, dirs, u,
                       out);
    return hipGetLastError();
}

}  // namespace ugp
