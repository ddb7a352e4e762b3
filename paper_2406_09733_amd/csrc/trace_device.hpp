// trace_device.hpp -- device side of the scene queries: the ray / primitive
// chord and ray integral, BVH traversal with an LDS stack, transmittance and
// the ordered sweep that implements primitive-level free-flight sampling.
//
// Precision: a primitive record holds M = S^-1 R^T rounded to float.  The ray
// is first moved to a reference point on it near the mean, p_e = (o - mu) +
// t_e w with t_e = -(o - mu).w; the closest-approach step from p_e and
// rho^2 = |M p_m|^2 at the closest point are then taken with FP64 products
// of the float M.  So the float rounding of M moves t_c only by ~1e-7 of the
// primitive's own extent (not of its distance to the ray origin), and the
// 1/s_n amplification of thin primitives never meets float rounding of an
// offset.  Kernel values (erf/erfc/exp) and all sums are FP32.
#pragma once
#include "ugp_internal.hpp"
#include "ugp_math.hpp"

namespace ugp {

constexpr int kBlock = 64;  // one wave64 per block for the traversal kernels

// per-lane traversal counters (always kept in registers; written out only
// when the scene carries a counter buffer, i.e. at profiling level 2)
struct TraceCount {
    uint32_t nodes = 0, prims = 0, reloads = 0, rounds = 0;
};

__device__ inline void flush_counts(const SceneDev &S, const TraceCount &c) {
    if (!S.count) return;
    unsigned long long v[3] = {c.nodes, c.prims, c.reloads};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        unsigned long long x = v[k];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if ((threadIdx.x & 63) == 0) atomicAdd(&S.count[k], x);
    }
}

struct RayD {
    float ox, oy, oz;     // origin
    float dx, dy, dz;     // direction (unit length)
    float t0;             // start of the parameter range
    double t1;            // end of the range (FP64: an emitter query ends at an exact chord exit)
    float idx, idy, idz;  // inverse direction for slab tests
};

__device__ __forceinline__ float safe_inv(float d) {
    const float a = fabsf(d) < 1e-20f ? copysignf(1e-20f, d) : d;
    return 1.f / a;
}

__device__ __forceinline__ RayD make_ray(float ox, float oy, float oz, float dx, float dy, float dz,
                                         float t0, double t1) {
    RayD r;
    r.ox = ox; r.oy = oy; r.oz = oz;
    r.dx = dx; r.dy = dy; r.dz = dz;
    r.t0 = t0; r.t1 = t1;
    r.idx = safe_inv(dx); r.idy = safe_inv(dy); r.idz = safe_inv(dz);
    return r;
}

__device__ __forceinline__ RayD load_ray(const float *rays, int64_t i) {
    const float4 a = reinterpret_cast<const float4 *>(rays)[2 * i];
    const float4 b = reinterpret_cast<const float4 *>(rays)[2 * i + 1];
    return make_ray(a.x, a.y, a.z, a.w, b.x, b.y, b.z, (double)b.w);
}

// Validation of a caller's ray, which only the device sees: a finite origin
// and direction, a direction of length within 1e-3 of 1, a finite t0 and a t1
// that is not NaN (+inf is allowed).  A ray that fails sets kErrRay in the
// error word (ugp_sync reports it as an invalid argument) and the query
// writes NaN (or "no primitive") for it without traversing.
__device__ __forceinline__ bool ray_ok(const RayD &r, uint32_t *err) {
    const bool fin = isfinite(r.ox) && isfinite(r.oy) && isfinite(r.oz) && isfinite(r.dx) && isfinite(r.dy) &&
                     isfinite(r.dz) && isfinite(r.t0) && !isnan(r.t1);
    const double len = sqrt((double)r.dx * r.dx + (double)r.dy * r.dy + (double)r.dz * r.dz);
    const bool ok = fin && fabs(len - 1.0) <= 1e-3;
    if (!ok) atomicOr(err, kErrRay);
    return ok;
}

// ---------------------------------------------------------------------------
// Chord of the cut-off ellipsoid and the closed-form ray integral
// (Sec. 4.1 eqs. ray_integral / cutoff_threshold, App. A).
// In the unit-Gaussian frame o' = M (o - mu), w' = M w:
//   A = w'.w', t_c = -(o'.w')/A, rho^2 = |o'|^2 - (o'.w')^2/A,
//   chord = t_c -/+ sqrt((r^2 - rho^2)/A) clipped to [t0, t1],
//   I(x, y) = d sqrt(pi/(2A)) exp(-rho^2/2) [erf(tau_y) - erf(tau_x)],
//   tau_t = sqrt(A/2) (t - t_c); at an unclipped end |tau| = sqrt((r^2-rho^2)/2).
// ---------------------------------------------------------------------------
struct Chord {
    double tc;     // closest approach
    double bd;     // clipped exit in full precision
    float a, b;    // clipped chord (rounded to float)
    float s;       // sqrt(A/2)
    float pref;    // d sqrt(pi/(2A)) exp(-rho^2/2)
    float ta, tb;  // tau at the clipped ends
    float W;       // 1/2 I(a, b)
    int orig;      // original index
    bool own;      // this reference holds the chord entry (always, for an uncut primitive)
};

__device__ __forceinline__ double rcp_d(double x) {
    double r = (double)(1.0f / (float)x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// erf(tb) - erf(ta) for ta <= tb, as a difference of erfc in the tails
__device__ __forceinline__ float erf_diff(float ta, float tb) {
    if (ta >= 0.f) return erfcf(ta) - erfcf(tb);
    if (tb <= 0.f) return erfcf(-tb) - erfcf(-ta);
    return erff(tb) - erff(ta);
}

// 64-byte primitive record: (mu.xyz, d), (M00 M01 M02 M10), (M11 M12 M20 M21),
// (M22, original index bits, 1/min(s), slab bits) with M = S^-1 R^T in float
struct HotRec {
    float mx, my, mz, d;
    float m[9];
    int orig;
    float mnorm;  // largest row norm of M
    int slab;     // slab index | count << 8 | long axis << 16
};

__device__ __forceinline__ HotRec load_hot(const float4 *hot, int i) {
    const float4 a = hot[4 * i], b = hot[4 * i + 1], c = hot[4 * i + 2], e = hot[4 * i + 3];
    return HotRec{a.x, a.y, a.z, a.w, {b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w, e.x}, __float_as_int(e.y), e.z,
                  __float_as_int(e.w)};
}

// Cheap float test that the ray surely misses the cut-off ellipsoid: the
// distance of closest approach in the unit frame is computed in float and
// compared with r plus a bound on its rounding error (offsets in float carry
// ~1e-6 of |o - mu|, magnified at most mnorm-fold by M).  Only candidates
// that survive take the FP64 path of chord().
__device__ __forceinline__ bool surely_missed(const HotRec &h, const RayD &r, float r2) {
    const float *M = h.m;
    const float ex = r.ox - h.mx, ey = r.oy - h.my, ez = r.oz - h.mz;
    const float te = -(ex * r.dx + ey * r.dy + ez * r.dz);
    const float px = fmaf(te, r.dx, ex), py = fmaf(te, r.dy, ey), pz = fmaf(te, r.dz, ez);
    const float w0 = M[0] * r.dx + M[1] * r.dy + M[2] * r.dz;
    const float w1 = M[3] * r.dx + M[4] * r.dy + M[5] * r.dz;
    const float w2 = M[6] * r.dx + M[7] * r.dy + M[8] * r.dz;
    const float q0 = M[0] * px + M[1] * py + M[2] * pz;
    const float q1 = M[3] * px + M[4] * py + M[5] * pz;
    const float q2 = M[6] * px + M[7] * py + M[8] * pz;
    const float A = w0 * w0 + w1 * w1 + w2 * w2;
    const float dt = -(q0 * w0 + q1 * w1 + q2 * w2) / A;
    const float u0 = fmaf(dt, w0, q0), u1 = fmaf(dt, w1, q1), u2 = fmaf(dt, w2, q2);
    const float rho = sqrtf(u0 * u0 + u1 * u1 + u2 * u2);
    const float err = 2e-6f * h.mnorm * (fabsf(ex) + fabsf(ey) + fabsf(ez)) +
                      2e-5f * (1.f + fabsf(q0) + fabsf(q1) + fabsf(q2));
    return rho > sqrtf(r2) + err;
}

// Returns false if the clipped chord is empty.
__device__ inline bool chord(const HotRec &h, const RayD &r, float r2, Chord &c, bool screened = false) {
    if (!screened && surely_missed(h, r, r2)) return false;
    const float *M = h.m;
    // reference point on the ray near mu: p_e = (o - mu) + t_e w, FP64
    const double dx = r.dx, dy = r.dy, dz = r.dz;
    const double ex = (double)r.ox - (double)h.mx, ey = (double)r.oy - (double)h.my,
                 ez = (double)r.oz - (double)h.mz;
    const double te = -(ex * dx + ey * dy + ez * dz);
    const double px = fma(te, dx, ex), py = fma(te, dy, ey), pz = fma(te, dz, ez);
    // unit-frame offset q = M p_e and direction w' = M w (FP64 products of the
    // float M: the normal row of a thin primitive amplifies rounding 1/s_n-fold)
    const double m0 = M[0], m1 = M[1], m2 = M[2], m3 = M[3], m4 = M[4], m5 = M[5], m6 = M[6],
                 m7 = M[7], m8 = M[8];
    const double w0 = m0 * dx + m1 * dy + m2 * dz;
    const double w1 = m3 * dx + m4 * dy + m5 * dz;
    const double w2 = m6 * dx + m7 * dy + m8 * dz;
    const double q0 = m0 * px + m1 * py + m2 * pz;
    const double q1 = m3 * px + m4 * py + m5 * pz;
    const double q2 = m6 * px + m7 * py + m8 * pz;
    const double A = w0 * w0 + w1 * w1 + w2 * w2;
    if (!(A > 0.0)) return false;
    // closest approach t_c = t_e + dt; rho^2 = |q + dt w'|^2
    const double dt = -(q0 * w0 + q1 * w1 + q2 * w2) * rcp_d(A);
    const double u0 = fma(dt, w0, q0), u1 = fma(dt, w1, q1), u2 = fma(dt, w2, q2);
    const float rho2f = (float)(u0 * u0 + u1 * u1 + u2 * u2);
    if (!(rho2f < r2)) return false;
    const float Af = (float)A;
    const double tc = te + dt;
    const float half = sqrtf((r2 - rho2f) / Af);
    const double tlo = tc - (double)half, thi = tc + (double)half;
    const double a = fmax((double)r.t0, tlo), b = fmin(r.t1, thi);
    if (!(a < b)) return false;
    const float s = sqrtf(0.5f * Af);
    const float taumax = sqrtf(0.5f * (r2 - rho2f));
    c.tc = tc;
    c.bd = b;
    c.s = s;
    c.ta = (a > tlo) ? fmaxf(s * (float)(a - tc), -taumax) : -taumax;
    c.tb = (b < thi) ? fminf(s * (float)(b - tc), taumax) : taumax;
    c.pref = h.d * (0.886226925452758f / s) * expf(-0.5f * rho2f);
    c.a = (float)a;
    c.b = (float)b;
    c.W = 0.5f * c.pref * erf_diff(c.ta, c.tb);
    c.orig = h.orig;
    // a cut primitive is reported by the slab holding the chord entry: the
    // long-axis coordinate of x(a) in the unit frame, q + (a - t_e) w', in
    // m equal slabs of [-r, r]
    const int m = (h.slab >> 8) & 255;
    c.own = true;
    if (m > 1) {
        const int L = h.slab >> 16;
        const double qL = L == 0 ? q0 : (L == 1 ? q1 : q2);
        const double wL = L == 0 ? w0 : (L == 1 ? w1 : w2);
        const double rr = (double)sqrtf(r2);
        const double v = fma(a - te, wL, qL);
        int own = (int)floor((v + rr) * (double)m / (2.0 * rr));
        own = own < 0 ? 0 : (own >= m ? m - 1 : own);
        c.own = own == (h.slab & 255);
    }
    return true;
}

// tau at a point t inside [a, b] (clamped to the chord ends)
__device__ __forceinline__ float tau_at(const Chord &c, double t) {
    if (t <= (double)c.a) return c.ta;
    if (t >= (double)c.b) return c.tb;
    return fminf(fmaxf(c.s * (float)(t - c.tc), c.ta), c.tb);
}
// 1/2 I(a, min(b, t))
__device__ __forceinline__ float half_integral_to(const Chord &c, double t) {
    if (t <= (double)c.a) return 0.f;
    if (t >= (double)c.b) return c.W;
    return 0.5f * c.pref * erf_diff(c.ta, tau_at(c, t));
}
// 1/2 G(x(t)) inside the chord: the free-flight pdf contribution (eq. free_flight_pdf)
__device__ __forceinline__ float half_kernel_at(const Chord &c, double t) {
    if (t <= (double)c.a || t >= (double)c.b) return 0.f;
    const float tau = c.s * (float)(t - c.tc);
    return 0.5f * c.pref * c.s * 1.1283791670955126f * expf(-tau * tau);
}

// ---------------------------------------------------------------------------
// BVH traversal: near child first, the far one on a per-lane LDS stack
// (column `lane` of a [kStackSize][kBlock] int array).  Leaf children are
// handled in their parent.  `leaf(prim)` returns true to stop the traversal;
// `hi()` is re-read after leaves so a shrinking upper bound culls at once.
// ---------------------------------------------------------------------------
// slab test of one box against the ray on [lo, hi]: entry distance or +inf
//
// The plane at coordinate x is crossed at t = (x - o) / d, taken as
// fma(x, 1/d, c) with c = -o/d.  Rounding c costs at most half an ulp of
// |o/d|; the per-ray constants move c outwards by 2^-22 |o/d| (the plane of
// the low corner is the entry when 1/d > 0, the exit otherwise), so a slab
// interval never shrinks below the exact one.
struct SlabC {
    float lx, hx, ly, hy, lz, hz;
};

__device__ __forceinline__ SlabC slab_consts(const RayD &r) {
    SlabC k;
    auto one = [](float o, float inv, float &cl, float &ch) __attribute__((always_inline)) {
        const float c = -o * inv, m = 2.384185791e-7f * fabsf(c);
        cl = inv >= 0.f ? c - m : c + m;
        ch = inv >= 0.f ? c + m : c - m;
    };
    one(r.ox, r.idx, k.lx, k.hx);
    one(r.oy, r.idy, k.ly, k.hy);
    one(r.oz, r.idz, k.lz, k.hz);
    return k;
}

__device__ __forceinline__ float slab(float lx, float ly, float lz, float hx, float hy, float hz,
                                      const RayD &r, const SlabC &k, float lo, float hi) {
    const float ax = fmaf(lx, r.idx, k.lx), bx = fmaf(hx, r.idx, k.hx);
    const float ay = fmaf(ly, r.idy, k.ly), by = fmaf(hy, r.idy, k.hy);
    const float az = fmaf(lz, r.idz, k.lz), bz = fmaf(hz, r.idz, k.hz);
    const float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), lo));
    const float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), hi));
    return (tn <= tf + 5e-7f * fmaxf(fabsf(tn), fabsf(tf))) ? tn : kInf;
}

__device__ __forceinline__ void cswap(float &ta, int &ra, float &tb, int &rb) {
    const bool s = tb < ta;
    const float t = s ? tb : ta;
    tb = s ? ta : tb;
    ta = t;
    const int r = s ? rb : ra;
    rb = s ? ra : rb;
    ra = r;
}

// 4-wide BVH traversal: the children of a node are tested together and
// visited nearest first; farther internal children go on a per-lane LDS stack
// (column `lane` of a [kStackSize][kBlock] int array).  Leaf children are not
// tested where they are found: they are queued per lane (LDS, up to kPend)
// and the lanes test their queued leaves together, after every lane of the
// wave has found leaves or run out of nodes (a lane with leaves queued keeps
// descending meanwhile) -- so the long leaf code runs with most lanes active.
// The queued leaves first go through the cheap screen `pre(prim)` (record
// fetch and float reject test); only the survivors, compacted in the queue,
// reach `leaf(prim)` (the exact chord and the caller's bookkeeping), which
// returns true to stop the traversal.  `hi()` is re-read before every node
// test so a shrinking bound culls as soon as leaves were tested.
//
// A traversal can be suspended: after a leaf phase, when at most
// `suspend_at` lanes of the wave still have nodes to visit, those lanes save
// their position (TravState; the stack stays in the lane's LDS column and
// `spill`) and return kTravSuspended, so the caller can give the idle lanes
// new rays; the next call with the same state resumes the walk.  The set of
// leaves a traversal reaches does not depend on where it was suspended.
constexpr int kPend = 12;

struct TravState {
    int ref;     // next node to visit
    int sp;      // stack depth
    bool nodes;  // `ref` is still to be visited
};

__device__ __forceinline__ void trav_begin(TravState &ts, const SceneDev &S) {
    ts.ref = S.root;
    ts.sp = 0;
    ts.nodes = true;
}

enum : int { kTravDone = 0, kTravStopped = 1, kTravSuspended = 2 };

template <class PreFn, class LeafFn, class HiFn>
__device__ __forceinline__ int traverse(const SceneDev &S, const RayD &r, float lo, HiFn &&hi, int *stack,
                                        int *spill, TravState &ts, int suspend_at, uint32_t *err,
                                        TraceCount &tc, PreFn &&pre, LeafFn &&leaf) {
    const int lane = threadIdx.x;
    int ref = ts.ref;
    if (ref < 0) {  // a tree of one primitive
        ts.nodes = false;
        ++tc.prims;
        return pre(~ref) && leaf(~ref) ? kTravStopped : kTravDone;
    }
    __shared__ int pend[kPend * kBlock];
    const SlabC kc = slab_consts(r);
    int np = 0;             // queued leaves of this lane
    bool nodes = ts.nodes;  // this lane still has a node to visit (ref)
    int sp = ts.sp;
    // the stack lives in LDS; deeper entries (a 4-wide node can push three)
    // spill to private memory, which is only touched in that rare case
    auto push = [&](int v) __attribute__((always_inline)) {
        if (sp < kStackSize) stack[sp * kBlock + lane] = v;
        else if (sp < kStackSize + kStackSpill) spill[sp - kStackSize] = v;
        else { atomicOr(err, kErrStack); return; }
        ++sp;
    };
    for (;;) {
        // descend while there is room for one more node's leaves
        while (nodes && np <= kPend - 4) {
            ++tc.nodes;
            const float4 *nd = S.nodes + 8 * (int64_t)ref;
            const float4 lx = nd[0], ly = nd[1], lz = nd[2], hx = nd[3], hy = nd[4], hz = nd[5], rf = nd[6];
            const float h0 = hi();
            float t0 = slab(lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, r, kc, lo, h0);
            float t1 = slab(lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, r, kc, lo, h0);
            float t2 = slab(lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, r, kc, lo, h0);
            float t3 = slab(lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, r, kc, lo, h0);
            int r0 = __float_as_int(rf.x), r1 = __float_as_int(rf.y), r2 = __float_as_int(rf.z),
                r3 = __float_as_int(rf.w);
            // unused slots carry an inverted box, which a slab test would take as
            // unbounded: mask them by their ref
            t0 = r0 == kEmptySlot ? kInf : t0;
            t1 = r1 == kEmptySlot ? kInf : t1;
            t2 = r2 == kEmptySlot ? kInf : t2;
            t3 = r3 == kEmptySlot ? kInf : t3;
            // sort the four (entry, ref) pairs by entry distance (misses are +inf)
            cswap(t0, r0, t1, r1);
            cswap(t2, r2, t3, r3);
            cswap(t0, r0, t2, r2);
            cswap(t1, r1, t3, r3);
            cswap(t1, r1, t2, r2);
            // queue the leaf children, nearest first
            if (t0 < kInf && r0 < 0) pend[(np++) * kBlock + lane] = ~r0;
            if (t1 < kInf && r1 < 0) pend[(np++) * kBlock + lane] = ~r1;
            if (t2 < kInf && r2 < 0) pend[(np++) * kBlock + lane] = ~r2;
            if (t3 < kInf && r3 < 0) pend[(np++) * kBlock + lane] = ~r3;
            // internal children within the bound (a miss is +inf and must
            // stay a miss when the bound itself is +inf)
            const float lim = h0 + 5e-7f * fabsf(h0);
            const bool g0 = t0 < kInf && t0 <= lim && r0 >= 0, g1 = t1 < kInf && t1 <= lim && r1 >= 0,
                       g2 = t2 < kInf && t2 <= lim && r2 >= 0, g3 = t3 < kInf && t3 <= lim && r3 >= 0;
            // push the farther ones (farthest first), descend into the nearest
            int next = -1;
            if (g3) next = r3;
            if (g2) { if (next >= 0) push(next); next = r2; }
            if (g1) { if (next >= 0) push(next); next = r1; }
            if (g0) { if (next >= 0) push(next); next = r0; }
            if (next >= 0) {
                ref = next;
            } else if (sp == 0) {
                nodes = false;
            } else {
                --sp;
                ref = sp < kStackSize ? stack[sp * kBlock + lane] : spill[sp - kStackSize];
            }
            // leaves are tested once every lane has some queued (or no nodes left)
            if (__all(np > 0 || !nodes)) break;
        }
        // screen the queued leaves, keep the survivors in order, then test them
        int ns = 0;
        for (int q = 0; q < np; ++q) {
            ++tc.prims;
            const int p = pend[q * kBlock + lane];
            if (pre(p)) pend[(ns++) * kBlock + lane] = p;
        }
        for (int q = 0; q < ns; ++q) {
            ++tc.reloads;  // the survivor's record is read again (from cache, normally)
            if (leaf(pend[q * kBlock + lane])) return kTravStopped;
        }
        np = 0;
        if (!nodes) {
            ts.nodes = false;
            return kTravDone;
        }
        if (__popcll(__ballot(1)) <= suspend_at) {
            ts.ref = ref;
            ts.sp = sp;
            return kTravSuspended;
        }
    }
}

// ---------------------------------------------------------------------------
// Transmittance (Sec. 4 eq. transmittance, Sec. 5.3): F = 1/2 sum I_k over
// clipped chords, deterministic; with early_out the traversal stops once
// F >= 1 (T = 0 from then on).
// ---------------------------------------------------------------------------
__device__ inline float transmittance_F(const SceneDev &S, const RayD &r, int excl, bool early_out,
                                        int *stack, uint32_t *err, TraceCount &tc) {
    float F = 0.f;
    const float lo = r.t0;
    const float hi1 = r.t1 < 3.0e38 ? (float)r.t1 : kInf;
    int spill[kStackSpill];
    TravState ts;
    trav_begin(ts, S);
    traverse(S, r, lo, [&]() __attribute__((always_inline)) { return hi1; }, stack, spill, ts, 0, err, tc,
             [&](int p) __attribute__((always_inline)) {
        const HotRec h = load_hot(S.hot, p);
        return h.orig != excl && !surely_missed(h, r, S.r2);
    },
             [&](int p) __attribute__((always_inline)) {
        const HotRec h = load_hot(S.hot, p);
        Chord c;
        if (!chord(h, r, S.r2, c, true) || !c.own) return false;
        F += c.W;
        return early_out && F >= 1.f;
    });
    return F;
}

// ---------------------------------------------------------------------------
// Exponential variant (App. D; eq. exp_ff): the same Gaussians read as a
// heterogeneous exponential medium with sigma_t = sum_k G_k.
//
// Optical depth of a ray: the sum of the ray integrals I_k = pref [erf tau_b -
// erf tau_a] of the clipped chords (the full integral; the linear model's
// free-flight weight is half of it).
// ---------------------------------------------------------------------------
__device__ inline float exp_depth(const SceneDev &S, const RayD &r, int excl, int *stack, uint32_t *err,
                                  TraceCount &tc) {
    const float hi = r.t1 < 3.0e38 ? (float)r.t1 : kInf;
    int spill[kStackSpill];
    TravState ts;
    trav_begin(ts, S);
    float depth = 0.f;
    traverse(S, r, r.t0, [&]() __attribute__((always_inline)) { return hi; }, stack, spill, ts, 0, err, tc,
             [&](int p) __attribute__((always_inline)) {
                 const HotRec h = load_hot(S.hot, p);
                 return h.orig != excl && !surely_missed(h, r, S.r2);
             },
             [&](int p) __attribute__((always_inline)) {
                 const HotRec h = load_hot(S.hot, p);
                 Chord c;
                 if (chord(h, r, S.r2, c, true) && c.own) depth += 2.f * c.W;
                 return false;
             });
    return depth;
}

// Analog decomposition tracking (App. D, after Kutz et al. 2017): each
// Gaussian k the ray meets draws y_k = -ln(1 - u_k) (u_k = uni(k), k the
// original index) and collides where its optical depth from the chord entry
// reaches y_k, if it does before the chord exit; the nearest such point wins.
// The inverse of the erf closed form is taken in FP64, through erfc in the
// tails.  The traversal is cut at the nearest collision found so far.
// Returns the original index (or -1, escape) and its distance in t.
template <class UniFn>
__device__ inline int exp_track(const SceneDev &S, const RayD &r, int excl, UniFn &&uni, int *stack, uint32_t *err,
                                TraceCount &tc, double &t) {
    const float t1f = r.t1 < 3.0e38 ? (float)r.t1 : kInf;
    int spill[kStackSpill];
    TravState ts;
    trav_begin(ts, S);
    double best = __builtin_huge_val();
    int bk = -1;
    traverse(S, r, r.t0, [&]() __attribute__((always_inline)) { return fminf(t1f, (float)best); }, stack, spill,
             ts, 0, err, tc,
             [&](int p) __attribute__((always_inline)) {
                 const HotRec h = load_hot(S.hot, p);
                 return h.orig != excl && !surely_missed(h, r, S.r2);
             },
             [&](int p) __attribute__((always_inline)) {
                 const HotRec h = load_hot(S.hot, p);
                 Chord c;
                 if (!chord(h, r, S.r2, c, true) || !c.own || !((double)c.a < best)) return false;
                 const double y = -log1p(-uni(h.orig));
                 const double pref = c.pref, ta = c.ta, tb = c.tb;
                 // I(a, t) = pref [erf tau(t) - erf ta]; collide if y < I(a, b)
                 double tau;
                 if (ta >= 0.0) {
                     const double q = erfc(ta) - y / pref;  // erfc tau
                     if (!(q > erfc(tb))) return false;
                     tau = erfcinv(q);
                 } else {
                     const double e = erf(ta) + y / pref;   // erf tau
                     if (!(e < erf(tb))) return false;
                     tau = e <= 0.0 ? -erfcinv(1.0 + e) : erfcinv(1.0 - e);
                 }
                 const double tk = c.tc + tau / (double)c.s;
                 if (tk < best) {
                     best = tk;
                     bk = h.orig;
                 }
                 return false;
             });
    t = best;
    return bk;
}

// ---------------------------------------------------------------------------
// Ordered sweep: primitive-level free-flight sampling (Sec. 5.2), the
// saturating distance and the emitter query.
//
// The canonical rule (tree independent): with t_sat the smallest t where
// F(t) = 1/2 sum_k I_k(a_k, min(b_k, t)) reaches 1 (t1 if never), primitive k
// has weight W_k = 1/2 I_k(a_k, min(b_k, t_sat)); they are ordered by
// (min(b_k, t_sat), k) and u selects the first k whose running sum exceeds it.
//
// The BVH has overlapping nodes, so the sweep works in windows.  A round
// traverses the tree and keeps, in a register-resident buffer sorted by
// entry key (a_k, k), the smallest entries above the previous round's bound;
// when the buffer is full the largest is evicted and its key becomes the cap,
// so every primitive entering before the cap is known.  The window
// [t_cur, cap] is then exact:
//   - an upper bound S + sum W (no saturation possible below 1) usually
//     finalises the window without touching partial integrals;
//   - otherwise F(cap) is evaluated exactly, and if it reaches 1 t_sat is
//     solved by a bracketed Newton iteration (dF/dt = 1/2 sum G_k,
//     eq. sampling_overlaps), the exits before t_sat are finalised in exit
//     order and the straddlers follow by index with clipped weights.
// Primitives still active at the cap stay in the buffer for the next round.
// During a round the traversal is also cut at a saturation bound: F(t) is at
// least the finalised weight plus the full weights of buffered primitives
// that exit by t, so once that sum passes 1 at the exit b of a newly buffered
// primitive, t_sat <= b and nothing entering after b can carry weight (all
// primitives entering before b are still gathered, so the round then
// saturates with F exact on [t_cur, b]).
// ---------------------------------------------------------------------------
struct Ev {
    float a, b, w;
    int id;  // original index
};

__device__ __forceinline__ bool key_less(float a1, int i1, float a2, int i2) {
    return a1 < a2 || (a1 == a2 && i1 < i2);
}

struct SweepOut {
    int prim;      // collide: selected original index or -1
    float t;       // collide: scatter distance; saturate: t_sat; emitter: factor
    int status;    // 0 ok, 1 event-buffer overflow
    double td;     // saturate: t_sat in full precision
};

// loops over the event buffer are unrolled (register arrays) only for small K
template <int K>
struct Unr {
    static constexpr int v = K <= 16 ? K : 1;
};

// A wide buffer (K > 16, in private memory) also keeps each entry's chord,
// so the saturation solve and the final walks read it back instead of
// re-deriving it from the primitive's record; the register buffer does not.
template <int K, bool kKeep = (K > 16)>
struct EvChords {
    __device__ __forceinline__ void move(int, int) {}
};
template <int K>
struct EvChords<K, true> {
    double tc[K];
    float s[K], pref[K], ta[K], tb[K];
    __device__ __forceinline__ void move(int d, int f) {
        tc[d] = tc[f]; s[d] = s[f]; pref[d] = pref[f]; ta[d] = ta[f]; tb[d] = tb[f];
    }
    __device__ __forceinline__ void put(int i, const Chord &c) {
        tc[i] = c.tc; s[i] = c.s; pref[i] = c.pref; ta[i] = c.ta; tb[i] = c.tb;
    }
};

// Event buffer as a structure of arrays; fields are copied one by one (a
// whole-struct copy becomes a memcpy that keeps the buffer out of registers).
template <int K>
struct EvBuf {
    float a[K], b[K], w[K];
    int id[K];
    int n;
    EvChords<K> ch;
    __device__ __forceinline__ void move(int dst, int src) {
        a[dst] = a[src]; b[dst] = b[src]; w[dst] = w[src]; id[dst] = id[src];
        ch.move(dst, src);
    }
};

// original index of event j (dynamic j).  For register arrays this is an OR
// over masked entries: a select of entries would be folded back into an
// indexed load and force the buffer into scratch memory.
template <int K>
__device__ __forceinline__ int ev_id(const EvBuf<K> &B, int j) {
    if constexpr (K > 16) {
        return B.id[j];
    } else {
        int r = 0;
#pragma unroll
        for (int i = 0; i < K; ++i) r |= (i == j) ? B.id[i] : 0;
        return r;
    }
}

// re-derive the chord of an event (bit-identical to the traversal's test)
__device__ __forceinline__ Chord ev_chord(const SceneDev &S, const RayD &r, int orig, TraceCount &tc) {
    ++tc.reloads;
    const HotRec h = load_hot(S.hot, S.inv[orig]);
    Chord c;
    c.a = c.b = 0.f;
    c.W = 0.f;
    chord(h, r, S.r2, c);
    return c;
}

// Chords of up to kChordCache buffered primitives that may straddle the
// saturation point are kept in LDS (two float4 per chord, column = lane)
// while t_sat is solved, so the Newton steps do not re-read their records.
constexpr int kChordCache = 4;

struct ChordCache {
    float4 *base;    // [kChordCache * 2][kBlock]
    uint64_t mask;   // buffer entries held (slot = rank among the set bits)
};

__device__ __forceinline__ void cache_put(ChordCache &cc, int slot, const Chord &c) {
    const int lane = threadIdx.x & (kBlock - 1);
    cc.base[(2 * slot) * kBlock + lane] =
        make_float4(__int_as_float(__double2loint(c.tc)), __int_as_float(__double2hiint(c.tc)), c.s, c.pref);
    cc.base[(2 * slot + 1) * kBlock + lane] = make_float4(c.ta, c.tb, c.a, c.b);
}

__device__ __forceinline__ Chord cache_get_slot(const ChordCache &cc, int slot) {
    const int lane = threadIdx.x & (kBlock - 1);
    const float4 x = cc.base[(2 * slot) * kBlock + lane], y = cc.base[(2 * slot + 1) * kBlock + lane];
    Chord c;
    c.tc = __hiloint2double(__float_as_int(x.y), __float_as_int(x.x));
    c.s = x.z;
    c.pref = x.w;
    c.ta = y.x;
    c.tb = y.y;
    c.a = y.z;
    c.b = y.w;
    c.bd = (double)y.w;
    c.W = 0.f;  // not kept: cached chords are only evaluated strictly inside (a, b)
    c.orig = -1;
    c.own = true;
    return c;
}

__device__ __forceinline__ Chord cache_get(const ChordCache &cc, int j) {
    return cache_get_slot(cc, __popcll(cc.mask & ((1ull << j) - 1ull)));
}

// chord of buffer entry j: kept in a wide buffer; from the cache when held,
// else re-derived
template <int K>
__device__ __forceinline__ Chord ev_chord_c(const SceneDev &S, const RayD &r, const EvBuf<K> &B, int j,
                                           const ChordCache *cc, TraceCount &tc) {
    if constexpr (K > 16) {
        Chord c;
        c.tc = B.ch.tc[j];
        c.s = B.ch.s[j];
        c.pref = B.ch.pref[j];
        c.ta = B.ch.ta[j];
        c.tb = B.ch.tb[j];
        c.a = B.a[j];
        c.b = B.b[j];
        c.bd = (double)B.b[j];
        c.W = B.w[j];
        c.orig = B.id[j];
        c.own = true;
        return c;
    } else {
        if (cc && ((cc->mask >> j) & 1ull)) return cache_get(*cc, j);
        return ev_chord(S, r, ev_id(B, j), tc);
    }
}

// F(t) and F'(t) over the buffer: S_fin + sum of (full weights of exits <= t,
// partial weights of entries before t that exit later)
template <int K>
__device__ __forceinline__ float sweep_F(const SceneDev &S, const RayD &r, const EvBuf<K> &B, float S_fin,
                                double t, float *dF, TraceCount &tc, const ChordCache *cc = nullptr) {
    float F = S_fin, G = 0.f;
    uint64_t partial = 0;
#pragma unroll Unr<K>::v
    for (int i = 0; i < K; ++i) {
        if (i < B.n) {
            if ((double)B.b[i] <= t) F += B.w[i];
            else if ((double)B.a[i] < t) partial |= 1ull << i;
        }
    }
    while (partial) {
        const int j = __builtin_ctzll(partial);
        partial &= partial - 1;
        const Chord c = ev_chord_c(S, r, B, j, cc, tc);
        F += half_integral_to(c, t);
        G += half_kernel_at(c, t);
    }
    if (dF) *dF = G;
    return F;
}

// State of one ray's sweep between rounds.
template <int K>
struct SweepState {
    EvBuf<K> B;
    float S_fin;     // finalised weight (exits before t_cur)
    double t_cur;
    float lb_a;      // entries with key <= (lb_a, lb_id) were seen
    int lb_id;
    int round;
    // the round in progress (its traversal may be suspended)
    bool in_round;
    float cap_a;     // key of the first evicted entry: the window ends there
    int cap_id;
    float cap_sat;   // saturation bound: t_sat <= cap_sat
    bool evicted, hidden;
    int n_before;    // buffered entries when the round began
    float wbuf;      // K > 16: sum of the buffered full weights (kept up to date)
    TravState ts;
};

template <int K>
__device__ __forceinline__ void sweep_start(SweepState<K> &st, SweepOut &out, const RayD &r, int mode) {
    out = SweepOut{-1, __builtin_nanf(""), 0};
    if (mode == kModeSaturate) {
        out.t = (float)r.t1;
        out.td = r.t1;
    }
    if (mode == kModeEmitter) out.t = 0.f;
    st.B.n = 0;
    st.wbuf = 0.f;
    st.S_fin = 0.f;
    st.t_cur = r.t0;
    st.lb_a = -kInf;
    st.lb_id = -1;
    st.round = 0;
    st.in_round = false;
}

// One round of the sweep: gather, then finalise the window (or solve the
// saturation inside it).  Returns true when the ray is done and `out` holds
// its result, false when another round is needed or the round's traversal
// was suspended (suspend_at > 0; the next call resumes it).
// stop_a (emitter mode): the target's chord entry; once a saturation bound
// falls at or before it the target is hidden (weight 0) and the sweep ends.
template <int K>
__device__ __forceinline__ bool sweep_round(const SceneDev &S, const RayD &r, int excl, int mode, float u,
                                            int target, float stop_a, SweepState<K> &st, SweepOut &out,
                                            int *stack, int *spill, int suspend_at, uint32_t *err,
                                            TraceCount &tc) {
    EvBuf<K> &B = st.B;
    float &S_fin = st.S_fin;
    double &t_cur = st.t_cur;
    float &lb_a = st.lb_a;
    int &lb_id = st.lb_id;
    const float t1f = r.t1 < 3.0e38 ? (float)r.t1 : kInf;
    float &cap_a = st.cap_a;
    int &cap_id = st.cap_id;
    float &cap_sat = st.cap_sat;
    bool &evicted = st.evicted, &hidden = st.hidden;
    if (!st.in_round) {
        if (st.round++ >= 4096) {
            out.status = 1;
            return true;
        }
        ++tc.rounds;
        cap_a = kInf;
        cap_id = 0x7fffffff;
        cap_sat = kInf;
        evicted = hidden = false;
        st.n_before = B.n;
        trav_begin(st.ts, S);
        st.in_round = true;
    }
    {
        const int n_before = st.n_before;
        const int tr = traverse(S, r, fmaxf(r.t0, lb_a),
                 [&]() __attribute__((always_inline)) { return fminf(fminf(cap_a, cap_sat), t1f); },
                 stack, spill, st.ts, suspend_at, err, tc,
                 [&](int p) __attribute__((always_inline)) {
                     const HotRec h = load_hot(S.hot, p);
                     return h.orig != excl && !surely_missed(h, r, S.r2);
                 },
                 [&](int p) __attribute__((always_inline)) {
                     const HotRec h = load_hot(S.hot, p);
                     Chord c;
                     if (!chord(h, r, S.r2, c, true) || !c.own) return false;
                     if (key_less(c.a, c.orig, lb_a, lb_id)) return false;    // seen before
                     if (!key_less(c.a, c.orig, cap_a, cap_id)) return false; // beyond cap
                     if (c.a > cap_sat) return false;                          // past saturation
                     float xa = c.a, xb = c.b, xw = c.W;
                     int xi = c.orig;
                     bool placed = false;
                     if constexpr (K > 16) {
                         // the buffer is in private memory: binary search for
                         // the slot, then shift the (usually short) tail up;
                         // entries arrive near-first, so mostly near the end
                         int lo = 0, hi = B.n;
                         while (lo < hi) {
                             const int mid = (lo + hi) >> 1;
                             if (key_less(B.a[mid], B.id[mid], xa, xi)) lo = mid + 1;
                             else hi = mid;
                         }
                         if (lo < K) {
                             const int last = B.n < K ? B.n : K - 1;
                             if (B.n == K) {  // the largest buffered entry leaves
                                 xa = B.a[K - 1]; xb = B.b[K - 1]; xw = B.w[K - 1]; xi = B.id[K - 1];
                                 st.wbuf -= xw;
                             } else {
                                 placed = true;
                             }
                             for (int i = last; i > lo; --i) B.move(i, i - 1);
                             B.a[lo] = c.a; B.b[lo] = c.b; B.w[lo] = c.W; B.id[lo] = c.orig;
                             B.ch.put(lo, c);
                             st.wbuf += c.W;
                         }
                     } else {
#pragma unroll Unr<K>::v
                     for (int i = 0; i < K; ++i) {
                         if (i < B.n) {
                             if (key_less(xa, xi, B.a[i], B.id[i])) {
                                 const float ta = B.a[i], tb = B.b[i], tw = B.w[i];
                                 const int ti = B.id[i];
                                 B.a[i] = xa; B.b[i] = xb; B.w[i] = xw; B.id[i] = xi;
                                 xa = ta; xb = tb; xw = tw; xi = ti;
                             }
                         } else if (!placed) {
                             B.a[i] = xa; B.b[i] = xb; B.w[i] = xw; B.id[i] = xi;
                             placed = true;
                         }
                     }
                     }
                     if (placed) {
                         ++B.n;
                     } else {  // x is the largest of K + 1: evict it
                         evicted = true;
                         cap_a = xa;
                         cap_id = xi;
                     }
                     // (wide buffer: skip the scan while all buffered weight
                     // together, an upper bound of the sum below, is short of 1)
                     if (c.b < cap_sat && key_less(c.a, c.orig, cap_a, cap_id) &&
                         (K <= 16 || S_fin + st.wbuf >= 1.f)) {
                         // the new primitive is buffered: lower bound of F(c.b)
                         float lo_F = S_fin;
#pragma unroll Unr<K>::v
                         for (int i = 0; i < K; ++i)
                             if (i < B.n && B.b[i] <= c.b) lo_F += B.w[i];
                         // margin: the exact F(b) sums the same terms in another order
                         if (lo_F >= 1.0001f) {
                             cap_sat = c.b;
                             if (cap_sat <= stop_a) {
                                 hidden = true;  // t_sat < entry of the target
                                 return true;
                             }
                         }
                     }
                     return false;
                 });
        if (tr == kTravSuspended) return false;
        st.in_round = false;
        if (hidden) return true;
        // window end: every primitive entering before t_w is in the buffer
        const double t_w = evicted ? (double)cap_a : r.t1;
        // progress check: nothing new and nothing can exit -> overflow
        // upper bound on F(t_w)
        float U = S_fin;
#pragma unroll Unr<K>::v
        for (int i = 0; i < K; ++i)
            if (i < B.n && (double)B.a[i] < t_w) U += B.w[i];
        bool saturated = false;
        if (U >= 1.f) {
            const float Fw = sweep_F<K>(S, r, B, S_fin, t_w, nullptr, tc);
            saturated = Fw >= 1.f;
        }
        if (!saturated) {
            // finalise exits inside the window (all of them if the ray is complete)
            float T = S_fin;
            uint64_t fin = 0;
#pragma unroll Unr<K>::v
            for (int i = 0; i < K; ++i)
                if (i < B.n && (!evicted || (double)B.b[i] <= t_w)) {
                    T += B.w[i];
                    fin |= 1ull << i;
                }
            if (mode == kModeCollide && T > u) {
                // walk the finalised exits in (b, id) order
                float run = S_fin, pb = -kInf;
                int pid = -1;
                for (int step = 0; step < K; ++step) {
                    float bb = kInf, bw = 0.f, ba = 0.f;
                    int bid = 0x7fffffff, bi = -1;
#pragma unroll Unr<K>::v
                    for (int i = 0; i < K; ++i)
                        if ((fin >> i) & 1ull) {
                            if (key_less(pb, pid, B.b[i], B.id[i]) && key_less(B.b[i], B.id[i], bb, bid)) {
                                bb = B.b[i]; bid = B.id[i]; bw = B.w[i]; ba = B.a[i]; bi = i;
                            }
                        }
                    if (bi < 0) break;
                    run += bw;
                    out.prim = bid;
                    out.t = 0.5f * (ba + bb);
                    if (run > u) break;
                    pb = bb;
                    pid = bid;
                }
                return true;
            }
            if (mode == kModeEmitter) {
#pragma unroll Unr<K>::v
                for (int i = 0; i < K; ++i)
                    if (((fin >> i) & 1ull) && B.id[i] == target) out.t = B.w[i];
            }
            if (!evicted) return true;  // ray complete without saturation
            if (fin == 0ull && B.n == K && n_before == K) {
                // a full buffer of primitives that all outlive the window:
                // more than K primitives overlap one point of the ray
                out.status = 1;
                return true;
            }
            // drop finalised events (stable, in place: the write index never
            // passes the read index)
            int wpos = 0;
            if constexpr (K > 16) {
                float ws = 0.f;
                for (int i = 0; i < B.n; ++i)
                    if (!((fin >> i) & 1ull)) {
                        ws += B.w[i];
                        B.move(wpos++, i);
                    }
                st.wbuf = ws;
            } else {
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    if (i < B.n && !((fin >> i) & 1ull)) {
#pragma unroll
                        for (int j = 0; j <= i; ++j)
                            if (j == wpos) B.move(j, i);
                        ++wpos;
                    }
                }
            }
            B.n = wpos;
            S_fin = T;
            t_cur = t_w;
            lb_a = cap_a;   // the next round gathers keys >= the first rejected one
            lb_id = cap_id;
            return false;
        }
        // saturation inside (t_cur, t_w]: bracketed Newton on F(t) = 1.
        // Bracket: F is constant after the last exit in the buffer; F(t) is at
        // most S_fin plus the full weights of the entries before t, so F < 1 at
        // every entry reached before that sum comes near 1; and t_sat <= cap_sat
        // (t_w itself may be +inf).
        double lo = t_cur, hi = t_w;
        {
            float bmax = -kInf, cum = S_fin, lo_a = -kInf;
#pragma unroll Unr<K>::v
            for (int i = 0; i < K; ++i)
                if (i < B.n && (double)B.a[i] < t_w) {
                    bmax = fmaxf(bmax, B.b[i]);
                    if (cum < 1.f - 1e-4f) lo_a = B.a[i];  // F(a_i) <= cum < 1
                    cum += B.w[i];
                }
            hi = fmin(fmin(hi, (double)bmax), (double)cap_sat);
            lo = fmax(lo, (double)lo_a);
        }
        // Entries exiting by lo count in full at every t of the bracket and
        // entries starting at or after hi not at all; the chords of the others
        // (the only ones that can straddle t) are kept in LDS while t_sat is
        // solved, with their full weights in registers (a wide buffer holds
        // its chords itself: the solve walks the mask of those entries).
        __shared__ float4 cc_lds[kChordCache * 2 * kBlock];
        ChordCache cc{cc_lds, 0ull};
        float F_base = S_fin;
        float wc[kChordCache];
        int ns = 0, n_act = 0;
        uint64_t act = 0;  // wide buffer: the entries that can straddle t
#pragma unroll Unr<K>::v
        for (int i = 0; i < K; ++i) {
            if (i < B.n) {
                if ((double)B.b[i] <= lo) {
                    F_base += B.w[i];
                } else if ((double)B.a[i] < hi) {
                    ++n_act;
                    if constexpr (K > 16) {
                        act |= 1ull << i;
                    } else if (ns < kChordCache) {
#pragma unroll
                        for (int k = 0; k < kChordCache; ++k)
                            if (k == ns) wc[k] = B.w[i];
                        cache_put(cc, ns++, ev_chord(S, r, B.id[i], tc));
                        cc.mask |= 1ull << i;
                    }
                }
            }
        }
        const bool cached = n_act <= kChordCache;
        // F(t) - 1 and F'(t) on the bracket
        auto eval = [&](double t, float &g) __attribute__((always_inline)) {
            if constexpr (K > 16) {
                float F = F_base, G = 0.f;
                for (uint64_t m = act; m; m &= m - 1) {
                    const Chord c = ev_chord_c(S, r, B, __builtin_ctzll(m), nullptr, tc);
                    F += half_integral_to(c, t);
                    G += half_kernel_at(c, t);
                }
                g = G;
                return F - 1.f;
            }
            if (!cached) return sweep_F<K>(S, r, B, S_fin, t, &g, tc, &cc) - 1.f;
            float F = F_base, G = 0.f;
#pragma unroll
            for (int k = 0; k < kChordCache; ++k) {
                if (k < ns) {
                    const Chord c = cache_get_slot(cc, k);
                    if (t >= c.bd) {
                        F += wc[k];
                    } else if (t > (double)c.a) {
                        F += 0.5f * c.pref * erf_diff(c.ta, tau_at(c, t));
                        G += half_kernel_at(c, t);
                    }
                }
            }
            g = G;
            return F - 1.f;
        };
        // Start at the middle of the bracket (for a lone saturating primitive
        // the middle of its chord, where its kernel peaks).  t_sat is resolved
        // far below float resolution in t (near a thin primitive dF/dt is ~1e4),
        // until F itself is within a few float ulps of 1, where the float sum
        // cannot tell the sides apart.
        double t = 0.5 * (lo + hi);
        for (int it = 0; it < 60; ++it) {
            float g;
            const float f = eval(t, g);
            if (fabsf(f) <= 3e-7f) break;
            if (f > 0.f) hi = t; else lo = t;
            if (hi - lo <= 1e-13 * fmax(fabs(hi), 1e-30)) break;
            double tn = (g > 0.f) ? t - (double)f / (double)g : 0.5 * (lo + hi);
            if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
            if (fabs(tn - t) <= 1e-13 * fmax(fabs(t), 1e-30)) { t = tn; break; }
            t = tn;
        }
        const double tsat = t;
        if (mode == kModeSaturate) {
            out.t = (float)tsat;
            out.td = tsat;
            return true;
        }
        if (mode == kModeEmitter) {
            int ti = -1;
#pragma unroll Unr<K>::v
            for (int i = 0; i < K; ++i)
                if (i < B.n && B.id[i] == target) ti = i;
            if (ti >= 0) {
                float tb = 0.f, ta = 0.f, tw = 0.f;
#pragma unroll Unr<K>::v
                for (int i = 0; i < K; ++i)
                    if (i == ti) { tb = B.b[i]; ta = B.a[i]; tw = B.w[i]; }
                if ((double)tb <= tsat) out.t = tw;
                else if ((double)ta < tsat) out.t = half_integral_to(ev_chord_c(S, r, B, ti, &cc, tc), tsat);
            }
            return true;
        }
        // collide: exits before t_sat in (b, id) order, then straddlers by id
        {
            float run = S_fin, pb = -kInf;
            int pid = -1;
            for (int step = 0; step < K; ++step) {
                float bb = kInf, bw = 0.f, ba = 0.f;
                int bid = 0x7fffffff, bi = -1;
#pragma unroll Unr<K>::v
                for (int i = 0; i < K; ++i)
                    if (i < B.n && (double)B.b[i] <= tsat) {
                        if (key_less(pb, pid, B.b[i], B.id[i]) && key_less(B.b[i], B.id[i], bb, bid)) {
                            bb = B.b[i]; bid = B.id[i]; bw = B.w[i]; ba = B.a[i]; bi = i;
                        }
                    }
                if (bi < 0) break;
                run += bw;
                out.prim = bid;
                out.t = 0.5f * (ba + bb);
                if (run > u) return true;
                pb = bb;
                pid = bid;
            }
            // straddlers a < t_sat < b, ascending original index
            int pidx = -1;
            for (int step = 0; step < K; ++step) {
                int bid = 0x7fffffff, bi = -1;
#pragma unroll Unr<K>::v
                for (int i = 0; i < K; ++i)
                    if (i < B.n && (double)B.b[i] > tsat && (double)B.a[i] < tsat &&
                        B.id[i] > pidx && B.id[i] < bid) {
                        bid = B.id[i];
                        bi = i;
                    }
                if (bi < 0) break;
                const Chord c = ev_chord_c(S, r, B, bi, &cc, tc);
                run += half_integral_to(c, tsat);
                out.prim = bid;
                out.t = 0.5f * (c.a + c.b);
                if (run > u) return true;
                pidx = bid;
            }
            // rounding left u above the total of 1: keep the last candidate
            return true;
        }
    }
    return false;  // not reached: every path above returns
}

// ---------------------------------------------------------------------------
// Persistent waves over a list of rays: a lane whose ray is done takes the
// next entry at once, and a traversal is suspended when at most kSuspendAt
// lanes of the wave are still walking the tree (the others then take new
// rays), so lanes do not wait for the slowest ray of their wave.
// ---------------------------------------------------------------------------
constexpr int kSuspendAt = 32;

// Lanes whose ray is done (want) take the next entries of the list: one
// atomic per wave, entries handed out in lane order.  Returns the list
// position for wanting lanes (>= n when the list is exhausted), -1 otherwise.
__device__ __forceinline__ int64_t lane_refill(bool want, int32_t *work) {
    const uint64_t m = __ballot(want);
    if (m == 0ull) return -1;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(work, __popcll(m));
    base = __shfl(base, leader);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    return want ? (int64_t)base + __popcll(m & below) : -1;
}

// The whole sweep of one ray.
template <int K>
__device__ __forceinline__ SweepOut sweep(const SceneDev &S, const RayD &r, int excl, int mode, float u,
                                          int target, int *stack, uint32_t *err, TraceCount &tc,
                                          float stop_a = -__builtin_huge_valf()) {
    SweepState<K> st;
    SweepOut out;
    int spill[kStackSpill];
    sweep_start(st, out, r, mode);
    while (!sweep_round<K>(S, r, excl, mode, u, target, stop_a, st, out, stack, spill, 0, err, tc)) {
    }
    return out;
}

}  // namespace ugp
