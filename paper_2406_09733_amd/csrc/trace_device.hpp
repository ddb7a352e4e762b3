// trace_device.hpp -- device side of the scene queries: the ray / primitive
// chord and ray integral, BVH traversal with an LDS stack, transmittance and
// the ordered sweep that implements primitive-level free-flight sampling.
//
// Precision: the ray-frame transform of each candidate primitive (rotation
// from the quaternion, the map M = S^-1 R^T, closest approach, rho^2) is done
// in FP64 from the FP32 inputs, because for thin primitives the closest
// approach cancels ~15 bits; kernel values (erf/erfc/exp) and all sums are FP32.
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
    double ox, oy, oz;     // origin (exact widening of the float input)
    double dx, dy, dz;     // direction
    double t0, t1;         // parameter range
    float fox, foy, foz;   // float origin for slab tests
    float idx, idy, idz;   // float inverse direction for slab tests
};

__device__ __forceinline__ float safe_inv(float d) {
    const float a = fabsf(d) < 1e-20f ? copysignf(1e-20f, d) : d;
    return 1.f / a;
}

__device__ __forceinline__ RayD make_ray(float ox, float oy, float oz, float dx, float dy, float dz,
                                         double t0, double t1) {
    RayD r;
    r.ox = ox; r.oy = oy; r.oz = oz;
    r.dx = dx; r.dy = dy; r.dz = dz;
    r.t0 = t0; r.t1 = t1;
    r.fox = ox; r.foy = oy; r.foz = oz;
    r.idx = safe_inv(dx); r.idy = safe_inv(dy); r.idz = safe_inv(dz);
    return r;
}

__device__ __forceinline__ RayD load_ray(const float *rays, int64_t i) {
    const float4 a = reinterpret_cast<const float4 *>(rays)[2 * i];
    const float4 b = reinterpret_cast<const float4 *>(rays)[2 * i + 1];
    return make_ray(a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w);
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

struct HotRec {
    float mx, my, mz, d;
    float qw, qx, qy, qz;
    float sx, sy, sz;
    int orig;
};

__device__ __forceinline__ HotRec load_hot(const float4 *hot, int i) {
    const float4 a = hot[3 * i], b = hot[3 * i + 1], c = hot[3 * i + 2];
    return HotRec{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, __float_as_int(c.w)};
}

// Returns false if the clipped chord is empty.
__device__ inline bool chord(const HotRec &h, const RayD &r, float r2, Chord &c) {
    const double w = h.qw, x = h.qx, y = h.qy, z = h.qz;
    const double s2 = 2.0 * rcp_d(w * w + x * x + y * y + z * z);
    const double xx = x * x * s2, yy = y * y * s2, zz = z * z * s2;
    const double xy = x * y * s2, xz = x * z * s2, yz = y * z * s2;
    const double wx = w * x * s2, wy = w * y * s2, wz = w * z * s2;
    // columns of R: the local axes in world space
    const double c00 = 1.0 - yy - zz, c01 = xy + wz, c02 = xz - wy;
    const double c10 = xy - wz, c11 = 1.0 - xx - zz, c12 = yz + wx;
    const double c20 = xz + wy, c21 = yz - wx, c22 = 1.0 - xx - yy;
    const double i0 = rcp_d(h.sx), i1 = rcp_d(h.sy), i2 = rcp_d(h.sz);
    const double ex = r.ox - (double)h.mx, ey = r.oy - (double)h.my, ez = r.oz - (double)h.mz;
    const double o0 = (c00 * ex + c01 * ey + c02 * ez) * i0;
    const double o1 = (c10 * ex + c11 * ey + c12 * ez) * i1;
    const double o2 = (c20 * ex + c21 * ey + c22 * ez) * i2;
    const double w0 = (c00 * r.dx + c01 * r.dy + c02 * r.dz) * i0;
    const double w1 = (c10 * r.dx + c11 * r.dy + c12 * r.dz) * i1;
    const double w2 = (c20 * r.dx + c21 * r.dy + c22 * r.dz) * i2;
    const double A = w0 * w0 + w1 * w1 + w2 * w2;
    const double B = o0 * w0 + o1 * w1 + o2 * w2;
    const double C = o0 * o0 + o1 * o1 + o2 * o2;
    const double iA = rcp_d(A);
    const double tc = -B * iA;
    const double rho2 = fmax(fma(B, tc, C), 0.0);
    if (!(rho2 < (double)r2)) return false;
    const float rho2f = (float)rho2;
    const double half = (double)sqrtf((float)(((double)r2 - rho2) * iA));
    const double tlo = tc - half, thi = tc + half;
    const double a = fmax(r.t0, tlo), b = fmin(r.t1, thi);
    if (!(a < b)) return false;
    const float s = sqrtf(0.5f * (float)A);
    const float taumax = sqrtf(0.5f * fmaxf(r2 - rho2f, 0.f));
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
__device__ __forceinline__ void slab2(const float4 &n0, const float4 &n1, const float4 &n2,
                                      const RayD &r, float lo, float hi, bool &hl, bool &hr,
                                      float &tl, float &tr) {
    const float ox = r.fox, oy = r.foy, oz = r.foz;
    const float ix = r.idx, iy = r.idy, iz = r.idz;
    // left box lo (n0.x, n0.y, n0.z) hi (n0.w, n1.x, n1.y)
    float ax = (n0.x - ox) * ix, bx = (n0.w - ox) * ix;
    float ay = (n0.y - oy) * iy, by = (n1.x - oy) * iy;
    float az = (n0.z - oz) * iz, bz = (n1.y - oz) * iz;
    float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), lo));
    float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), hi));
    hl = tn <= tf + 5e-7f * fmaxf(fabsf(tn), fabsf(tf));
    tl = tn;
    // right box lo (n1.z, n1.w, n2.x) hi (n2.y, n2.z, n2.w)
    ax = (n1.z - ox) * ix; bx = (n2.y - ox) * ix;
    ay = (n1.w - oy) * iy; by = (n2.z - oy) * iy;
    az = (n2.x - oz) * iz; bz = (n2.w - oz) * iz;
    tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), lo));
    tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), hi));
    hr = tn <= tf + 5e-7f * fmaxf(fabsf(tn), fabsf(tf));
    tr = tn;
}

template <class LeafFn, class HiFn>
__device__ inline bool traverse(const SceneDev &S, const RayD &r, float lo, HiFn &&hi, int *stack,
                                uint32_t *err, TraceCount &tc, LeafFn &&leaf) {
    const int lane = threadIdx.x;
    int ref = S.root;
    if (ref < 0) {
        ++tc.prims;
        return leaf(~ref);
    }
    int sp = 0;
    for (;;) {
        ++tc.nodes;
        const float4 *nd = S.nodes + 4 * (int64_t)ref;
        const float4 n0 = nd[0], n1 = nd[1], n2 = nd[2], n3 = nd[3];
        const int cl = __float_as_int(n3.x), cr = __float_as_int(n3.y);
        bool hl, hr;
        float tl, tr;
        slab2(n0, n1, n2, r, lo, hi(), hl, hr, tl, tr);
        // leaf children first (the nearer one first)
        int leaves[2];
        int nl = 0;
        const bool lleaf = hl && cl < 0, rleaf = hr && cr < 0;
        if (lleaf && rleaf) {
            leaves[0] = tl <= tr ? ~cl : ~cr;
            leaves[1] = tl <= tr ? ~cr : ~cl;
            nl = 2;
        } else if (lleaf) {
            leaves[nl++] = ~cl;
        } else if (rleaf) {
            leaves[nl++] = ~cr;
        }
        for (int i = 0; i < nl; ++i) {
            ++tc.prims;
            if (leaf(leaves[i])) return true;
        }
        const float h = hi();
        const bool gl = hl && cl >= 0 && tl <= h + 5e-7f * fabsf(h);
        const bool gr = hr && cr >= 0 && tr <= h + 5e-7f * fabsf(h);
        if (gl && gr) {
            const int nearc = tl <= tr ? cl : cr, farc = tl <= tr ? cr : cl;
            if (sp < kStackSize) {
                stack[sp * kBlock + lane] = farc;
                ++sp;
            } else {
                atomicOr(err, kErrStack);
            }
            ref = nearc;
        } else if (gl) {
            ref = cl;
        } else if (gr) {
            ref = cr;
        } else {
            if (sp == 0) return false;
            --sp;
            ref = stack[sp * kBlock + lane];
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
    const float lo = (float)r.t0;
    const float hi1 = r.t1 < 3.0e38 ? (float)r.t1 : kInf;
    traverse(S, r, lo, [&]() { return hi1; }, stack, err, tc, [&](int p) {
        const HotRec h = load_hot(S.hot, p);
        if (h.orig == excl) return false;
        Chord c;
        if (!chord(h, r, S.r2, c)) return false;
        F += c.W;
        return early_out && F >= 1.f;
    });
    return F;
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
};

// loops over the event buffer are unrolled (register arrays) only for small K
template <int K>
struct Unr {
    static constexpr int v = K <= 16 ? K : 1;
};

template <int K>
struct EvBuf {
    Ev e[K];
    int n;
};

// select event j (dynamic) out of the register array
template <int K>
__device__ __forceinline__ Ev ev_get(const EvBuf<K> &B, int j) {
    if constexpr (K > 16) {
        return B.e[j];
    } else {
        Ev r = B.e[0];
#pragma unroll
        for (int i = 1; i < K; ++i)
            if (i == j) r = B.e[i];
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

// F(t) and F'(t) over the buffer: S_fin + sum of (full weights of exits <= t,
// partial weights of entries before t that exit later)
template <int K>
__device__ inline float sweep_F(const SceneDev &S, const RayD &r, const EvBuf<K> &B, float S_fin,
                                double t, float *dF, TraceCount &tc) {
    float F = S_fin, G = 0.f;
    uint64_t partial = 0;
#pragma unroll Unr<K>::v
    for (int i = 0; i < K; ++i) {
        if (i < B.n) {
            if ((double)B.e[i].b <= t) F += B.e[i].w;
            else if ((double)B.e[i].a < t) partial |= 1ull << i;
        }
    }
    while (partial) {
        const int j = __builtin_ctzll(partial);
        partial &= partial - 1;
        const Chord c = ev_chord(S, r, ev_get(B, j).id, tc);
        F += half_integral_to(c, t);
        G += half_kernel_at(c, t);
    }
    if (dF) *dF = G;
    return F;
}

template <int K>
__device__ inline SweepOut sweep(const SceneDev &S, const RayD &r, int excl, int mode, float u,
                                 int target, int *stack, uint32_t *err, TraceCount &tc) {
    SweepOut out{-1, __builtin_nanf(""), 0};
    if (mode == kModeSaturate) out.t = (float)r.t1;
    if (mode == kModeEmitter) out.t = 0.f;
    EvBuf<K> B;
    B.n = 0;
    float S_fin = 0.f;          // finalised weight (exits before t_cur)
    double t_cur = r.t0;
    float lb_a = -kInf;         // entries with key <= (lb_a, lb_id) were seen
    int lb_id = -1;
    const float t1f = r.t1 < 3.0e38 ? (float)r.t1 : kInf;
    for (int round = 0; round < 4096; ++round) {
        ++tc.rounds;
        float cap_a = kInf;
        int cap_id = 0x7fffffff;
        bool evicted = false;
        const int n_before = B.n;
        traverse(S, r, fmaxf((float)r.t0, lb_a), [&]() { return fminf(cap_a, t1f); }, stack, err, tc,
                 [&](int p) {
                     const HotRec h = load_hot(S.hot, p);
                     if (h.orig == excl) return false;
                     Chord c;
                     if (!chord(h, r, S.r2, c)) return false;
                     if (key_less(c.a, c.orig, lb_a, lb_id)) return false;    // seen before
                     if (!key_less(c.a, c.orig, cap_a, cap_id)) return false; // beyond cap
                     Ev x{c.a, c.b, c.W, c.orig};
                     bool placed = false;
#pragma unroll Unr<K>::v
                     for (int i = 0; i < K; ++i) {
                         if (i < B.n) {
                             if (key_less(x.a, x.id, B.e[i].a, B.e[i].id)) {
                                 const Ev t = B.e[i];
                                 B.e[i] = x;
                                 x = t;
                             }
                         } else if (!placed) {
                             B.e[i] = x;
                             placed = true;
                         }
                     }
                     if (placed) {
                         ++B.n;
                     } else {  // x is the largest of K + 1: evict it
                         evicted = true;
                         cap_a = x.a;
                         cap_id = x.id;
                     }
                     return false;
                 });
        // window end: every primitive entering before t_w is in the buffer
        const double t_w = evicted ? (double)cap_a : r.t1;
        // progress check: nothing new and nothing can exit -> overflow
        // upper bound on F(t_w)
        float U = S_fin;
#pragma unroll Unr<K>::v
        for (int i = 0; i < K; ++i)
            if (i < B.n && (double)B.e[i].a < t_w) U += B.e[i].w;
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
                if (i < B.n && (!evicted || (double)B.e[i].b <= t_w)) {
                    T += B.e[i].w;
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
                            const Ev &e = B.e[i];
                            if (key_less(pb, pid, e.b, e.id) && key_less(e.b, e.id, bb, bid)) {
                                bb = e.b; bid = e.id; bw = e.w; ba = e.a; bi = i;
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
                return out;
            }
            if (mode == kModeEmitter) {
#pragma unroll Unr<K>::v
                for (int i = 0; i < K; ++i)
                    if (((fin >> i) & 1ull) && B.e[i].id == target) out.t = B.e[i].w;
            }
            if (!evicted) return out;  // ray complete without saturation
            if (fin == 0ull && B.n == K && n_before == K) {
                // a full buffer of primitives that all outlive the window:
                // more than K primitives overlap one point of the ray
                out.status = 1;
                return out;
            }
            // drop finalised events (stable, in place: the write index never
            // passes the read index)
            int wpos = 0;
            if constexpr (K > 16) {
                for (int i = 0; i < B.n; ++i)
                    if (!((fin >> i) & 1ull)) B.e[wpos++] = B.e[i];
            } else {
#pragma unroll Unr<K>::v
                for (int i = 0; i < K; ++i) {
                    if (i < B.n && !((fin >> i) & 1ull)) {
#pragma unroll Unr<K>::v
                        for (int j = 0; j <= i; ++j)
                            if (j == wpos) B.e[j] = B.e[i];
                        ++wpos;
                    }
                }
            }
            B.n = wpos;
            S_fin = T;
            t_cur = t_w;
            lb_a = cap_a;   // the next round gathers keys >= the first rejected one
            lb_id = cap_id;
            continue;
        }
        // saturation inside (t_cur, t_w]: bracketed Newton on F(t) = 1.  F is
        // constant after the last exit in the buffer, so that bounds the bracket
        // (t_w itself may be +inf).
        double lo = t_cur, hi = t_w;
        {
            float bmax = -kInf;
#pragma unroll Unr<K>::v
            for (int i = 0; i < K; ++i)
                if (i < B.n && (double)B.e[i].a < t_w) bmax = fmaxf(bmax, B.e[i].b);
            hi = fmin(hi, (double)bmax);
        }
        double t = hi;
        // Iterate in t to well below float resolution: near a thin primitive
        // dF/dt is ~1e4, so t_sat must be resolved far finer than t's ulp for
        // the clipped weights to be accurate; F itself is float.
        for (int it = 0; it < 60; ++it) {
            float g;
            const float f = sweep_F<K>(S, r, B, S_fin, t, &g, tc) - 1.f;
            if (f == 0.f) break;
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
            return out;
        }
        if (mode == kModeEmitter) {
#pragma unroll Unr<K>::v
            for (int i = 0; i < K; ++i)
                if (i < B.n && B.e[i].id == target) {
                    if ((double)B.e[i].b <= tsat) out.t = B.e[i].w;
                    else if ((double)B.e[i].a < tsat) {
                        const Chord c = ev_chord(S, r, target, tc);
                        out.t = half_integral_to(c, tsat);
                    }
                }
            return out;
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
                    if (i < B.n && (double)B.e[i].b <= tsat) {
                        const Ev &e = B.e[i];
                        if (key_less(pb, pid, e.b, e.id) && key_less(e.b, e.id, bb, bid)) {
                            bb = e.b; bid = e.id; bw = e.w; ba = e.a; bi = i;
                        }
                    }
                if (bi < 0) break;
                run += bw;
                out.prim = bid;
                out.t = 0.5f * (ba + bb);
                if (run > u) return out;
                pb = bb;
                pid = bid;
            }
            // straddlers a < t_sat < b, ascending original index
            int pidx = -1;
            for (int step = 0; step < K; ++step) {
                int bid = 0x7fffffff, bi = -1;
#pragma unroll Unr<K>::v
                for (int i = 0; i < K; ++i)
                    if (i < B.n && (double)B.e[i].b > tsat && (double)B.e[i].a < tsat &&
                        B.e[i].id > pidx && B.e[i].id < bid) {
                        bid = B.e[i].id;
                        bi = i;
                    }
                if (bi < 0) break;
                const Chord c = ev_chord(S, r, bid, tc);
                run += half_integral_to(c, tsat);
                out.prim = bid;
                out.t = 0.5f * (c.a + c.b);
                if (run > u) return out;
                pidx = bid;
            }
            // rounding left u above the total of 1: keep the last candidate
            return out;
        }
    }
    out.status = 1;
    return out;
}

}  // namespace ugp
