// ugp_math.hpp -- device math for libugp: small vectors, the Philox4x32-10
// counter-based generator, orthonormal frames, the delta-NDF and SGGX phase functions
// and the pinhole camera.  FP32 unless a name says otherwise.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ugp {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kInvPi = 0.318309886183790671538f;
constexpr float kInf = __builtin_huge_valf();

struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator-(V3 a) { return v3(-a.x, -a.y, -a.z); }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ V3 mul(V3 a, V3 b) { return v3(a.x * b.x, a.y * b.y, a.z * b.z); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ V3 normalize(V3 a) { return rsqrtf(dot(a, a)) * a; }
__device__ __forceinline__ bool nonzero(V3 a) { return a.x > 0.f || a.y > 0.f || a.z > 0.f; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies (hi/lo halves), a word permutation and an xor with the round key;
// the key advances by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// top 24 bits -> [0,1), exact in float
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

struct Rng4 {
    float u[4];
};
__device__ __forceinline__ Rng4 rng4(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t vertex,
                                     uint32_t group) {
    uint4 x = philox4x32_10(make_uint4(pixel, sample, vertex, group), (uint32_t)seed,
                            (uint32_t)(seed >> 32));
    return Rng4{{u01(x.x), u01(x.y), u01(x.z), u01(x.w)}};
}

// Orthonormal basis around unit n (Duff et al., "Building an Orthonormal Basis,
// Revisited", JCGT 2017).
__device__ __forceinline__ void onb(V3 n, V3 &b1, V3 &b2) {
    const float sign = n.z >= 0.f ? 1.f : -1.f;
    const float a = -1.f / (sign + n.z);
    const float b = n.x * n.y * a;
    b1 = v3(1.f + sign * n.x * n.x * a, sign * b, -sign * n.x);
    b2 = v3(b, sign + n.y * n.y * a, -n.y);
}

// ---------------------------------------------------------------------------
// Delta-NDF phase function (Sec. 6): with a single facet normal the phase
// function of eq. phase_function is the surface BSDF times the cosine.  The
// facet normal is flipped toward w_o; only reflection scatters.
//   diffuse: f = albedo/pi cos_i, pdf = cos_i/pi (cosine sampling)
//   glossy : GGX with alpha = roughness^2 (>= 1e-4), height-correlated Smith
//            G2, Schlick Fresnel with F0 = albedo; sampled by visible normals
//            (Heitz, "Sampling the GGX Distribution of Visible Normals",
//            JCGT 2018): f = F D G2/(4 cos_o), pdf = G1(w_o) D / (4 cos_o).
// ---------------------------------------------------------------------------
struct Facet {
    V3 n, b1, b2;
};
__device__ __forceinline__ Facet facet(V3 nrm, V3 wo) {
    Facet f;
    f.n = dot(nrm, wo) >= 0.f ? nrm : -nrm;
    onb(f.n, f.b1, f.b2);
    return f;
}
__device__ __forceinline__ V3 to_local(const Facet &f, V3 v) { return v3(dot(v, f.b1), dot(v, f.b2), dot(v, f.n)); }
__device__ __forceinline__ V3 to_world(const Facet &f, V3 l) {
    return l.x * f.b1 + l.y * f.b2 + l.z * f.n;
}

__device__ __forceinline__ float ggx_alpha(float rough) { return fmaxf(rough * rough, 1e-4f); }
__device__ __forceinline__ float ggx_D(float a, float ch) {
    const float a2 = a * a;
    const float t = ch * ch * (a2 - 1.f) + 1.f;
    return a2 / (kPi * t * t);
}
__device__ __forceinline__ float ggx_lambda(float a, float c) {
    const float c2 = c * c;
    const float tan2 = fmaxf(0.f, 1.f - c2) / c2;
    return 0.5f * (-1.f + sqrtf(1.f + a * a * tan2));
}
__device__ __forceinline__ float pow5(float x) {
    const float x2 = x * x;
    return x2 * x2 * x;
}

// local frame: returns f (rgb) and pdf
__device__ inline V3 phase_eval_local(int mat, V3 alb, float rough, V3 wo, V3 wi, float &pdf) {
    pdf = 0.f;
    if (wo.z <= 0.f || wi.z <= 0.f) return v3(0.f, 0.f, 0.f);
    if (mat == 0) {
        pdf = wi.z * kInvPi;
        return (wi.z * kInvPi) * alb;
    }
    const float a = ggx_alpha(rough);
    const V3 h = normalize(wo + wi);
    const float D = ggx_D(a, h.z);
    const float lo = ggx_lambda(a, wo.z), li = ggx_lambda(a, wi.z);
    const float G2 = 1.f / (1.f + lo + li), G1 = 1.f / (1.f + lo);
    const float sch = pow5(1.f - fmaxf(0.f, dot(wi, h)));
    const float k = D * G2 / (4.f * wo.z);
    pdf = G1 * D / (4.f * wo.z);
    return v3((alb.x + (1.f - alb.x) * sch) * k, (alb.y + (1.f - alb.y) * sch) * k,
              (alb.z + (1.f - alb.z) * sch) * k);
}

// (d f_c / d albedo_c) / f_c of the phase function above, per channel, for
// the pair (wo, wi): f is linear in the albedo -- the diffuse lobe is
// albedo/pi cos_i, the glossy lobe's Schlick term is F0 + (1 - F0) m with
// m = (1 - wi.h)^5 -- so a path term's derivative is the term times this
// ratio.  A channel whose f is zero (a diffuse one of zero albedo) reports 0.
__device__ inline V3 phase_albedo_ratio(int mat, V3 alb, V3 wo, V3 wi) {
    auto r = [](float num, float den) __attribute__((always_inline)) { return den > 0.f ? num / den : 0.f; };
    if (mat != 1) return v3(r(1.f, alb.x), r(1.f, alb.y), r(1.f, alb.z));  // Lambert and SGGX-Lambert
    const V3 h = normalize(wo + wi);
    const float m = pow5(1.f - fmaxf(0.f, dot(wi, h)));
    return v3(r(1.f - m, alb.x + (1.f - alb.x) * m), r(1.f - m, alb.y + (1.f - alb.y) * m),
              r(1.f - m, alb.z + (1.f - alb.z) * m));
}

// d log f / d roughness of the phase function above for the pair (wo, wi),
// the same for every channel: the glossy lobe's D and G2 depend on alpha =
// roughness^2 (Schlick F does not), the diffuse and SGGX-Lambert lobes not
// at all; 0 where alpha is clamped (roughness <= 0.01).
//   d log D / d alpha  = 2/alpha - 4 alpha c_h^2 / (c_h^2 (alpha^2 - 1) + 1)
//   d log G2 / d alpha = -(dLambda_o + dLambda_i) G2,
//   dLambda / d alpha  = alpha tan^2 / (2 sqrt(1 + alpha^2 tan^2))
__device__ inline float phase_rough_ratio(int mat, float rough, V3 wo, V3 wi) {
    const float a = rough * rough;
    if (mat != 1 || !(a > 1e-4f) || wo.z <= 0.f || wi.z <= 0.f) return 0.f;
    const V3 h = normalize(wo + wi);
    const float c2 = h.z * h.z;
    const float dlogD = 2.f / a - 4.f * a * c2 / (c2 * (a * a - 1.f) + 1.f);
    auto dlam = [a](float c) __attribute__((always_inline)) {
        const float t2 = fmaxf(0.f, 1.f - c * c) / (c * c);
        return a * t2 / (2.f * sqrtf(1.f + a * a * t2));
    };
    const float G2 = 1.f / (1.f + ggx_lambda(a, wo.z) + ggx_lambda(a, wi.z));
    return 2.f * rough * (dlogD - (dlam(wo.z) + dlam(wi.z)) * G2);
}

// local frame sample: returns wi, weight f/pdf; pdf 0 = no sample
__device__ inline V3 phase_sample_local(int mat, V3 alb, float rough, V3 wo, float u1, float u2,
                                        V3 &wgt, float &pdf) {
    pdf = 0.f;
    wgt = v3(0.f, 0.f, 0.f);
    if (wo.z <= 0.f) return v3(0.f, 0.f, 1.f);
    float sp, cp;
    sincosf(2.f * kPi * u2, &sp, &cp);
    if (mat == 0) {
        const float r = sqrtf(u1);
        const V3 wi = v3(r * cp, r * sp, sqrtf(fmaxf(0.f, 1.f - u1)));
        if (wi.z <= 0.f) return wi;
        pdf = wi.z * kInvPi;
        wgt = alb;
        return wi;
    }
    const float a = ggx_alpha(rough);
    const V3 Vh = normalize(v3(a * wo.x, a * wo.y, wo.z));
    const float lensq = Vh.x * Vh.x + Vh.y * Vh.y;
    V3 T1 = lensq > 0.f ? rsqrtf(lensq) * v3(-Vh.y, Vh.x, 0.f) : v3(1.f, 0.f, 0.f);
    const V3 T2 = cross(Vh, T1);
    const float r = sqrtf(u1);
    const float p1 = r * cp;
    float p2 = r * sp;
    const float s = 0.5f * (1.f + Vh.z);
    p2 = (1.f - s) * sqrtf(fmaxf(0.f, 1.f - p1 * p1)) + s * p2;
    const float p3 = sqrtf(fmaxf(0.f, 1.f - p1 * p1 - p2 * p2));
    const V3 Nh = p1 * T1 + p2 * T2 + p3 * Vh;
    const V3 h = normalize(v3(a * Nh.x, a * Nh.y, fmaxf(0.f, Nh.z)));
    const float c = dot(wo, h);
    const V3 wi = (2.f * c) * h - wo;
    if (wi.z <= 0.f) return wi;
    const float D = ggx_D(a, h.z);
    const float lo = ggx_lambda(a, wo.z), li = ggx_lambda(a, wi.z);
    const float G2 = 1.f / (1.f + lo + li), G1 = 1.f / (1.f + lo);
    pdf = G1 * D / (4.f * wo.z);
    const float sch = pow5(1.f - fmaxf(0.f, c));
    const float k = G2 / G1;
    wgt = v3((alb.x + (1.f - alb.x) * sch) * k, (alb.y + (1.f - alb.y) * sch) * k,
             (alb.z + (1.f - alb.z) * sch) * k);
    return wi;
}

// ---------------------------------------------------------------------------
// SGGX microflakes with a Lambertian base BSDF (material 2; Sec. 4.2, eq. vndf,
// eq. phase_function; App. B), in the world frame, per unit albedo.
// S is symmetric positive definite.  The flakes' normals are those of the
// ellipsoid x^T S x = 1: D(n) = 1 / (pi sqrt(det S) (n^T S^-1 n)^2), projected
// area sigma(w) = sqrt(w^T S w), visible normals D_wo(n) = <wo.n> D(n) /
// sigma(wo).  Per matrix a 64-B record, prepared in FP64 from the six float
// inputs (the inverse of a flat S cancels badly in FP32):
//   [0] S xx, yy, zz, xy   [1] S xz, yz, S^-1 xx, yy
//   [2] S^-1 zz, xy, xz, yz   [3] 1 / (pi sqrt(det S)), metallic, p_spec, 0
// A primitive holds two: its S, and the roughened S of App. B used by the
// approximate MIS pdf of material 3 (128 B).
// ---------------------------------------------------------------------------
struct Sggx {
    float xx, yy, zz, xy, xz, yz;        // S
    float ixx, iyy, izz, ixy, ixz, iyz;  // S^-1
    float dn;                            // 1 / (pi sqrt(det S))
    float met, ps;                       // metallic, probability of the specular lobe (material 3)
};

// record of s = (xx, yy, zz, xy, xz, yz); false (record zeroed) unless S is
// finite and positive definite (leading minors > 0)
__device__ inline bool sggx_prepare(const double s[6], float4 rec[4]) {
    const double xx = s[0], yy = s[1], zz = s[2], xy = s[3], xz = s[4], yz = s[5];
    const double axx = yy * zz - yz * yz, ayy = xx * zz - xz * xz, azz = xx * yy - xy * xy;
    const double axy = xz * yz - xy * zz, axz = xy * yz - xz * yy, ayz = xy * xz - xx * yz;
    const double det = xx * axx + xy * axy + xz * axz;
    bool ok = xx > 0.0 && azz > 0.0 && det > 0.0 && isfinite(det);
    for (int i = 0; i < 6; ++i) ok = ok && isfinite(s[i]);
    if (!ok) {
        for (int i = 0; i < 4; ++i) rec[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        return false;
    }
    const double id = 1.0 / det;
    rec[0] = make_float4((float)xx, (float)yy, (float)zz, (float)xy);
    rec[1] = make_float4((float)xz, (float)yz, (float)(axx * id), (float)(ayy * id));
    rec[2] = make_float4((float)(azz * id), (float)(axy * id), (float)(axz * id), (float)(ayz * id));
    rec[3] = make_float4((float)(1.0 / (3.14159265358979323846 * sqrt(det))), 0.f, 0.f, 0.f);
    return true;
}

// Largest eigenvalue of a symmetric S = (xx, yy, zz, xy, xz, yz) by the
// trigonometric closed form of the characteristic cubic, and a unit
// eigenvector of it: the largest cross product of two rows of S - lambda I,
// or, when the largest eigenvalue is repeated (rows all parallel), a unit
// vector orthogonal to the largest row (any vector of the eigenspace).
__device__ inline double sym3_top(const double s[6], double v[3]) {
    const double xx = s[0], yy = s[1], zz = s[2], xy = s[3], xz = s[4], yz = s[5];
    const double p1 = xy * xy + xz * xz + yz * yz;
    const double q = (xx + yy + zz) / 3.0;
    const double p2 = (xx - q) * (xx - q) + (yy - q) * (yy - q) + (zz - q) * (zz - q) + 2.0 * p1;
    if (!(p2 > 0.0)) {  // a multiple of I
        v[0] = 0.0; v[1] = 0.0; v[2] = 1.0;
        return q;
    }
    const double p = sqrt(p2 / 6.0), ip = 1.0 / p;
    const double bxx = (xx - q) * ip, byy = (yy - q) * ip, bzz = (zz - q) * ip;
    const double bxy = xy * ip, bxz = xz * ip, byz = yz * ip;
    double r = 0.5 * (bxx * (byy * bzz - byz * byz) - bxy * (bxy * bzz - byz * bxz) + bxz * (bxy * byz - byy * bxz));
    r = fmin(1.0, fmax(-1.0, r));
    const double lam = q + 2.0 * p * cos(acos(r) / 3.0);
    const double R[3][3] = {{xx - lam, xy, xz}, {xy, yy - lam, yz}, {xz, yz, zz - lam}};
    double best = -1.0;
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b) {
            const double c[3] = {R[a][1] * R[b][2] - R[a][2] * R[b][1], R[a][2] * R[b][0] - R[a][0] * R[b][2],
                                 R[a][0] * R[b][1] - R[a][1] * R[b][0]};
            const double l2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
            if (l2 > best) { best = l2; v[0] = c[0]; v[1] = c[1]; v[2] = c[2]; }
        }
    double rn = 0.0;
    int ra = 0;
    for (int a = 0; a < 3; ++a) {
        const double l2 = R[a][0] * R[a][0] + R[a][1] * R[a][1] + R[a][2] * R[a][2];
        if (l2 > rn) { rn = l2; ra = a; }
    }
    if (!(best > 1e-24 * rn * rn)) {  // repeated top eigenvalue: orthogonal to the largest row
        const double *w = R[ra];
        const int k = fabs(w[0]) <= fabs(w[1]) ? (fabs(w[0]) <= fabs(w[2]) ? 0 : 2) : (fabs(w[1]) <= fabs(w[2]) ? 1 : 2);
        const double e[3] = {k == 0 ? 1.0 : 0.0, k == 1 ? 1.0 : 0.0, k == 2 ? 1.0 : 0.0};
        v[0] = w[1] * e[2] - w[2] * e[1]; v[1] = w[2] * e[0] - w[0] * e[2]; v[2] = w[0] * e[1] - w[1] * e[0];
    }
    const double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int i = 0; i < 3; ++i) v[i] /= n;
    return lam;
}

// Both records of a primitive: S, and the roughened S~ = S + a^2 s3 (I - v3
// v3^T) of App. B (a = GGX alpha of the roughness, s3 the largest eigenvalue
// of S, v3 its eigenvector); the specular-lobe probability 1 / (1 + (1 - m)
// luminance(albedo)) and the metallic m ride in the first record.
__device__ inline bool sggx_prepare_prim(const double s[6], float rough, float met, const float alb[3],
                                         float4 rec[8]) {
    bool ok = sggx_prepare(s, rec);
    double v[3];
    const double top = ok ? sym3_top(s, v) : 0.0;
    const double a = (double)ggx_alpha(rough), c = a * a * top;
    const double r6[6] = {s[0] + c * (1.0 - v[0] * v[0]), s[1] + c * (1.0 - v[1] * v[1]), s[2] + c * (1.0 - v[2] * v[2]),
                          s[3] - c * v[0] * v[1], s[4] - c * v[0] * v[2], s[5] - c * v[1] * v[2]};
    ok = ok && sggx_prepare(r6, rec + 4);
    const double lum = 0.2126 * alb[0] + 0.7152 * alb[1] + 0.0722 * alb[2];
    rec[3].y = met;
    rec[3].z = (float)(1.0 / (1.0 + (1.0 - (double)met) * lum));
    return ok;
}

__device__ __forceinline__ Sggx sggx_load(const float4 *rec) {
    const float4 a = rec[0], b = rec[1], c = rec[2], d = rec[3];
    return Sggx{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w, d.x, d.y, d.z};
}
__device__ __forceinline__ V3 sggx_S(const Sggx &g, V3 v) {
    return v3(g.xx * v.x + g.xy * v.y + g.xz * v.z, g.xy * v.x + g.yy * v.y + g.yz * v.z,
              g.xz * v.x + g.yz * v.y + g.zz * v.z);
}
__device__ __forceinline__ V3 sggx_Sinv(const Sggx &g, V3 v) {
    return v3(g.ixx * v.x + g.ixy * v.y + g.ixz * v.z, g.ixy * v.x + g.iyy * v.y + g.iyz * v.z,
              g.ixz * v.x + g.iyz * v.y + g.izz * v.z);
}
__device__ __forceinline__ float sggx_sigma(const Sggx &g, V3 w) { return sqrtf(fmaxf(0.f, dot(w, sggx_S(g, w)))); }
// D_wo(n) given sigma(wo)
__device__ __forceinline__ float sggx_vndf(const Sggx &g, V3 wo, V3 n, float sig_o) {
    const float c = dot(wo, n);
    if (!(c > 0.f) || !(sig_o > 0.f)) return 0.f;
    const float q = dot(n, sggx_Sinv(g, n));
    return c * (g.dn / (q * q)) / sig_o;
}

// A visible normal: a point uniform in the ellipsoid's shadow along wo (the
// ellipse of the 2x2 matrix [e_a^T S^-1 e_b] on the plane (e1, e2) orthogonal
// to wo, from the unit disk by its Cholesky factor), lifted to the front
// surface x = q + t wo (larger root of x^T S x = 1); the normal is S x.
// The shadow's quadratic form (the Schur complement of S along wo, the
// inverse of that 2x2 matrix) maps q back to the disk point of radius^2 u1,
// so the root is t = -B/A + sqrt((1 - u1) / A) with A = wo^T S wo, B =
// q^T S wo: written so, with 1 - u1 exact in float, neither the
// discriminant nor S x = (S q - (B/A) S wo) + sqrt((1 - u1)/A) S wo cancels
// near the shadow's rim.
__device__ inline V3 sggx_sample_vndf(const Sggx &g, V3 wo, float u1, float u2) {
    V3 e1, e2;
    onb(wo, e1, e2);
    const V3 i2 = sggx_Sinv(g, e2);
    const float s11 = dot(e1, sggx_Sinv(g, e1)), s22 = dot(e2, i2), s12 = dot(e1, i2);
    const float l11 = sqrtf(s11), l21 = s12 / l11, l22 = sqrtf(fmaxf(0.f, s22 - l21 * l21));
    const float r = sqrtf(u1);
    float sp, cp;
    sincosf(2.f * kPi * u2, &sp, &cp);
    const float a = r * cp, b = r * sp;
    const V3 q = (l11 * a) * e1 + (l21 * a + l22 * b) * e2;
    const V3 Sw = sggx_S(g, wo), Sq = sggx_S(g, q);
    const float A = dot(wo, Sw), B = dot(q, Sw);
    return normalize((Sq - (B / A) * Sw) + sqrtf((1.f - u1) / A) * Sw);
}

// a direction cosine-distributed about the unit vector m
__device__ __forceinline__ V3 cosine_about(V3 m, float u1, float u2) {
    V3 b1, b2;
    onb(m, b1, b2);
    const float r = sqrtf(u1), z = sqrtf(fmaxf(0.f, 1.f - u1));
    float sp, cp;
    sincosf(2.f * kPi * u2, &sp, &cp);
    return (r * cp) * b1 + (r * sp) * b2 + z * m;
}

// Stochastic evaluation of f_p(wi, wo) / albedo with internal MIS: one normal
// from the visible NDF (u0, u1) and one from the Lambertian base's sampling
// reversed, cosine-distributed about wi (u2, u3), each weighted by the
// one-sample balance heuristic between the two densities.
__device__ inline float sggx_phase_est(const Sggx &g, V3 wo, V3 wi, float u0, float u1, float u2, float u3) {
    const float so = sggx_sigma(g, wo);
    const V3 n1 = sggx_sample_vndf(g, wo, u0, u1);
    const float p1 = sggx_vndf(g, wo, n1, so);
    const float f1 = fmaxf(0.f, dot(wi, n1)) * kInvPi;  // base BSDF at n1, also n1's density about wi
    float est = p1 > 0.f ? f1 * p1 / (p1 + f1) : 0.f;
    const V3 n3 = cosine_about(wi, u2, u3);
    const float p3 = sggx_vndf(g, wo, n3, so);
    const float c3 = fmaxf(0.f, dot(n3, wi)) * kInvPi;
    if (c3 > 0.f && p3 > 0.f) est += p3 * c3 / (c3 + p3);
    return est;
}

// The approximate MIS pdf of the Lambertian component (App. B): <w_h . w_o> / pi.
__device__ __forceinline__ float sggx_pdf_approx(V3 wo, V3 wi) {
    const V3 h = wo + wi;
    const float l2 = dot(h, h);
    return l2 > 0.f ? fmaxf(0.f, dot(h, wo)) * rsqrtf(l2) * kInvPi : 0.f;
}

// Importance sampling (Sec. 4.2): a visible normal, then the base BSDF's
// cosine sampling about it; weight = albedo (the visible-normal sampling is
// exact), pdf reported for MIS = the approximate one.
__device__ __forceinline__ V3 sggx_sample(const Sggx &g, V3 wo, float u0, float u1, float v0, float v1) {
    return cosine_about(sggx_sample_vndf(g, wo, u0, u1), v0, v1);
}

// ---------------------------------------------------------------------------
// Material 3: SGGX microflakes with a Disney-style base BSDF (Sec. 4.2: a
// microfacet specular component and a diffuse component with empirical
// retro-reflection).  At a flake normal n, cosine-weighted, for base colour
// c, roughness r (GGX alpha = r^2; r itself in the retro-reflection) and
// metallic m:
//   specular fs = F D G2 / (4 <n.wo>), Schlick F0 = 0.04 (1 - m) + c m
//   diffuse  fd = (1 - m) c / pi (1 + (F_D90 - 1)(1 - <n.wi>)^5)
//                 (1 + (F_D90 - 1)(1 - <n.wo>)^5) <n.wi>, F_D90 = 1/2 + 2 r <wi.h>^2
// both zero unless wi and wo lie on n's side.
// ---------------------------------------------------------------------------
__device__ inline void disney_base(V3 c, float rough, float met, V3 n, V3 wo, V3 wi, V3 &fs, V3 &fd) {
    fs = v3(0.f, 0.f, 0.f);
    fd = fs;
    const float co = dot(n, wo), ci = dot(n, wi);
    if (!(co > 0.f) || !(ci > 0.f)) return;
    const float a = ggx_alpha(rough);
    const V3 h = normalize(wo + wi);
    const float D = ggx_D(a, dot(n, h));
    const float G2 = 1.f / (1.f + ggx_lambda(a, co) + ggx_lambda(a, ci));
    const float cd = fmaxf(0.f, dot(wi, h));
    const float sch = pow5(1.f - cd);
    const float fd90 = 0.5f + 2.f * rough * cd * cd;
    const float rl = 1.f + (fd90 - 1.f) * pow5(1.f - ci), rv = 1.f + (fd90 - 1.f) * pow5(1.f - co);
    const float ks = D * G2 / (4.f * co), kd = (1.f - met) * kInvPi * rl * rv * ci;
    const float f0x = 0.04f * (1.f - met) + c.x * met, f0y = 0.04f * (1.f - met) + c.y * met,
                f0z = 0.04f * (1.f - met) + c.z * met;
    fs = v3((f0x + (1.f - f0x) * sch) * ks, (f0y + (1.f - f0y) * sch) * ks, (f0z + (1.f - f0z) * sch) * ks);
    fd = kd * c;
}

// a normal about the half vector h with density D(<n.h>) <n.h> (the GGX
// distribution's own sampling with normal and half vector exchanged)
__device__ __forceinline__ V3 ggx_ndf_about(V3 h, float a, float u1, float u2) {
    V3 b1, b2;
    onb(h, b1, b2);
    const float t2 = a * a * u1 / (1.f - u1);
    const float ct = rsqrtf(1.f + t2), st = sqrtf(t2) * ct;
    float sp, cp;
    sincosf(2.f * kPi * u2, &sp, &cp);
    return (st * cp) * b1 + (st * sp) * b2 + ct * h;
}

// Improved stochastic evaluation of f_p (rgb) for material 3: per lobe, the
// visible-normal sample n1 (u0, u1) and the lobe's own sampling reversed -- a
// GGX normal about the half vector (u2, u3) for the specular lobe, a normal
// cosine-distributed about wi (u4, u5) for the diffuse lobe -- combined by
// the one-sample balance heuristic.
__device__ inline V3 sggx_disney_est(const Sggx &g, V3 c, float rough, V3 wo, V3 wi, const float u[6]) {
    const float a = ggx_alpha(rough), so = sggx_sigma(g, wo);
    V3 f = v3(0.f, 0.f, 0.f), fs, fd;
    const V3 hs = wo + wi;
    const float hl2 = dot(hs, hs);
    const bool hok = hl2 > 0.f;
    const V3 h = hok ? rsqrtf(hl2) * hs : v3(0.f, 0.f, 1.f);
    const V3 n1 = sggx_sample_vndf(g, wo, u[0], u[1]);
    const float p1 = sggx_vndf(g, wo, n1, so);
    if (p1 > 0.f) {
        disney_base(c, rough, g.met, n1, wo, wi, fs, fd);
        const float hn = hok ? dot(h, n1) : 0.f;
        const float pm = hn > 0.f ? ggx_D(a, hn) * hn : 0.f;
        const float pc = fmaxf(0.f, dot(wi, n1)) * kInvPi;
        f = (p1 / (p1 + pm)) * fs + (p1 / (p1 + pc)) * fd;
    }
    if (hok) {
        const V3 n2 = ggx_ndf_about(h, a, u[2], u[3]);
        const float hn = dot(n2, h);
        const float p2 = hn > 0.f ? ggx_D(a, hn) * hn : 0.f;
        const float q2 = sggx_vndf(g, wo, n2, so);
        if (p2 > 0.f && q2 > 0.f) {
            disney_base(c, rough, g.met, n2, wo, wi, fs, fd);
            f = f + (q2 / (p2 + q2)) * fs;
        }
    }
    const V3 n3 = cosine_about(wi, u[4], u[5]);
    const float p3 = fmaxf(0.f, dot(n3, wi)) * kInvPi;
    const float q3 = sggx_vndf(g, wo, n3, so);
    if (p3 > 0.f && q3 > 0.f) {
        disney_base(c, rough, g.met, n3, wo, wi, fs, fd);
        f = f + (q3 / (p3 + q3)) * fd;
    }
    return f;
}

// Importance sampling of material 3: a visible normal n (u0, u1), then the
// base BSDF at n -- the specular lobe (GGX visible normals of n, reflected)
// with probability ps, else cosine about n -- chosen by v0, direction from
// (v1, v2).  wgt = base f / lobe-mixture pdf; false when no direction.
__device__ inline bool sggx_disney_sample(const Sggx &g, V3 c, float rough, V3 wo, float u0, float u1, float v0,
                                          float v1, float v2, V3 &wi, V3 &wgt) {
    wgt = v3(0.f, 0.f, 0.f);
    const V3 n = sggx_sample_vndf(g, wo, u0, u1);
    if (v0 < g.ps) {
        V3 b1, b2, w1;
        onb(n, b1, b2);
        float pd;
        const V3 li = phase_sample_local(1, v3(1.f, 1.f, 1.f), rough, v3(dot(wo, b1), dot(wo, b2), dot(wo, n)), v1,
                                         v2, w1, pd);
        if (!(pd > 0.f)) return false;
        wi = li.x * b1 + li.y * b2 + li.z * n;
    } else {
        wi = cosine_about(n, v1, v2);
    }
    const float co = dot(n, wo), ci = dot(n, wi);
    if (!(co > 0.f) || !(ci > 0.f)) return false;
    const float a = ggx_alpha(rough);
    const float pdf = g.ps * ggx_D(a, dot(n, normalize(wo + wi))) / ((1.f + ggx_lambda(a, co)) * 4.f * co) +
                      (1.f - g.ps) * ci * kInvPi;
    if (!(pdf > 0.f)) return false;
    V3 fs, fd;
    disney_base(c, rough, g.met, n, wo, wi, fs, fd);
    wgt = (1.f / pdf) * (fs + fd);
    return true;
}

// Approximate MIS pdf of material 3 (App. B): ps times the roughened SGGX's
// visible NDF at the half vector plus (1 - ps) <w_h . w_o> / pi.
__device__ __forceinline__ float sggx_disney_pdf_approx(const Sggx &gr, float ps, V3 wo, V3 wi) {
    const V3 hs = wo + wi;
    const float l2 = dot(hs, hs);
    if (!(l2 > 0.f)) return 0.f;
    const V3 h = rsqrtf(l2) * hs;
    return ps * sggx_vndf(gr, wo, h, sggx_sigma(gr, wo)) + (1.f - ps) * fmaxf(0.f, dot(h, wo)) * kInvPi;
}

// Camera set up on the host: origin, forward f, right r' = tan(vfov/2) aspect r,
// up u' = tan(vfov/2) u.
struct CamDev {
    float ox, oy, oz;
    float fx, fy, fz;
    float rx, ry, rz;
    float ux, uy, uz;
    int32_t width, height;
};
__device__ __forceinline__ V3 camera_dir(const CamDev &c, int px, int py, float jx, float jy) {
    const float sx = 2.f * ((float)px + jx) / (float)c.width - 1.f;
    const float sy = 1.f - 2.f * ((float)py + jy) / (float)c.height;
    return normalize(v3(c.fx + sx * c.rx + sy * c.ux, c.fy + sx * c.ry + sy * c.uy,
                        c.fz + sx * c.rz + sy * c.uz));
}

}  // namespace ugp
