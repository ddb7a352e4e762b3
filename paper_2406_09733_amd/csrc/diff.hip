// diff.hip -- differentiation of the accumulated free-flight CDF of a ray
// (Sec. 7.2, eq. accum_cdf) with respect to every primitive parameter, the
// transmittance-image loss built on it, jittered camera rays for such images,
// and the Adam update with the clamps of the transmittance optimisation.
//
// C = sum_k 1/2 I_k(a_k, min(b_k, t_sat)) over the primitives the ray meets,
// each clipped at the ray's saturating distance (t1 when the ray never
// saturates).  As in Sec. 7.2 the derivative of C with respect to a parameter
// of primitive k is the derivative of its own term with t_sat held fixed.
#include "trace_device.hpp"

namespace ugp {
namespace {

// 1/2 I(a, min(b, tcl)) of the primitive of record h along ray r, and its
// gradient with respect to (mu[3], M[3][3] row-major, d) = g[13], for the clip
// point tcl held fixed.  The closed form of the ray integral (Sec. 4.1, eq.
// ray_integral), in the unit frame o' = M (o - mu), w' = M w:
//   A = w'.w', P = o'.w', t_c = -P / A, rho^2 = o'.o' - P^2 / A,
//   tau(t) = sqrt(A / 2) (t - t_c),
//   1/2 I = 1/2 d sqrt(pi / (2 A)) exp(-rho^2 / 2) [erf tau_b - erf tau_a].
// An end on the cut-off ellipsoid has |tau| = sqrt((r^2 - rho^2) / 2) (it moves
// with the parameters); an end clipped at t0 or at tcl has tau(t) at that t.
// Plain FP64 throughout (few primitives per ray; the sum C itself comes from
// the traversal's chord, as in every other query).
__device__ double w_and_grad(const HotRec &h, const RayD &r, double r2, double tcl, double g[13]) {
    for (int k = 0; k < 13; ++k) g[k] = 0.0;
    const double M[9] = {h.m[0], h.m[1], h.m[2], h.m[3], h.m[4], h.m[5], h.m[6], h.m[7], h.m[8]};
    const double p[3] = {(double)r.ox - (double)h.mx, (double)r.oy - (double)h.my, (double)r.oz - (double)h.mz};
    const double w[3] = {r.dx, r.dy, r.dz};
    double op[3], wp[3];
    for (int i = 0; i < 3; ++i) {
        op[i] = M[3 * i] * p[0] + M[3 * i + 1] * p[1] + M[3 * i + 2] * p[2];
        wp[i] = M[3 * i] * w[0] + M[3 * i + 1] * w[1] + M[3 * i + 2] * w[2];
    }
    const double A = wp[0] * wp[0] + wp[1] * wp[1] + wp[2] * wp[2];
    const double P = op[0] * wp[0] + op[1] * wp[1] + op[2] * wp[2];
    if (!(A > 0.0)) return 0.0;
    const double tc = -P / A;
    const double rho2 = op[0] * op[0] + op[1] * op[1] + op[2] * op[2] - P * P / A;
    if (!(rho2 < r2)) return 0.0;
    const double half = sqrt((r2 - rho2) / A);
    const double tlo = tc - half, thi = tc + half;
    const double a = fmax((double)r.t0, tlo), b = fmin(fmin(r.t1, thi), tcl);
    if (!(a < b)) return 0.0;
    const bool clip_a = a > tlo, clip_b = b < thi;
    const double s = sqrt(0.5 * A), q = sqrt(0.5 * (r2 - rho2));
    const double ta = clip_a ? s * (a - tc) : -q, tb = clip_b ? s * (b - tc) : q;
    const double base = sqrt(M_PI / (2.0 * A)) * exp(-0.5 * rho2);
    const double d = h.d, pref = d * base;
    const double E = erf(tb) - erf(ta);
    const double W = 0.5 * pref * E;
    // gradients of the scalars with respect to o' and w'
    double tc_o[3], tc_w[3], r_o[3], r_w[3], ta_o[3], ta_w[3], tb_o[3], tb_w[3], W_o[3], W_w[3];
    const double ka = 2.0 / sqrt(M_PI) * exp(-ta * ta), kb = 2.0 / sqrt(M_PI) * exp(-tb * tb);
    for (int i = 0; i < 3; ++i) {
        tc_o[i] = -wp[i] / A;
        tc_w[i] = -op[i] / A + 2.0 * P * wp[i] / (A * A);
        r_o[i] = 2.0 * op[i] - 2.0 * P * wp[i] / A;
        r_w[i] = -2.0 * P * op[i] / A + 2.0 * P * P * wp[i] / (A * A);
        const double s_w = wp[i] / (2.0 * s);
        if (clip_a) {
            ta_o[i] = -s * tc_o[i];
            ta_w[i] = s_w * (a - tc) - s * tc_w[i];
        } else {
            ta_o[i] = -r_o[i] / (4.0 * ta);
            ta_w[i] = -r_w[i] / (4.0 * ta);
        }
        if (clip_b) {
            tb_o[i] = -s * tc_o[i];
            tb_w[i] = s_w * (b - tc) - s * tc_w[i];
        } else {
            tb_o[i] = -r_o[i] / (4.0 * tb);
            tb_w[i] = -r_w[i] / (4.0 * tb);
        }
        const double lp_o = -0.5 * r_o[i], lp_w = -wp[i] / A - 0.5 * r_w[i];
        W_o[i] = 0.5 * pref * (E * lp_o + kb * tb_o[i] - ka * ta_o[i]);
        W_w[i] = 0.5 * pref * (E * lp_w + kb * tb_w[i] - ka * ta_w[i]);
    }
    // o' = M (o - mu), w' = M w
    for (int j = 0; j < 3; ++j) g[j] = -(M[j] * W_o[0] + M[3 + j] * W_o[1] + M[6 + j] * W_o[2]);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) g[3 + 3 * i + j] = W_o[i] * p[j] + W_w[i] * w[j];
    g[12] = 0.5 * base * E;
    return W;
}

// One lane per ray.  RGB = false: C (eq. accum_cdf), and with a target the
// loss loss_scale * (C - target)^2 and its gradient with respect to (mu, M, d)
// of every primitive the ray meets before t_sat, accumulated per original
// index (13 floats per primitive).  RGB = true, the radiance-field mode
// (Sec. 8, eq. rf): L = sum_k W_k L_e,k with the emission of the scene, the
// loss loss_scale * |L - target|^2 and its gradient with respect to
// (mu, M, d, L_e) (16 floats per primitive): the shape terms are the same
// derivative of W_k, weighted by dLoss/dL . L_e,k.  With dout (a caller's
// dLoss/dC or dLoss/dL per ray) instead of a target, that is the weight and
// no loss is formed; the first traversal then runs only for `out`.
template <bool RGB>
__global__ __launch_bounds__(kBlock) void k_cdf(SceneDev S, int64_t n, const float *rays, const int32_t *excl,
                                                const double *tsat, const float *target, float loss_scale,
                                                const float *dout, float *out, float *loss, float *g,
                                                uint32_t *err) {
    constexpr int kG = RGB ? 16 : 13;
    __shared__ int stack[kStackSize * kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    float l2 = 0.f;
    // a ray that failed validation in the saturation sweep has a NaN t_sat:
    // NaN outputs, no loss or gradient
    const bool bad = i < n && isnan(tsat[i]);
    if (bad && out)
        for (int k = 0; k < (RGB ? 3 : 1); ++k) out[(RGB ? 3 : 1) * i + k] = __builtin_nanf("");
    if (i < n && !bad) {
        const RayD r = load_ray(rays, i);
        const int ex = excl ? excl[i] : -1;
        const double tcl = tsat[i];
        const float hi = tcl < 3.0e38 ? (float)tcl : kInf;
        TraceCount tc;
        int spill[kStackSpill];
        auto pre = [&](int p) __attribute__((always_inline)) {
            const HotRec h = load_hot(S.hot, p);
            return h.orig != ex && !surely_missed(h, r, S.r2);
        };
        float acc[3] = {0.f, 0.f, 0.f};
        if (out || target) {
            TravState ts;
            trav_begin(ts, S);
            traverse(S, r, r.t0, [&]() __attribute__((always_inline)) { return hi; }, stack, spill, ts, 0, err, tc,
                     pre, [&](int p) __attribute__((always_inline)) {
                         const HotRec h = load_hot(S.hot, p);
                         Chord c;
                         if (!chord(h, r, S.r2, c, true) || !c.own) return false;
                         const float w = half_integral_to(c, tcl);
                         if (RGB) {
                             const float4 e = S.cold[3 * (int64_t)h.orig + 2];
                             acc[0] += w * e.x; acc[1] += w * e.y; acc[2] += w * e.z;
                         } else {
                             acc[0] += w;
                         }
                         return false;
                     });
        }
        constexpr int nc = RGB ? 3 : 1;
        if (out)
            for (int k = 0; k < nc; ++k) out[nc * i + k] = acc[k];
        if (target || dout) {
            double dL[3] = {0.0, 0.0, 0.0};
            bool any = false;
            for (int k = 0; k < nc; ++k) {
                if (dout) {
                    dL[k] = (double)dout[nc * i + k];
                } else {
                    const float diff = acc[k] - target[nc * i + k];
                    l2 += loss_scale * diff * diff;
                    dL[k] = 2.0 * (double)loss_scale * (double)diff;
                }
                any = any || dL[k] != 0.0;
            }
            if (g && any) {
                TravState ts;
                trav_begin(ts, S);
                traverse(S, r, r.t0, [&]() __attribute__((always_inline)) { return hi; }, stack, spill, ts, 0, err,
                         tc, pre, [&](int p) __attribute__((always_inline)) {
                             const HotRec h = load_hot(S.hot, p);
                             Chord c;
                             if (!chord(h, r, S.r2, c, true) || !c.own) return false;
                             double gk[13];
                             const double W = w_and_grad(h, r, (double)S.r2, tcl, gk);
                             float *dst = g + kG * (int64_t)h.orig;
                             double wt = dL[0];
                             if (RGB) {
                                 const float4 e = S.cold[3 * (int64_t)h.orig + 2];
                                 wt = dL[0] * e.x + dL[1] * e.y + dL[2] * e.z;
                                 for (int k = 0; k < 3; ++k)
                                     if (W != 0.0 && dL[k] != 0.0) atomicAdd(dst + 13 + k, (float)(dL[k] * W));
                             }
                             if (wt != 0.0)
                                 for (int k = 0; k < 13; ++k)
                                     if (gk[k] != 0.0) atomicAdd(dst + k, (float)(wt * gk[k]));
                             return false;
                         });
            }
        }
    }
    if (loss) {
        for (int off = 32; off > 0; off >>= 1) l2 += __shfl_xor(l2, off);
        if ((threadIdx.x & 63) == 0 && l2 != 0.f) atomicAdd(loss, l2);
    }
}

// Chain rule from (mu, M, d) to the primitive parameters (mu, s, q, d): with
// the rotation of the unit quaternion q / |q| (the normalisation included),
// M = S^-1 R^T, M_ij = R_ji / s_i.  grad [n][11] = (mu, s, q, d) is added to;
// with emission gradients (gin rows of 16) grad rows are 14, the last three
// the emission's.
__global__ void k_cdf_chain(int64_t n, const float *scale, const float *rot, const float *gin, bool rgb,
                            float *grad) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float *g = gin + (rgb ? 16 : 13) * k;
    const double qw = rot[4 * k], qx = rot[4 * k + 1], qy = rot[4 * k + 2], qz = rot[4 * k + 3];
    const double nq = qw * qw + qx * qx + qy * qy + qz * qz;
    const double t = 2.0 / nq;
    // R = I + t Q(q)
    const double Q[3][3] = {{-(qy * qy + qz * qz), qx * qy - qw * qz, qx * qz + qw * qy},
                            {qx * qy + qw * qz, -(qx * qx + qz * qz), qy * qz - qw * qx},
                            {qx * qz - qw * qy, qy * qz + qw * qx, -(qx * qx + qy * qy)}};
    // dQ_ij / d(w, x, y, z)
    const double dQ[4][3][3] = {
        {{0, -qz, qy}, {qz, 0, -qx}, {-qy, qx, 0}},
        {{0, qy, qz}, {qy, -2 * qx, -qw}, {qz, qw, -2 * qx}},
        {{-2 * qy, qx, qw}, {qx, 0, qz}, {-qw, qz, -2 * qy}},
        {{-2 * qz, -qw, qx}, {qw, -2 * qz, qy}, {qx, qy, 0}}};
    const double qa[4] = {qw, qx, qy, qz};
    double R[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] = (i == j ? 1.0 : 0.0) + t * Q[i][j];
    const double s[3] = {scale[3 * k], scale[3 * k + 1], scale[3 * k + 2]};
    double gs[3], gR[3][3];
    for (int i = 0; i < 3; ++i) {
        gs[i] = 0.0;
        for (int j = 0; j < 3; ++j) {
            const double gm = g[3 + 3 * i + j];
            gs[i] -= gm * R[j][i] / (s[i] * s[i]);
            gR[j][i] = gm / s[i];
        }
    }
    double gq[4];
    for (int a = 0; a < 4; ++a) {
        double acc = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) acc += gR[i][j] * t * (dQ[a][i][j] - 2.0 * qa[a] * Q[i][j] / nq);
        gq[a] = acc;
    }
    float *o = grad + (rgb ? 14 : 11) * k;
    o[0] += g[0]; o[1] += g[1]; o[2] += g[2];
    o[3] += (float)gs[0]; o[4] += (float)gs[1]; o[5] += (float)gs[2];
    o[6] += (float)gq[0]; o[7] += (float)gq[1]; o[8] += (float)gq[2]; o[9] += (float)gq[3];
    o[10] += g[12];
    if (rgb) {
        o[11] += g[13]; o[12] += g[14]; o[13] += g[15];
    }
}

// Jittered pinhole rays, one per pixel: jitter from the counter-based
// generator of sample `sample` (the renderer's camera paths use the same
// stream), origin the camera, t in [0, inf).
__global__ void k_camera_rays(CamDev cam, uint64_t seed, uint32_t sample, float *rays) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npix = (int64_t)cam.width * cam.height;
    if (i >= npix) return;
    const int px = (int)(i % cam.width), py = (int)(i / cam.width);
    const Rng4 g = rng4(seed, (uint32_t)i, sample, 0, 0);
    const V3 d = camera_dir(cam, px, py, g.u[0], g.u[1]);
    float4 *o = reinterpret_cast<float4 *>(rays) + 2 * i;
    o[0] = make_float4(cam.ox, cam.oy, cam.oz, d.x);
    o[1] = make_float4(d.y, d.z, 0.f, __builtin_huge_valf());
}

// Adam on the primitive parameters (the transmittance optimisation of
// Sec. 7.2): gradient [n][11] = (mu, s, q, d), moments m, v of the same
// layout, step `t` (from 1).  Means, rotations and densities take plain Adam
// steps (rates lr_mean, lr_rot, lr_dens); scales take them on log s (the
// moments are of s dL/ds, the update multiplies s by exp(-step)), so a rate
// is relative to each primitive's own extent -- thin axes are orders of
// magnitude below the others.  With emission (rows of 14: the radiance-field
// mode) the emissions take plain steps at lr_emis.  Then, as in Sec. 7.2,
// scales are clamped to at least s_min, densities and emissions to at least
// 0, rotations renormalised.
__global__ void k_fit_adam(int64_t n, float *mean, float *scale, float *rot, float *dens, float *emis,
                           const float *grad, float *m, float *v, int t, float lr_mean, float lr_log_scale,
                           float lr_rot, float lr_dens, float lr_emis, float b1, float b2, float eps, float s_min) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int np = emis ? 14 : 11;
    float *prm[14] = {mean + 3 * k, mean + 3 * k + 1, mean + 3 * k + 2, scale + 3 * k, scale + 3 * k + 1,
                      scale + 3 * k + 2, rot + 4 * k, rot + 4 * k + 1, rot + 4 * k + 2, rot + 4 * k + 3, dens + k,
                      emis ? emis + 3 * k : nullptr, emis ? emis + 3 * k + 1 : nullptr,
                      emis ? emis + 3 * k + 2 : nullptr};
    const double c1 = 1.0 - pow((double)b1, t), c2 = 1.0 - pow((double)b2, t);
    for (int j = 0; j < np; ++j) {
        const int64_t e = np * k + j;
        const bool is_scale = j >= 3 && j < 6;
        const float g = is_scale ? grad[e] * *prm[j] : grad[e];
        const float mj = b1 * m[e] + (1.f - b1) * g;
        const float vj = b2 * v[e] + (1.f - b2) * g * g;
        m[e] = mj;
        v[e] = vj;
        const double step = (mj / c1) / (sqrt(vj / c2) + eps);
        if (is_scale) {
            *prm[j] = (float)((double)*prm[j] * exp(-(double)lr_log_scale * step));
        } else {
            const float rate = j < 3 ? lr_mean : (j < 10 ? lr_rot : (j == 10 ? lr_dens : lr_emis));
            *prm[j] -= (float)(rate * step);
        }
    }
    for (int j = 0; j < 3; ++j) scale[3 * k + j] = fmaxf(scale[3 * k + j], s_min);
    dens[k] = fmaxf(dens[k], 0.f);
    if (emis)
        for (int j = 0; j < 3; ++j) emis[3 * k + j] = fmaxf(emis[3 * k + j], 0.f);
    const float qn = sqrtf(rot[4 * k] * rot[4 * k] + rot[4 * k + 1] * rot[4 * k + 1] +
                           rot[4 * k + 2] * rot[4 * k + 2] + rot[4 * k + 3] * rot[4 * k + 3]);
    if (qn > 0.f)
        for (int j = 0; j < 4; ++j) rot[4 * k + j] /= qn;
    else
        rot[4 * k] = 1.f;
}

}  // namespace

hipError_t accum_cdf(ugp_ctx ctx, const ugp_scene *scene, int64_t n, const float *rays, const int32_t *excl,
                     const float *target, float loss_scale, const float *dout, bool rgb, float *out, float *loss,
                     float *grad) {
    const bool backward = target || dout;
    hipStream_t st = ctx->stream;
    const SceneDev &S = ctx->scene;
    const int kg = rgb ? 16 : 13;
    double *tsat = nullptr;
    float *gtmp = nullptr;
    hipError_t e = hipMallocAsync((void **)&tsat, sizeof(double) * (size_t)n, st);
    if (e != hipSuccess) return e;
    if (grad) {
        e = hipMallocAsync((void **)&gtmp, sizeof(float) * kg * (size_t)S.n, st);
        if (e == hipSuccess) e = hipMemsetAsync(gtmp, 0, sizeof(float) * kg * (size_t)S.n, st);
    }
    if (e == hipSuccess)
        e = launch_sweep(ctx, kModeSaturate, n, rays, excl, nullptr, nullptr, nullptr, nullptr, nullptr, tsat);
    if (e == hipSuccess) {
        const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
        if (rgb)
            hipLaunchKernelGGL(k_cdf<true>, grid, dim3(kBlock), 0, st, S, n, rays, excl, (const double *)tsat, target,
                               loss_scale, dout, out, target ? loss : nullptr, backward ? gtmp : nullptr, ctx->err);
        else
            hipLaunchKernelGGL(k_cdf<false>, grid, dim3(kBlock), 0, st, S, n, rays, excl, (const double *)tsat,
                               target, loss_scale, dout, out, target ? loss : nullptr, backward ? gtmp : nullptr,
                               ctx->err);
        e = hipGetLastError();
    }
    if (e == hipSuccess && grad && backward) {
        hipLaunchKernelGGL(k_cdf_chain, dim3((unsigned)((S.n + 255) / 256)), dim3(256), 0, st, S.n, scene->scale,
                           scene->rotation, (const float *)gtmp, rgb, grad);
        e = hipGetLastError();
    }
    hipFreeAsync(tsat, st);
    if (gtmp) hipFreeAsync(gtmp, st);
    return e;
}

hipError_t camera_rays(ugp_ctx ctx, const ugp_camera *cam, uint64_t seed, uint32_t sample, float *rays) {
    CamDev c;
    make_cam_dev(cam, &c);
    const int64_t npix = (int64_t)cam->width * cam->height;
    hipLaunchKernelGGL(k_camera_rays, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, ctx->stream, c, seed,
                       sample, rays);
    return hipGetLastError();
}

hipError_t fit_adam(ugp_ctx ctx, int64_t n, float *mean, float *scale, float *rot, float *dens, float *emis,
                    const float *grad, float *m, float *v, int t, const float lr[5], float b1, float b2, float eps,
                    float s_min) {
    hipLaunchKernelGGL(k_fit_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, n, mean, scale,
                       rot, dens, emis, grad, m, v, t, lr[0], lr[1], lr[2], lr[3], emis ? lr[4] : 0.f, b1, b2, eps,
                       s_min);
    return hipGetLastError();
}

}  // namespace ugp
