// api.hip -- the C ABI of libugp (declared in include/ugp.h): host-side
// argument checks, the context, and dispatch to the kernels.  No C++ exception
// crosses this boundary; every failure is a ugp_status.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

#include "ugp_internal.hpp"

namespace ugp {

void *ctx_scratch(ugp_ctx ctx, size_t bytes) {
    if (ctx->scratch_bytes >= bytes) return ctx->scratch;
    hipStreamSynchronize(ctx->stream);
    hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
    const size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
    if (hipMalloc(&ctx->scratch, want) != hipSuccess) return nullptr;
    ctx->scratch_bytes = want;
    return ctx->scratch;
}

}  // namespace ugp

namespace {

ugp_status from_hip(hipError_t e) {
    if (e == hipSuccess) return UGP_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return UGP_ERR_OUT_OF_MEMORY;
    if (e == hipErrorInvalidValue) return UGP_ERR_INVALID_ARGUMENT;
    if (e == hipErrorNotSupported) return UGP_ERR_UNSUPPORTED;
    return UGP_ERR_DEVICE;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int d) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != d) hipSetDevice(d);
    }
    ~DeviceGuard() {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

bool query_args_ok(ugp_ctx ctx, int64_t n, const float *rays) {
    return ctx && n >= 0 && n < (int64_t(1) << 31) && (n == 0 || rays);
}

// Shared argument checks of the two vector-Jacobian products.
ugp_status vjp_args(ugp_ctx ctx, const ugp_scene *scene, int64_t n, const float *rays, const float *dout,
                    const float *grad) {
    if (!query_args_ok(ctx, n, rays) || (n > 0 && !dout) || !grad) return UGP_ERR_INVALID_ARGUMENT;
    if (!scene || !scene->scale || !scene->rotation) return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (scene->n != ctx->scene.n) return UGP_ERR_INVALID_ARGUMENT;
    return UGP_OK;
}

// Shared argument checks of the render entry points.
ugp_status render_args(ugp_ctx ctx, const ugp_camera *cam, const ugp_render_params *p) {
    if (!ctx || !cam || !p) return UGP_ERR_INVALID_ARGUMENT;
    if (cam->width < 1 || cam->height < 1 || (int64_t)cam->width * cam->height >= (int64_t(1) << 31) ||
        !(cam->vfov_deg > 0.f && cam->vfov_deg < 180.f))
        return UGP_ERR_INVALID_ARGUMENT;
    if (p->spp < 1 || p->max_depth < 0 || p->max_depth > 1000 || p->mis_mode < 0 || p->mis_mode > 2 ||
        p->sample_offset < 0 || p->sample_offset + p->spp > (int64_t(1) << 32))
        return UGP_ERR_INVALID_ARGUMENT;
    for (int c = 0; c < 3; ++c)
        if (!(p->env_radiance[c] >= 0.f) || !std::isfinite(p->env_radiance[c])) return UGP_ERR_INVALID_ARGUMENT;
    if (p->nrc_mode < 0 || p->nrc_mode > 3) return UGP_ERR_INVALID_ARGUMENT;
    if (p->nrc_mode != 0 && p->nrc_terminate_after < 1) return UGP_ERR_INVALID_ARGUMENT;
    if (p->nrc_mode == 1 && (p->nrc_train_records < 1 || p->nrc_train_records > (1 << 20)))
        return UGP_ERR_INVALID_ARGUMENT;
    if (!(p->nrc_lr >= 0.f) || !std::isfinite(p->nrc_lr)) return UGP_ERR_INVALID_ARGUMENT;
    if (p->nrc_train_steps < 0 || p->nrc_train_steps > 64) return UGP_ERR_INVALID_ARGUMENT;
    if (!(p->nrc_radiance_scale >= 0.f) || !std::isfinite(p->nrc_radiance_scale)) return UGP_ERR_INVALID_ARGUMENT;
    if (!(p->nrc_target_clamp >= 0.f) || !std::isfinite(p->nrc_target_clamp)) return UGP_ERR_INVALID_ARGUMENT;
    for (int k = 0; k < 6; ++k)
        if (!std::isfinite(p->nrc_box[k])) return UGP_ERR_INVALID_ARGUMENT;
    if (p->transport < 0 || p->transport > 1) return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    // the exponential variant is rendered without the radiance cache
    if (p->transport == 1 && p->nrc_mode != 0) return UGP_ERR_UNSUPPORTED;
    return UGP_OK;
}

}  // namespace

extern "C" {

const char *ugp_status_string(ugp_status s) {
    switch (s) {
        case UGP_OK: return "ok";
        case UGP_ERR_INVALID_ARGUMENT: return "invalid argument";
        case UGP_ERR_OUT_OF_MEMORY: return "out of device memory";
        case UGP_ERR_DEVICE: return "device error";
        case UGP_ERR_NO_SCENE: return "no scene has been built";
        case UGP_ERR_UNSUPPORTED: return "unsupported (device or scene)";
        case UGP_ERR_OVERFLOW: return "a per-ray buffer overflowed";
    }
    return "unknown status";
}

ugp_status ugp_create(int device, void *hip_stream, ugp_ctx *out) {
    if (!out) return UGP_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return UGP_ERR_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return UGP_ERR_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return UGP_ERR_UNSUPPORTED;
    DeviceGuard g(device);
    ugp_ctx c = new (std::nothrow) ugp_ctx_s();
    if (!c) return UGP_ERR_OUT_OF_MEMORY;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (hipMalloc((void **)&c->err, sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&c->stats, sizeof(int64_t) * 8) != hipSuccess) {
        hipFree(c->err);
        delete c;
        return UGP_ERR_OUT_OF_MEMORY;
    }
    hipMemset(c->err, 0, sizeof(uint32_t));
    hipMemset(c->stats, 0, sizeof(int64_t) * 8);
    // address of this device's copy of the allocation-free query's buffer
    // (a failure here only disables ugp_sample_collision_noalloc)
    (void)ugp::noalloc_init(device);
    *out = c;
    return UGP_OK;
}

ugp_status ugp_destroy(ugp_ctx ctx) {
    if (!ctx) return UGP_ERR_INVALID_ARGUMENT;
    DeviceGuard g(ctx->device);
    hipStreamSynchronize(ctx->stream);
    ugp::free_scene(ctx->scene);
    ugp::free_render(ctx);
    ugp::nrc_free(ctx);
    hipFree(ctx->scratch);
    hipFree(ctx->err);
    hipFree(ctx->stats);
    hipFree(ctx->counters);
    for (hipEvent_t ev : ctx->ev_pool) hipEventDestroy(ev);
    delete ctx;
    return UGP_OK;
}

ugp_status ugp_set_stream(ugp_ctx ctx, void *hip_stream) {
    if (!ctx) return UGP_ERR_INVALID_ARGUMENT;
    ctx->stream = (hipStream_t)hip_stream;
    return UGP_OK;
}

ugp_status ugp_build_bvh(ugp_ctx ctx, const ugp_scene *s, float eps) {
    if (!ctx || !s || s->n < 1 || s->n >= (int64_t(1) << 31) || !(eps > 0.f && eps < 1.f)) return UGP_ERR_INVALID_ARGUMENT;
    if (!s->mean || !s->scale || !s->rotation || !s->density || !s->albedo || !s->roughness ||
        !s->emission || !s->material)
        return UGP_ERR_INVALID_ARGUMENT;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::build_scene(ctx, s, eps));
}

ugp_status ugp_refit_bvh(ugp_ctx ctx, const ugp_scene *s) {
    if (!ctx || !s) return UGP_ERR_INVALID_ARGUMENT;
    if (!s->mean || !s->scale || !s->rotation || !s->density || !s->albedo || !s->roughness ||
        !s->emission || !s->material)
        return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (s->n != ctx->scene.n) return UGP_ERR_INVALID_ARGUMENT;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::refit_scene(ctx, s));
}

ugp_status ugp_transmittance(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *exclude, float *T,
                             float *F) {
    if (!query_args_ok(ctx, n, rays) || (n > 0 && !T)) return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::launch_transmittance(ctx, n, rays, exclude, T, F));
}

ugp_status ugp_sample_collision(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *exclude,
                                const float *u, int32_t *prim, float *t) {
    if (!query_args_ok(ctx, n, rays) || (n > 0 && (!u || !prim || !t))) return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::launch_sweep(ctx, ugp::kModeCollide, n, rays, exclude, u, nullptr, prim, t));
}

ugp_status ugp_sample_collision_noalloc(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *exclude,
                                        const float *u, int32_t *prim, float *t) {
    if (!query_args_ok(ctx, n, rays) || (n > 0 && (!u || !prim || !t))) return UGP_ERR_INVALID_ARGUMENT;
    if (n > UGP_NOALLOC_MAX_RAYS) return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    const hipError_t e = ugp::launch_sweep_noalloc(ctx, ugp::kModeCollide, n, rays, exclude, u, nullptr, prim, t);
    if (e == hipErrorNotInitialized) return UGP_ERR_DEVICE;
    return from_hip(e);
}

ugp_status ugp_ray_integral(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *prim, float *I_out) {
    if (!query_args_ok(ctx, n, rays) || (n > 0 && (!prim || !I_out))) return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::launch_ray_integral(ctx, n, rays, prim, I_out));
}

ugp_status ugp_philox(ugp_ctx ctx, int64_t n, const uint32_t *counters, uint64_t key, uint32_t *out) {
    if (!ctx || n < 0 || (n > 0 && (!counters || !out))) return UGP_ERR_INVALID_ARGUMENT;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::launch_philox(ctx, n, counters, key, out));
}

ugp_status ugp_saturation(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *exclude, float *tsat) {
    if (!query_args_ok(ctx, n, rays) || (n > 0 && !tsat)) return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::launch_sweep(ctx, ugp::kModeSaturate, n, rays, exclude, nullptr, nullptr, nullptr, tsat));
}

ugp_status ugp_emitter_query(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *exclude,
                             const int32_t *target, float *out) {
    if (!query_args_ok(ctx, n, rays) || (n > 0 && (!target || !out))) return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::launch_sweep(ctx, ugp::kModeEmitter, n, rays, exclude, nullptr, target, nullptr, out));
}

ugp_status ugp_trace_counts(ugp_ctx ctx, int mode, int64_t n, const float *rays, const int32_t *exclude,
                            const float *u, const int32_t *target, int32_t *counts) {
    if (!query_args_ok(ctx, n, rays) || (n > 0 && !counts) || mode < 0 || mode > 2) return UGP_ERR_INVALID_ARGUMENT;
    if (mode == ugp::kModeCollide && n > 0 && !u) return UGP_ERR_INVALID_ARGUMENT;
    if (mode == ugp::kModeEmitter && n > 0 && !target) return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    float *fo = nullptr;
    int32_t *po = nullptr;
    if (hipMallocAsync((void **)&fo, sizeof(float) * n, ctx->stream) != hipSuccess) return UGP_ERR_OUT_OF_MEMORY;
    if (hipMallocAsync((void **)&po, sizeof(int32_t) * n, ctx->stream) != hipSuccess) {
        hipFreeAsync(fo, ctx->stream);
        return UGP_ERR_OUT_OF_MEMORY;
    }
    hipError_t e = ugp::launch_sweep(ctx, mode, n, rays, exclude, u, target, po, fo, counts);
    hipFreeAsync(fo, ctx->stream);
    hipFreeAsync(po, ctx->stream);
    return from_hip(e);
}

ugp_status ugp_render(ugp_ctx ctx, const ugp_camera *cam, const ugp_render_params *p, float *sum,
                      float *sumsq) {
    if (!sum) return UGP_ERR_INVALID_ARGUMENT;
    const ugp_status s = render_args(ctx, cam, p);
    if (s != UGP_OK) return s;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::render(ctx, cam, p, sum, sumsq));
}

ugp_status ugp_render_grads(ugp_ctx ctx, const ugp_camera *cam, const ugp_render_params *p, const float *d_image,
                            float *grad_albedo, float *grad_roughness, float *grad_density, float *sum) {
    if (!d_image || !(grad_albedo || grad_roughness || grad_density)) return UGP_ERR_INVALID_ARGUMENT;
    const ugp_status s = render_args(ctx, cam, p);
    if (s != UGP_OK) return s;
    // the radiance cache and the exponential variant are refused by every
    // adjoint, material 3 by the shading ones
    if (p->nrc_mode != 0 || p->transport != 0 || ((grad_albedo || grad_roughness) && ctx->scene.has_mat3))
        return UGP_ERR_UNSUPPORTED;
    DeviceGuard g(ctx->device);
    ugp::RenderAdjoint adj{d_image};
    adj.grad_albedo = grad_albedo;
    adj.grad_roughness = grad_roughness;
    adj.grad_density = grad_density;
    return from_hip(ugp::render(ctx, cam, p, sum, nullptr, &adj));
}

ugp_status ugp_render_albedo_grad(ugp_ctx ctx, const ugp_camera *cam, const ugp_render_params *p,
                                  const float *d_image, float *grad_albedo, float *sum) {
    if (!grad_albedo) return UGP_ERR_INVALID_ARGUMENT;
    return ugp_render_grads(ctx, cam, p, d_image, grad_albedo, nullptr, nullptr, sum);
}

ugp_status ugp_render_roughness_grad(ugp_ctx ctx, const ugp_camera *cam, const ugp_render_params *p,
                                     const float *d_image, float *grad_roughness, float *sum) {
    if (!grad_roughness) return UGP_ERR_INVALID_ARGUMENT;
    return ugp_render_grads(ctx, cam, p, d_image, nullptr, grad_roughness, nullptr, sum);
}

ugp_status ugp_render_density_grad(ugp_ctx ctx, const ugp_camera *cam, const ugp_render_params *p,
                                   const float *d_image, float *grad_density, float *sum) {
    if (!grad_density) return UGP_ERR_INVALID_ARGUMENT;
    return ugp_render_grads(ctx, cam, p, d_image, nullptr, nullptr, grad_density, sum);
}

ugp_status ugp_exp_transmittance(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *exclude, float *T_out) {
    if (!query_args_ok(ctx, n, rays) || (n > 0 && !T_out)) return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::launch_exp(ctx, n, rays, exclude, false, 0, T_out, nullptr, nullptr));
}

ugp_status ugp_exp_sample_collision(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *exclude,
                                    uint64_t seed, int32_t *prim_out, float *t_out) {
    if (!query_args_ok(ctx, n, rays) || (n > 0 && (!prim_out || !t_out))) return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::launch_exp(ctx, n, rays, exclude, true, seed, nullptr, prim_out, t_out));
}

ugp_status ugp_accum_cdf(ugp_ctx ctx, const ugp_scene *scene, int64_t n, const float *rays,
                         const int32_t *exclude, const float *target, float loss_scale, float *C_out,
                         float *loss_out, float *grad) {
    if (!query_args_ok(ctx, n, rays) || !std::isfinite(loss_scale)) return UGP_ERR_INVALID_ARGUMENT;
    if ((loss_out || grad) && !target) return UGP_ERR_INVALID_ARGUMENT;
    if (grad && (!scene || !scene->scale || !scene->rotation || scene->n != ctx->scene.n))
        return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    return from_hip(
        ugp::accum_cdf(ctx, scene, n, rays, exclude, target, loss_scale, nullptr, false, C_out, loss_out, grad));
}

ugp_status ugp_rf_render(ugp_ctx ctx, const ugp_scene *scene, int64_t n, const float *rays, const int32_t *exclude,
                         const float *target, float loss_scale, float *L_out, float *loss_out, float *grad) {
    if (!query_args_ok(ctx, n, rays) || !std::isfinite(loss_scale)) return UGP_ERR_INVALID_ARGUMENT;
    if ((loss_out || grad) && !target) return UGP_ERR_INVALID_ARGUMENT;
    if (grad && (!scene || !scene->scale || !scene->rotation || scene->n != ctx->scene.n))
        return UGP_ERR_INVALID_ARGUMENT;
    if (ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    return from_hip(
        ugp::accum_cdf(ctx, scene, n, rays, exclude, target, loss_scale, nullptr, true, L_out, loss_out, grad));
}

ugp_status ugp_accum_cdf_backward(ugp_ctx ctx, const ugp_scene *scene, int64_t n, const float *rays,
                                  const int32_t *exclude, const float *dC, float *grad) {
    const ugp_status s = vjp_args(ctx, scene, n, rays, dC, grad);
    if (s != UGP_OK || n == 0) return s;
    DeviceGuard g(ctx->device);
    return from_hip(
        ugp::accum_cdf(ctx, scene, n, rays, exclude, nullptr, 0.f, dC, false, nullptr, nullptr, grad));
}

ugp_status ugp_rf_render_backward(ugp_ctx ctx, const ugp_scene *scene, int64_t n, const float *rays,
                                  const int32_t *exclude, const float *dL, float *grad) {
    const ugp_status s = vjp_args(ctx, scene, n, rays, dL, grad);
    if (s != UGP_OK || n == 0) return s;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::accum_cdf(ctx, scene, n, rays, exclude, nullptr, 0.f, dL, true, nullptr, nullptr, grad));
}

ugp_status ugp_camera_rays(ugp_ctx ctx, const ugp_camera *cam, uint64_t seed, int64_t sample, float *rays) {
    if (!ctx || !cam || !rays) return UGP_ERR_INVALID_ARGUMENT;
    if (cam->width < 1 || cam->height < 1 || (int64_t)cam->width * cam->height >= (int64_t(1) << 31) ||
        !(cam->vfov_deg > 0.f && cam->vfov_deg < 180.f) || sample < 0 || sample >= (int64_t(1) << 32))
        return UGP_ERR_INVALID_ARGUMENT;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::camera_rays(ctx, cam, seed, (uint32_t)sample, rays));
}

ugp_status ugp_fit_adam(ugp_ctx ctx, int64_t n, float *mean, float *scale, float *rotation, float *density,
                        float *emission, const float *grad, float *m, float *v, int32_t step, const float lr[5],
                        float min_scale) {
    if (!ctx || n < 0 || step < 1 || !lr || !(min_scale > 0.f) || !std::isfinite(min_scale))
        return UGP_ERR_INVALID_ARGUMENT;
    for (int k = 0; k < (emission ? 5 : 4); ++k)
        if (!(lr[k] >= 0.f) || !std::isfinite(lr[k])) return UGP_ERR_INVALID_ARGUMENT;
    if (n > 0 && (!mean || !scale || !rotation || !density || !grad || !m || !v)) return UGP_ERR_INVALID_ARGUMENT;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::fit_adam(ctx, n, mean, scale, rotation, density, emission, grad, m, v, step, lr, 0.9f,
                                  0.999f, 1e-8f, min_scale));
}

ugp_status ugp_sggx_phase(ugp_ctx ctx, int64_t n, const float *sggx, const float *base, const float *dirs,
                          const float *u, float *out) {
    if (!ctx || n < 0) return UGP_ERR_INVALID_ARGUMENT;
    if (n == 0) return UGP_OK;
    if (!sggx || !dirs || !u || !out) return UGP_ERR_INVALID_ARGUMENT;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::sggx_phase(ctx, n, sggx, base, dirs, u, out));
}

ugp_status ugp_sync(ugp_ctx ctx) {
    if (!ctx) return UGP_ERR_INVALID_ARGUMENT;
    DeviceGuard g(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return from_hip(e);
    uint32_t h = 0;
    e = hipMemcpy(&h, ctx->err, sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return from_hip(e);
    if (h) {
        hipMemset(ctx->err, 0, sizeof(uint32_t));
        return (h & ugp::kErrRay) ? UGP_ERR_INVALID_ARGUMENT : UGP_ERR_OVERFLOW;
    }
    return UGP_OK;
}

ugp_status ugp_set_profiling(ugp_ctx ctx, int level) {
    if (!ctx || level < 0 || level > 2) return UGP_ERR_INVALID_ARGUMENT;
    if (level >= 2 && !ctx->counters) {
        DeviceGuard g(ctx->device);
        if (hipMalloc((void **)&ctx->counters, sizeof(unsigned long long) * 12) != hipSuccess)
            return UGP_ERR_OUT_OF_MEMORY;
    }
    ctx->profiling = level;
    return UGP_OK;
}

ugp_status ugp_set_path_pool(ugp_ctx ctx, int64_t slots) {
    if (!ctx || slots < 0 || (slots > 0 && slots < 64)) return UGP_ERR_INVALID_ARGUMENT;
    ctx->path_pool = slots;
    return UGP_OK;
}

ugp_status ugp_set_tail_paths(ugp_ctx ctx, int64_t paths) {
    if (!ctx || paths < 0) return UGP_ERR_INVALID_ARGUMENT;
    ctx->tail_paths = paths;
    return UGP_OK;
}

ugp_status ugp_get_render_stats(ugp_ctx ctx, ugp_render_stats *out) {
    if (!ctx || !out) return UGP_ERR_INVALID_ARGUMENT;
    DeviceGuard g(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    int64_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpy(h, ctx->stats, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return from_hip(e);
    std::memset(out, 0, sizeof(*out));
    out->paths = ctx->last_paths;
    out->collision_rays = h[0];
    out->light_rays = h[1];
    out->env_rays = h[2];
    out->nrc_queries = h[3];
    out->nrc_records = h[4];
    out->nrc_loss = NAN;
    if (const float *lp = ugp::render_nrc_loss(ctx)) {
        float l = NAN;
        if (hipMemcpy(&l, lp, sizeof(float), hipMemcpyDeviceToHost) == hipSuccess) out->nrc_loss = l;
    }
    out->node_visits = out->prim_tests = out->prim_reloads = -1;
    for (int c = 0; c < 4; ++c) out->cat_nodes[c] = out->cat_prims[c] = out->cat_reloads[c] = -1;
    if (ctx->profiling >= 2 && ctx->counters) {
        unsigned long long c[12];
        e = hipMemcpy(c, ctx->counters, sizeof(c), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return from_hip(e);
        out->node_visits = out->prim_tests = out->prim_reloads = 0;
        for (int k = 0; k < 4; ++k) {
            out->cat_nodes[k] = (int64_t)c[3 * k];
            out->cat_prims[k] = (int64_t)c[3 * k + 1];
            out->cat_reloads[k] = (int64_t)c[3 * k + 2];
            out->node_visits += out->cat_nodes[k];
            out->prim_tests += out->cat_prims[k];
            out->prim_reloads += out->cat_reloads[k];
        }
    }
    out->ms_collide = out->ms_collide_wide = out->ms_light = out->ms_env = out->ms_shade = out->ms_sort = -1.0;
    out->ms_nrc_infer = out->ms_nrc_train = out->ms_tail = -1.0;
    if (ctx->ev_cat_valid) {
        double ms[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        int cnt[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (const auto &u : ctx->ev_used) {
            float t = 0.f;
            if (u.first >= 0 && u.first < 9 &&
                hipEventElapsedTime(&t, ctx->ev_pool[u.second], ctx->ev_pool[u.second + 1]) == hipSuccess) {
                ms[u.first] += t;
                cnt[u.first] += 1;
            }
        }
        out->ms_collide = ms[0];
        out->ms_collide_wide = ms[1];
        out->ms_light = ms[2];
        out->ms_env = ms[3];
        out->ms_shade = ms[4];
        out->ms_sort = ms[5];
        out->ms_nrc_infer = ms[6];
        out->ms_nrc_train = ms[7];
        out->ms_tail = ms[8];
        out->launches_collide = cnt[0];
        out->launches_light = cnt[2];
        out->launches_env = cnt[3];
    }
    return UGP_OK;
}

int32_t ugp_nrc_num_params(void) { return ugp::nrc_num_params(); }

ugp_status ugp_nrc_set_weights(ugp_ctx ctx, const float *weights) {
    if (!ctx || !weights) return UGP_ERR_INVALID_ARGUMENT;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::nrc_set_weights(ctx, weights));
}

ugp_status ugp_nrc_get_weights(ugp_ctx ctx, float *weights_out) {
    if (!ctx || !weights_out || !ugp::nrc_ready(ctx)) return UGP_ERR_INVALID_ARGUMENT;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::nrc_get_weights(ctx, weights_out));
}

ugp_status ugp_nrc_encode(ugp_ctx ctx, int64_t n, const float *inputs, const float *box, float *feat_out) {
    if (!ctx || n < 0 || n > (int64_t(1) << 28) || (n > 0 && (!inputs || !feat_out))) return UGP_ERR_INVALID_ARGUMENT;
    if (!box && ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::nrc_encode(ctx, n, inputs, 16, box, feat_out));
}

ugp_status ugp_nrc_forward(ugp_ctx ctx, int64_t n, const float *x, int32_t x_kind, const float *box,
                           float *y_out) {
    if (!ctx || n < 0 || n > (int64_t(1) << 28) || x_kind < 0 || x_kind > 1 || (n > 0 && (!x || !y_out)))
        return UGP_ERR_INVALID_ARGUMENT;
    if (x_kind == 0 && !box && ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    if (n == 0) return UGP_OK;
    DeviceGuard g(ctx->device);
    hipError_t e = ugp::nrc_ensure(ctx);
    if (e == hipSuccess) e = ugp::nrc_forward(ctx, n, nullptr, x, x_kind == 0 ? 16 : 96, x_kind, box, y_out, nullptr);
    return from_hip(e);
}

ugp_status ugp_nrc_train_step(ugp_ctx ctx, int64_t n, const float *x, int32_t x_kind, const float *box,
                              const float *targets, float lr, float *loss_out, float *grad_out) {
    if (!ctx || n < 1 || n > (int64_t(1) << 22) || x_kind < 0 || x_kind > 1 || !x || !targets ||
        !(lr >= 0.f) || !std::isfinite(lr))
        return UGP_ERR_INVALID_ARGUMENT;
    if (x_kind == 0 && !box && ctx->scene.n == 0) return UGP_ERR_NO_SCENE;
    DeviceGuard g(ctx->device);
    hipError_t e = ugp::nrc_ensure(ctx);
    if (e == hipSuccess)
        e = ugp::nrc_train_step(ctx, n, nullptr, x, x_kind == 0 ? 16 : 96, x_kind, box, targets, lr, loss_out,
                                grad_out);
    return from_hip(e);
}

ugp_status ugp_nrc_records(ugp_ctx ctx, int64_t cap, float *records_out, float *targets_out, int64_t *count_out) {
    if (!ctx || cap < 0 || !count_out || (cap > 0 && !records_out)) return UGP_ERR_INVALID_ARGUMENT;
    DeviceGuard g(ctx->device);
    return from_hip(ugp::render_nrc_records(ctx, cap, records_out, targets_out, count_out));
}

}  // extern "C"
