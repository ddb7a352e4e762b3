// trace.hip -- per-ray scene queries exported through the C ABI:
// transmittance, primitive-level free-flight sampling, saturating distance and
// the emitter (light-sampling) query.  One lane per ray, one wave64 per block,
// the traversal stack in LDS.  Rays whose event buffer overflows in the main
// (register) sweep are queued and re-run by a wide sweep.
#include "trace_device.hpp"

namespace ugp {
namespace {

__global__ __launch_bounds__(kBlock) void k_transmittance(SceneDev S, int64_t n, const float *rays,
                                                          const int32_t *excl, float *T, float *F,
                                                          uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const RayD r = load_ray(rays, i);
    TraceCount tc;
    const float f = transmittance_F(S, r, excl ? excl[i] : -1, F == nullptr, stack, err, tc);
    T[i] = fmaxf(0.f, 1.f - f);
    if (F) F[i] = f;
}

struct SweepArgs {
    int mode;
    int64_t n;
    const float *rays;
    const int32_t *excl;
    const float *u;
    const int32_t *target;
    int32_t *prim_out;
    float *f_out;
    int32_t *ovf_list;   // rays that overflowed the main buffer
    int32_t *ovf_count;
    int32_t *counts;     // optional [n][4] per-ray traversal counters
    double *td_out;      // optional: saturate mode, t_sat in full precision
};

// emitter mode: clip the ray at the exit of the target's chord
__device__ __forceinline__ bool emitter_ray(const SceneDev &S, RayD &r, int target, int excl, float &entry) {
    if (target < 0 || target >= S.n || target == excl) return false;
    const HotRec h = load_hot(S.hot, S.inv[target]);
    Chord c;
    if (!chord(h, r, S.r2, c)) return false;
    r.t1 = c.bd;  // the exit in full precision (the float b is rounded)
    entry = c.a;
    return true;
}

template <int K>
__device__ __forceinline__ void run_sweep(const SceneDev &S, const SweepArgs &A, int64_t i, int *stack,
                                          uint32_t *err, bool wide) {
    RayD r = load_ray(A.rays, i);
    const int ex = A.excl ? A.excl[i] : -1;
    int target = -1;
    float entry = -__builtin_huge_valf();
    if (A.mode == kModeEmitter) {
        target = A.target[i];
        if (!emitter_ray(S, r, target, ex, entry)) {
            A.f_out[i] = 0.f;
            return;
        }
    }
    const float u = A.u ? A.u[i] : 0.f;
    TraceCount tc;
    const SweepOut o = sweep<K>(S, r, ex, A.mode, u, target, stack, err, tc, entry);
    if (A.counts) {
        int32_t *c = A.counts + 4 * i;
        if (wide) {  // add to the main pass's counts
            c[0] += (int32_t)tc.nodes; c[1] += (int32_t)tc.prims; c[2] += (int32_t)tc.reloads;
            c[3] += (int32_t)tc.rounds;
        } else {
            c[0] = (int32_t)tc.nodes; c[1] = (int32_t)tc.prims; c[2] = (int32_t)tc.reloads;
            c[3] = (int32_t)tc.rounds;
        }
    }
    if (o.status != 0) {
        if (!wide) {
            const int slot = atomicAdd(A.ovf_count, 1);
            A.ovf_list[slot] = (int32_t)i;
        } else {
            atomicOr(err, kErrEvents);
        }
        if (A.prim_out) A.prim_out[i] = -1;
        if (A.f_out) A.f_out[i] = __builtin_nanf("");
        if (A.td_out) A.td_out[i] = __builtin_nan("");
        return;
    }
    if (A.prim_out) A.prim_out[i] = o.prim;
    if (A.f_out) A.f_out[i] = o.t;
    if (A.td_out) A.td_out[i] = o.td;
}

__global__ __launch_bounds__(kBlock, 2) void k_sweep_main(SceneDev S, SweepArgs A, uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= A.n) return;
    run_sweep<kEventsMain>(S, A, i, stack, err, false);
}

__global__ __launch_bounds__(kBlock) void k_sweep_wide(SceneDev S, SweepArgs A, uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= *A.ovf_count) return;
    run_sweep<kEventsWide>(S, A, A.ovf_list[j], stack, err, true);
}

}  // namespace

hipError_t launch_transmittance(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *excl, float *T,
                                float *F) {
    const unsigned g = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_transmittance, dim3(g), dim3(kBlock), 0, ctx->stream, ctx->scene, n, rays, excl, T,
                       F, ctx->err);
    return hipGetLastError();
}

hipError_t launch_sweep(ugp_ctx ctx, int mode, int64_t n, const float *rays, const int32_t *excl,
                        const float *u, const int32_t *target, int32_t *prim_out, float *f_out,
                        int32_t *counts, double *td_out) {
    int32_t *buf = (int32_t *)ctx_scratch(ctx, sizeof(int32_t) * (size_t)(n + 1));
    if (!buf) return hipErrorOutOfMemory;
    hipError_t e = hipMemsetAsync(buf, 0, sizeof(int32_t), ctx->stream);
    if (e != hipSuccess) return e;
    SweepArgs A{mode, n, rays, excl, u, target, prim_out, f_out, buf + 1, buf, counts, td_out};
    const unsigned g = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_sweep_main, dim3(g), dim3(kBlock), 0, ctx->stream, ctx->scene, A, ctx->err);
    hipLaunchKernelGGL(k_sweep_wide, dim3(g), dim3(kBlock), 0, ctx->stream, ctx->scene, A, ctx->err);
    return hipGetLastError();
}

}  // namespace ugp
