// trace.hip -- per-ray scene queries exported through the C ABI:
// transmittance, primitive-level free-flight sampling, saturating distance and
// the emitter (light-sampling) query.  One lane per ray, one wave64 per block,
// the traversal stack in LDS.  Rays whose event buffer overflows in the main
// (register) sweep are queued and re-run by a wide sweep.
#include <mutex>

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
    if (!ray_ok(r, err)) {
        T[i] = __builtin_nanf("");
        if (F) F[i] = __builtin_nanf("");
        return;
    }
    TraceCount tc;
    const float f = transmittance_F(S, r, excl ? excl[i] : -1, F == nullptr, stack, err, tc);
    T[i] = fmaxf(0.f, 1.f - f);
    if (F) F[i] = f;
}

// ---------------------------------------------------------------------------
// Exponential variant (App. D; eq. exp_ff), per ray: T = exp(-depth) and
// decomposition tracking (exp_depth, exp_track).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_exp_transmittance(SceneDev S, int64_t n, const float *rays,
                                                              const int32_t *excl, float *T, uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const RayD r = load_ray(rays, i);
    if (!ray_ok(r, err)) {
        T[i] = __builtin_nanf("");
        return;
    }
    TraceCount tc;
    T[i] = expf(-exp_depth(S, r, excl ? excl[i] : -1, stack, err, tc));
}

// the uniform of Gaussian k on ray i: Philox4x32-10 with counter (ray index,
// k, 0) and key seed; top 24 bits of the first word
__device__ __forceinline__ double exp_uniform(uint64_t seed, int64_t i, int k) {
    const uint4 x = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)k, 0u),
                                  (uint32_t)seed, (uint32_t)(seed >> 32));
    return (double)(x.x >> 8) * (1.0 / 16777216.0);
}

__global__ __launch_bounds__(kBlock) void k_exp_sample(SceneDev S, int64_t n, const float *rays, const int32_t *excl,
                                                       uint64_t seed, int32_t *prim_out, float *t_out,
                                                       uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const RayD r = load_ray(rays, i);
    if (!ray_ok(r, err)) {
        prim_out[i] = -1;
        t_out[i] = __builtin_nanf("");
        return;
    }
    TraceCount tc;
    double t;
    const int bk = exp_track(S, r, excl ? excl[i] : -1,
                             [&](int k) __attribute__((always_inline)) { return exp_uniform(seed, i, k); }, stack,
                             err, tc, t);
    prim_out[i] = bk;
    t_out[i] = bk >= 0 ? (float)t : __builtin_nanf("");
}

// Test hook of the ray integral (Sec. 4.1 eq. ray_integral, App. A): the
// kernel's integral I_k over the ray's clipped chord of primitive k, computed
// by the same chord() the sweeps use (on k's first reference; the chord is
// the primitive's whatever slab holds it).  A missed primitive gives 0.
__global__ void k_ray_integral(SceneDev S, int64_t n, const float *rays, const int32_t *prim, float *I,
                               uint32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const RayD r = load_ray(rays, i);
    if (!ray_ok(r, err)) {
        I[i] = __builtin_nanf("");
        return;
    }
    const int k = prim[i];
    if (k < 0 || k >= S.n) {
        atomicOr(err, kErrRay);
        I[i] = __builtin_nanf("");
        return;
    }
    Chord c;
    I[i] = chord(load_hot(S.hot, S.inv[k]), r, S.r2, c) ? 2.f * c.W : 0.f;
}

// Test hook of the counter-based generator: Philox4x32-10 of counters
// [n][4] under one key, the function every random number of the renderer
// comes from.
__global__ void k_philox(int64_t n, const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 c = reinterpret_cast<const uint4 *>(ctr)[i];
    reinterpret_cast<uint4 *>(out)[i] = philox4x32_10(c, k0, k1);
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
    float4 *ovf_state;   // optional [ovf_slots][kOvfStateVecs]: the main pass's
                         // state of the first overflowed rays, resumed by the wide pass
    int64_t ovf_slots;   // overflowed rays with a saved state (the rest restart)
};

// An overflow happens at the end of a round that began with a full buffer of
// carried entries, none of which exits in the window: the round's new entries
// all have larger keys than the carried ones and were evicted, so the state
// at the overflow is the state at the start of that round.  The wide pass
// resumes from it instead of starting the ray again.
constexpr int64_t kOvfStateSlots = int64_t(1) << 20;
constexpr int kOvfStateVecs = 2 + kEventsMain;

__device__ __forceinline__ void save_state(float4 *p, const SweepState<kEventsMain> &st) {
    p[0] = make_float4(st.S_fin, st.lb_a, __int_as_float(st.lb_id), __int_as_float(st.round));
    p[1] = make_float4(__int_as_float(__double2loint(st.t_cur)), __int_as_float(__double2hiint(st.t_cur)),
                       __int_as_float(st.B.n), 0.f);
#pragma unroll
    for (int i = 0; i < kEventsMain; ++i)
        if (i < st.B.n) p[2 + i] = make_float4(st.B.a[i], st.B.b[i], st.B.w[i], __int_as_float(st.B.id[i]));
}

// the wide buffer re-derives the chords of the carried entries
__device__ __forceinline__ void load_state(const float4 *p, SweepState<kEventsWide> &st, const SceneDev &S,
                                           const RayD &r, TraceCount &tc) {
    const float4 h0 = p[0], h1 = p[1];
    st.S_fin = h0.x;
    st.lb_a = h0.y;
    st.lb_id = __float_as_int(h0.z);
    st.round = __float_as_int(h0.w);
    st.t_cur = __hiloint2double(__float_as_int(h1.y), __float_as_int(h1.x));
    const int n = __float_as_int(h1.z);
    float ws = 0.f;
    for (int i = 0; i < n; ++i) {
        const float4 e = p[2 + i];
        st.B.a[i] = e.x;
        st.B.b[i] = e.y;
        st.B.w[i] = e.z;
        st.B.id[i] = __float_as_int(e.w);
        st.B.ch.put(i, ev_chord(S, r, st.B.id[i], tc));
        ws += e.z;
    }
    st.B.n = n;
    st.wbuf = ws;
}

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

// results of ray i; an overflow of the main pass lists the ray for the wide
// one (returns its slot in the list, else -1)
__device__ __forceinline__ int write_out(const SweepArgs &A, int64_t i, const SweepOut &o, uint32_t *err,
                                         bool wide) {
    if (o.status != 0) {
        int slot = -1;
        if (!wide) {
            slot = atomicAdd(A.ovf_count, 1);
            A.ovf_list[slot] = (int32_t)i;
        } else {
            atomicOr(err, kErrEvents);
        }
        if (A.prim_out) A.prim_out[i] = -1;
        if (A.f_out) A.f_out[i] = __builtin_nanf("");
        if (A.td_out) A.td_out[i] = __builtin_nan("");
        return slot;
    }
    if (A.prim_out) A.prim_out[i] = o.prim;
    if (A.f_out) A.f_out[i] = o.t;
    if (A.td_out) A.td_out[i] = o.td;
    return -1;
}

// outputs of a ray that failed validation
__device__ __forceinline__ void write_invalid(const SweepArgs &A, int64_t i) {
    if (A.prim_out) A.prim_out[i] = -1;
    if (A.f_out) A.f_out[i] = __builtin_nanf("");
    if (A.td_out) A.td_out[i] = __builtin_nan("");
}

template <int K>
__device__ __forceinline__ void run_sweep(const SceneDev &S, const SweepArgs &A, int64_t i, int *stack,
                                          uint32_t *err, bool wide) {
    RayD r = load_ray(A.rays, i);
    if (!ray_ok(r, err)) {
        write_invalid(A, i);
        return;
    }
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
    write_out(A, i, o, err, wide);
}

__global__ __launch_bounds__(kBlock, 2) void k_sweep_main(SceneDev S, SweepArgs A, uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= A.n) return;
    run_sweep<kEventsMain>(S, A, i, stack, err, false);
}

// Persistent waves (lane_refill and suspended traversals): the sweep of each
// ray in rounds, lanes refilled from the caller's rays (LIST = false, the
// main pass with the K-entry buffer) or from the main pass's overflow list
// (LIST = true, the wide pass) as their rays finish.  (k_sweep_main and
// k_sweep_wide, one ray per lane, serve the per-ray traversal counters.)
template <int K, bool LIST>
__global__ __launch_bounds__(kBlock, 2) void k_sweep_persist(SceneDev S, SweepArgs A, int32_t *work,
                                                             uint32_t *err) {
    __shared__ int stack[kStackSize * kBlock];
    const int64_t n = LIST ? (int64_t)*A.ovf_count : A.n;
    int64_t i = -1;
    bool exhausted = false;
    RayD r = make_ray(0.f, 0.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.0);
    int ex = -1, target = -1;
    float u = 0.f, entry = -kInf;
    SweepState<K> st;
    SweepOut so;
    TraceCount tc;
    int spill[kStackSpill];
    for (;;) {
        const int64_t j = lane_refill(i < 0 && !exhausted, work);
        bool fresh = false;
        if (j >= 0) {
            if (j < n) {
                const int64_t ray = LIST ? (int64_t)A.ovf_list[j] : j;
                fresh = true;
                r = load_ray(A.rays, ray);
                ex = A.excl ? A.excl[ray] : -1;
                target = -1;
                entry = -kInf;
                // the wide pass takes only rays the main pass validated
                bool ok = LIST || ray_ok(r, err);
                if (!ok) write_invalid(A, ray);
                if (ok && A.mode == kModeEmitter) {
                    target = A.target[ray];
                    ok = emitter_ray(S, r, target, ex, entry);
                    if (!ok) A.f_out[ray] = 0.f;
                }
                if (ok) {
                    u = A.u ? A.u[ray] : 0.f;
                    i = ray;
                    sweep_start(st, so, r, A.mode);
                    if constexpr (LIST)
                        if (A.ovf_state && j < A.ovf_slots)
                            load_state(A.ovf_state + j * kOvfStateVecs, st, S, r, tc);
                }
            } else {
                exhausted = true;
            }
        }
        if (!__any(i >= 0 || fresh)) break;
        const int susp = __any(exhausted) ? 0 : kSuspendAt;
        if (i >= 0 && sweep_round<K>(S, r, ex, A.mode, u, target, entry, st, so, stack, spill, susp, err, tc)) {
            const int slot = write_out(A, i, so, err, LIST);
            if constexpr (!LIST)
                if (slot >= 0 && slot < A.ovf_slots && A.ovf_state)
                    save_state(A.ovf_state + (int64_t)slot * kOvfStateVecs, st);
            i = -1;
        }
    }
}

// clears the sweep's three counters (a kernel rather than a memset node, so
// that a caller may capture the launches in a graph)
__global__ void k_zero_counters(int32_t *c) {
    if (threadIdx.x < 3) c[threadIdx.x] = 0;
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

hipError_t launch_ray_integral(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *prim, float *I) {
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_ray_integral, dim3(g), dim3(256), 0, ctx->stream, ctx->scene, n, rays, prim, I, ctx->err);
    return hipGetLastError();
}

hipError_t launch_philox(ugp_ctx ctx, int64_t n, const uint32_t *ctr, uint64_t key, uint32_t *out) {
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_philox, dim3(g), dim3(256), 0, ctx->stream, n, ctr, (uint32_t)key, (uint32_t)(key >> 32),
                       out);
    return hipGetLastError();
}

hipError_t launch_exp(ugp_ctx ctx, int64_t n, const float *rays, const int32_t *excl, bool sample, uint64_t seed,
                      float *T, int32_t *prim_out, float *t_out) {
    const unsigned g = (unsigned)((n + kBlock - 1) / kBlock);
    if (sample)
        hipLaunchKernelGGL(k_exp_sample, dim3(g), dim3(kBlock), 0, ctx->stream, ctx->scene, n, rays, excl, seed,
                           prim_out, t_out, ctx->err);
    else
        hipLaunchKernelGGL(k_exp_transmittance, dim3(g), dim3(kBlock), 0, ctx->stream, ctx->scene, n, rays, excl,
                           T, ctx->err);
    return hipGetLastError();
}

// The sweep's working memory: [0] overflow count, [1] main-pass work counter,
// [2] wide-pass work counter, [3..3+n) overflow list; then (16-B aligned) the
// resumable states of the first `slots` overflowed rays (none with counts:
// the wide pass then starts each ray again and adds its own counts).
static size_t sweep_list_bytes(int64_t n) { return (sizeof(int32_t) * (size_t)(n + 3) + 15) & ~(size_t)15; }

static hipError_t launch_sweep_in(ugp_ctx ctx, int mode, int64_t n, const float *rays, const int32_t *excl,
                                  const float *u, const int32_t *target, int32_t *prim_out, float *f_out,
                                  int32_t *counts, double *td_out, char *mem, int64_t slots) {
    const size_t list_bytes = sweep_list_bytes(n);
    int32_t *buf = (int32_t *)mem;
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, ctx->stream, buf);
    float4 *state = (counts || slots == 0) ? nullptr : (float4 *)(mem + list_bytes);
    SweepArgs A{mode, n, rays, excl, u, target, prim_out, f_out, buf + 3, buf, counts, td_out, state,
                state ? slots : 0};
    const unsigned g = (unsigned)((n + kBlock - 1) / kBlock);
    const unsigned gp = std::min<unsigned>(g, 4096u);
    if (counts) {
        hipLaunchKernelGGL(k_sweep_main, dim3(g), dim3(kBlock), 0, ctx->stream, ctx->scene, A, ctx->err);
        hipLaunchKernelGGL(k_sweep_wide, dim3(g), dim3(kBlock), 0, ctx->stream, ctx->scene, A, ctx->err);
    } else {
        hipLaunchKernelGGL((k_sweep_persist<kEventsMain, false>), dim3(gp), dim3(kBlock), 0, ctx->stream,
                           ctx->scene, A, buf + 1, ctx->err);
        hipLaunchKernelGGL((k_sweep_persist<kEventsWide, true>), dim3(gp), dim3(kBlock), 0, ctx->stream,
                           ctx->scene, A, buf + 2, ctx->err);
    }
    return hipGetLastError();
}

hipError_t launch_sweep(ugp_ctx ctx, int mode, int64_t n, const float *rays, const int32_t *excl,
                        const float *u, const int32_t *target, int32_t *prim_out, float *f_out,
                        int32_t *counts, double *td_out) {
    const int64_t slots = counts ? 0 : std::min(n, kOvfStateSlots);
    const size_t bytes = sweep_list_bytes(n) + sizeof(float4) * kOvfStateVecs * (size_t)slots;
    char *mem = (char *)ctx_scratch(ctx, bytes);
    if (!mem) return hipErrorOutOfMemory;
    return launch_sweep_in(ctx, mode, n, rays, excl, u, target, prim_out, f_out, counts, td_out, mem, slots);
}

// ---------------------------------------------------------------------------
// Working memory of the allocation-free collision query: one fixed buffer per
// GPU in a file-scope device array, held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): it uses the device address that
// hipGetSymbolAddress returns, taken once per device with that device current.
// Every call on one GPU shares the buffer, so calls that overlap on a GPU race.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocBytes = size_t(32) << 20;
static_assert(sizeof(int32_t) * (size_t)(kNoAllocMaxRays + 3) + 16 + (size_t(1) << 20) <= kNoAllocBytes,
              "the overflow list of the largest call leaves room for resumable states");
static_assert(kNoAllocMaxRays == UGP_NOALLOC_MAX_RAYS, "the header states the library's limit");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices] = {};
hipError_t g_noalloc_status[kMaxDevices] = {};
bool g_noalloc_done[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_done[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));  // the caller made `device` current
        g_noalloc_status[device] = e;
        g_noalloc_ptr[device] = e == hipSuccess ? ptr : nullptr;
        g_noalloc_done[device] = true;
    }
    return g_noalloc_status[device];
}

hipError_t launch_sweep_noalloc(ugp_ctx ctx, int mode, int64_t n, const float *rays, const int32_t *excl,
                                const float *u, const int32_t *target, int32_t *prim_out, float *f_out) {
    if (n > kNoAllocMaxRays) return hipErrorInvalidValue;
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices && g_noalloc_done[ctx->device])
            base = g_noalloc_ptr[ctx->device];
    }
    if (!base) return hipErrorNotInitialized;
    const size_t list_bytes = sweep_list_bytes(n);
    const int64_t slots = std::min<int64_t>(
        n, (int64_t)((kNoAllocBytes - list_bytes) / (sizeof(float4) * kOvfStateVecs)));
    return launch_sweep_in(ctx, mode, n, rays, excl, u, target, prim_out, f_out, nullptr, nullptr,
                           (char *)base, slots);
}

}  // namespace ugp
