// build.hip -- scene packing and linear BVH construction on the GPU.
//
// 1. pack: per primitive (FP64 from the FP32 inputs) the rotation R from the
//    quaternion, the facet normal R e_argmin(s), the bounding-sphere radius
//    r max(s) and the box of the cut-off ellipsoid |S^-1 R^T (x - mu)| = r
//    (eq. cutoff_threshold), half-extent r sqrt(sum_i (R_ji s_i)^2), rounded
//    outward to float.  Inputs are validated here.
// 2. References: a primitive whose largest scale exceeds 4x its middle one is
//    cut along its long axis into m <= 8 slabs of equal thickness in its unit
//    frame, each referenced by its own (much tighter) box; the others have one
//    reference with the whole box.  A ray reports such a primitive only
//    through the slab that holds its chord entry point, so every primitive is
//    seen once.
// 3. 30-bit Morton codes of the reference box centres in the scene bounds,
//    stable LSD radix sort of (code, reference), 4 passes of 8 bits.
// 4. Binary radix tree over the sorted codes (Karras, "Maximizing Parallelism
//    in the Construction of BVHs, Octrees, and k-d Trees", HPG 2012); equal
//    codes are split by position.
// 5. Bottom-up refit: every leaf climbs, the second child to arrive at a node
//    forms its box (agent-scope atomics and fences, so it is safe across XCDs).
// 6. Scatter the hot records into leaf order, one per reference: hot = (mu,
//    d, M = S^-1 R^T rounded to float, original index, slab), 64 B; the cold
//    records (facet normal, material, albedo, roughness, emission,
//    bounding-sphere radius, 48 B) stay in original order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ugp_internal.hpp"
#include "ugp_math.hpp"

namespace ugp {
namespace {
constexpr int kThreads = 256;
}  // namespace

namespace {

// ---------------------------------------------------------------------------
// exclusive scan of int32 (device-wide, recursive over block sums)
// ---------------------------------------------------------------------------
constexpr int kScanItems = 4;
constexpr int kScanTile = kThreads * kScanItems;

__device__ __forceinline__ int block_exclusive_scan(int v, int *sh, int &total) {
    // Hillis-Steele over kThreads values in LDS
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        const int x = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    total = sh[kThreads - 1];
    const int incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_tiles(const int *in, int *out, int64_t n, int *tile_sums) {
    __shared__ int sh[kThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int sum = 0;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        sum += v[i];
    }
    int total;
    int run = block_exclusive_scan(sum, sh, total);
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0 && tile_sums) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_add(int *out, int64_t n, const int *tile_off) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    const int add = tile_off[blockIdx.x];
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) out[base + i] += add;
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits
// ---------------------------------------------------------------------------
constexpr int kSortChunks = 16;
constexpr int kSortTile = kThreads * kSortChunks;

__global__ void k_sort_hist(const uint32_t *keys, int64_t n, int shift, int *hist, int nblocks) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int c = 0; c < kSortChunks; ++c) {
        const int64_t i = base + (int64_t)c * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_sort_scatter(const uint32_t *keys, const int32_t *vals, uint32_t *okeys,
                               int32_t *ovals, int64_t n, int shift, const int *offs, int nblocks) {
    __shared__ int base[256];
    __shared__ int cnt[kThreads / 64][256];
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    base[t] = offs[(int64_t)t * nblocks + blockIdx.x];
    const int64_t tile = (int64_t)blockIdx.x * kSortTile;
    for (int c = 0; c < kSortChunks; ++c) {
        for (int w = 0; w < kThreads / 64; ++w) cnt[w][t] = 0;
        __syncthreads();
        const int64_t i = tile + (int64_t)c * kThreads + t;
        const bool valid = i < n;
        const uint32_t key = valid ? keys[i] : 0u;
        const int32_t val = valid ? vals[i] : 0;
        const uint32_t dig = (key >> shift) & 255u;
        // lanes of this wave holding the same digit
        uint64_t same = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot((dig >> b) & 1u);
            same &= ((dig >> b) & 1u) ? bal : ~bal;
        }
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        const int rank = __popcll(same & below);
        if (valid && rank == 0) cnt[wave][dig] = __popcll(same);
        __syncthreads();
        if (valid) {
            int pos = base[dig] + rank;
            for (int w = 0; w < wave; ++w) pos += cnt[w][dig];
            okeys[pos] = key;
            ovals[pos] = val;
        }
        __syncthreads();
        int tot = 0;
        for (int w = 0; w < kThreads / 64; ++w) tot += cnt[w][t];
        base[t] += tot;
        __syncthreads();
    }
}

}  // namespace

hipError_t exclusive_scan(const int *in, int *out, int64_t n, hipStream_t st) {
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles <= 1) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kThreads), 0, st, in, out, n, (int *)nullptr);
        return hipGetLastError();
    }
    int *sums = nullptr;
    hipError_t e = hipMallocAsync((void **)&sums, sizeof(int) * 2 * tiles, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kThreads), 0, st, in, out, n, sums);
    e = exclusive_scan(sums, sums + tiles, tiles, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(kThreads), 0, st, out, n,
                           (const int *)(sums + tiles));
        e = hipGetLastError();
    }
    hipFreeAsync(sums, st);
    return e;
}

hipError_t radix_sort(uint32_t *keys, int32_t *vals, uint32_t *tk, int32_t *tv, int64_t n,
                      hipStream_t st) {
    const int nblocks = (int)((n + kSortTile - 1) / kSortTile);
    int *hist = nullptr;
    hipError_t e = hipMallocAsync((void **)&hist, sizeof(int) * 2 * 256 * (size_t)nblocks, st);
    if (e != hipSuccess) return e;
    int *offs = hist + 256 * (size_t)nblocks;
    uint32_t *ka = keys, *kb = tk;
    int32_t *va = vals, *vb = tv;
    for (int shift = 0; shift < 32 && e == hipSuccess; shift += 8) {
        hipLaunchKernelGGL(k_sort_hist, dim3(nblocks), dim3(kThreads), 0, st, ka, n, shift, hist, nblocks);
        e = exclusive_scan(hist, offs, 256 * (int64_t)nblocks, st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_sort_scatter, dim3(nblocks), dim3(kThreads), 0, st, ka, va, kb, vb, n, shift,
                           offs, nblocks);
        e = hipGetLastError();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    hipFreeAsync(hist, st);
    return e;  // 4 passes: result back in keys / vals
}


namespace {


__device__ __forceinline__ float round_down(double x) {
    float f = (float)x;
    return ((double)f > x) ? nextafterf(f, -__builtin_huge_valf()) : f;
}
__device__ __forceinline__ float round_up(double x) {
    float f = (float)x;
    return ((double)f < x) ? nextafterf(f, __builtin_huge_valf()) : f;
}

// order-preserving float <-> uint for atomic min / max
__device__ __forceinline__ uint32_t f2o(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ __forceinline__ float o2f(uint32_t u) {
    uint32_t v = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
    float f;
    __builtin_memcpy(&f, &v, 4);
    return f;
}

struct PackIn {
    int64_t n;
    const float *mean, *scale, *rot, *dens, *alb, *rough, *emis;
    const int32_t *mat;
    const float *sggx;  // [n][6] or null
    const float *met;   // [n] or null (0)
    double r;
};

// boxes [n][6] (lo.xyz, hi.xyz) in original order; cold written in original
// order into a temporary; bounds[6] ordered-uint min/max of box centres
// slabs of a primitive: 1, or up to 8 along the long axis when it is more
// than 4x longer than its middle scale
__device__ __forceinline__ int slab_count(const double s[3]) {
    const double smax = fmax(s[0], fmax(s[1], s[2])), smin = fmin(s[0], fmin(s[1], s[2]));
    const double smid = s[0] + s[1] + s[2] - smax - smin;
    const double ratio = smax / smid;
    return ratio > 4.0 ? (int)fmin(8.0, ceil(ratio / 2.5)) : 1;
}

__device__ __forceinline__ void quat_to_R(const PackIn &in, int64_t k, double R[3][3]) {
    const double qw = in.rot[4 * k], qx = in.rot[4 * k + 1], qy = in.rot[4 * k + 2], qz = in.rot[4 * k + 3];
    const double qn = qw * qw + qx * qx + qy * qy + qz * qz;
    const double t = 2.0 / qn;
    const double xx = qx * qx * t, yy = qy * qy * t, zz = qz * qz * t;
    const double xy = qx * qy * t, xz = qx * qz * t, yz = qy * qz * t;
    const double wx = qw * qx * t, wy = qw * qy * t, wz = qw * qz * t;
    R[0][0] = 1.0 - yy - zz; R[0][1] = xy - wz; R[0][2] = xz + wy;
    R[1][0] = xy + wz; R[1][1] = 1.0 - xx - zz; R[1][2] = yz - wx;
    R[2][0] = xz - wy; R[2][1] = yz + wx; R[2][2] = 1.0 - xx - yy;
}

__global__ void k_pack(PackIn in, float *boxes, float4 *cold_tmp, float *mtmp, uint32_t *bounds,
                       int32_t *pieces, float4 *sggx_out, uint32_t *err) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= in.n) return;
    const double qw = in.rot[4 * k], qx = in.rot[4 * k + 1], qy = in.rot[4 * k + 2], qz = in.rot[4 * k + 3];
    const double s[3] = {in.scale[3 * k], in.scale[3 * k + 1], in.scale[3 * k + 2]};
    const double mu[3] = {in.mean[3 * k], in.mean[3 * k + 1], in.mean[3 * k + 2]};
    const double qn = qw * qw + qx * qx + qy * qy + qz * qz;
    const float d = in.dens[k];
    const int m = in.mat[k];
    bool bad = !(qn > 0.0) || !isfinite(qn) || !(d >= 0.f) || !isfinite(d) || m < 0 || m > 3 ||
               (m >= 2 && !in.sggx);
    for (int i = 0; i < 3; ++i) bad = bad || !(s[i] > 0.0) || !isfinite(s[i]) || !isfinite(mu[i]);
    const float met = in.met ? in.met[k] : 0.f;
    bad = bad || !(met >= 0.f && met <= 1.f);
    if (in.sggx) {
        double g[6];
        for (int i = 0; i < 6; ++i) g[i] = in.sggx[6 * k + i];
        const float alb[3] = {in.alb[3 * k], in.alb[3 * k + 1], in.alb[3 * k + 2]};
        float4 rec[8];
        bad = !sggx_prepare_prim(g, in.rough[k], met, alb, rec) || bad;
        for (int i = 0; i < 8; ++i) sggx_out[8 * k + i] = rec[i];
    }
    if (m == 3) atomicOr(err, 32u);  // (not an error: the scene holds material 3)
    if (bad) {
        atomicOr(err, 8u);
        for (int i = 0; i < 6; ++i) boxes[6 * k + i] = 0.f;
        pieces[k] = 1;
        return;
    }
    double R[3][3];
    quat_to_R(in, k, R);
    pieces[k] = slab_count(s);
    int am = 0;
    if (s[1] < s[am]) am = 1;
    if (s[2] < s[am]) am = 2;
    const double smax = fmax(s[0], fmax(s[1], s[2]));
    float lo[3], hi[3];
    for (int j = 0; j < 3; ++j) {
        double h2 = 0.0;
        for (int i = 0; i < 3; ++i) h2 += (R[j][i] * s[i]) * (R[j][i] * s[i]);
        const double h = in.r * sqrt(h2) * (1.0 + 1e-6);
        lo[j] = round_down(mu[j] - h);
        hi[j] = round_up(mu[j] + h);
        boxes[6 * k + j] = lo[j];
        boxes[6 * k + 3 + j] = hi[j];
    }
    // M = S^-1 R^T (row i = column i of R over s_i), rounded to float
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) mtmp[9 * k + 3 * i + j] = (float)(R[j][i] / s[i]);
    cold_tmp[3 * k] = make_float4((float)R[0][am], (float)R[1][am], (float)R[2][am], __int_as_float(m));
    cold_tmp[3 * k + 1] = make_float4(in.alb[3 * k], in.alb[3 * k + 1], in.alb[3 * k + 2], in.rough[k]);
    cold_tmp[3 * k + 2] = make_float4(in.emis[3 * k], in.emis[3 * k + 1], in.emis[3 * k + 2],
                                      (float)(in.r * smax));
    for (int j = 0; j < 3; ++j) {
        const float c = 0.5f * (lo[j] + hi[j]);
        atomicMin(&bounds[j], f2o(c));
        atomicMax(&bounds[3 + j], f2o(c));
    }
}

// References of primitive k at roff[k] ..: the whole box, or the boxes of its
// slabs.  Slab i of m holds the unit-frame points y with |y| <= r and y_L in
// [-r + 2 r i / m, -r + 2 r (i + 1) / m] (L = the long axis).  Its box bounds
// mu + A_L y_L (the axis segment) plus the cross-section disc of radius
// sqrt(r^2 - min y_L^2) spanned by A_a, A_b (A = R S), widened by a small
// margin so that a chord entry computed with the float M falls inside the
// box of the slab that owns it; it is clipped to the whole box.
__device__ __forceinline__ void slab_box(const PackIn &in, int64_t k, const double R[3][3], int i, int m, int L,
                                         const float *boxes, float *out) {
    const double s[3] = {in.scale[3 * k], in.scale[3 * k + 1], in.scale[3 * k + 2]};
    const int a = (L + 1) % 3, b = (L + 2) % 3;
    const double r = in.r * (1.0 + 1e-5), dl = 1e-4 * in.r;
    const double v0 = fmax(-r, -in.r + 2.0 * in.r * i / m - dl);
    const double v1 = fmin(r, -in.r + 2.0 * in.r * (i + 1) / m + dl);
    const double rho = (v0 <= 0.0 && v1 >= 0.0) ? r : sqrt(fmax(0.0, r * r - fmin(v0 * v0, v1 * v1)));
    for (int d = 0; d < 3; ++d) {
        const double mu = in.mean[3 * k + d];
        const double AL = R[d][L] * s[L], Aa = R[d][a] * s[a], Ab = R[d][b] * s[b];
        const double c0 = AL * v0, c1 = AL * v1;
        const double cs = rho * sqrt(Aa * Aa + Ab * Ab);
        const double lo = fmax(mu + fmin(c0, c1) - cs, (double)boxes[6 * k + d]);
        const double hi = fmin(mu + fmax(c0, c1) + cs, (double)boxes[6 * k + 3 + d]);
        out[d] = round_down(lo);
        out[3 + d] = round_up(hi);
    }
}

__global__ void k_refs(PackIn in, const int32_t *pieces, const int32_t *roff, const float *boxes, float *rbox,
                       int32_t *rprim, int32_t *rinfo) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= in.n) return;
    const int m = pieces[k];
    const int64_t j0 = roff[k];
    if (m == 1) {
        for (int c = 0; c < 6; ++c) rbox[6 * j0 + c] = boxes[6 * k + c];
        rprim[j0] = (int32_t)k;
        rinfo[j0] = 1 << 8;
        return;
    }
    double R[3][3];
    quat_to_R(in, k, R);
    const double s[3] = {in.scale[3 * k], in.scale[3 * k + 1], in.scale[3 * k + 2]};
    int L = 0;
    if (s[1] > s[L]) L = 1;
    if (s[2] > s[L]) L = 2;
    for (int i = 0; i < m; ++i) {
        const int64_t j = j0 + i;
        slab_box(in, k, R, i, m, L, boxes, rbox + 6 * j);
        rprim[j] = (int32_t)k;
        rinfo[j] = i | (m << 8) | (L << 16);
    }
}

__global__ void k_emit_flags(int64_t n, const float4 *cold, int32_t *flag) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float4 e = cold[3 * k + 2];
    flag[k] = (e.x > 0.f || e.y > 0.f || e.z > 0.f) ? 1 : 0;
}

__global__ void k_init_bounds(uint32_t *b) {
    if (threadIdx.x < 3) b[threadIdx.x] = 0xffffffffu;
    else if (threadIdx.x < 6) b[threadIdx.x] = 0u;
}

__device__ __forceinline__ uint32_t expand10(uint32_t v) {
    v = (v * 0x00010001u) & 0xFF0000FFu;
    v = (v * 0x00000101u) & 0x0F00F00Fu;
    v = (v * 0x00000011u) & 0xC30C30C3u;
    v = (v * 0x00000005u) & 0x49249249u;
    return v;
}

__global__ void k_morton(int64_t n, const float *boxes, const uint32_t *bounds, uint32_t *keys,
                         int32_t *vals) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t code = 0;
    uint32_t q[3];
    for (int j = 0; j < 3; ++j) {
        const float lo = o2f(bounds[j]), hi = o2f(bounds[3 + j]);
        const float c = 0.5f * (boxes[6 * k + j] + boxes[6 * k + 3 + j]);
        const float ext = hi - lo;
        float f = ext > 0.f ? (c - lo) / ext : 0.5f;
        f = fminf(fmaxf(f, 0.f), 1.f);
        q[j] = min((uint32_t)(f * 1024.f), 1023u);
    }
    code = (expand10(q[0]) << 2) | (expand10(q[1]) << 1) | expand10(q[2]);
    keys[k] = code;
    vals[k] = (int32_t)k;
}

// ---------------------------------------------------------------------------
// Karras radix tree
// ---------------------------------------------------------------------------
__device__ __forceinline__ int delta(const uint32_t *keys, int64_t n, int64_t i, int64_t j) {
    if (j < 0 || j >= n) return -1;
    const uint32_t a = keys[i], b = keys[j];
    if (a == b) return 32 + __clz((uint32_t)(i ^ j));
    return __clz(a ^ b);
}

__global__ void k_karras(const uint32_t *keys, int64_t n, float4 *nodes, int32_t *parent_node,
                         int32_t *parent_leaf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = delta(keys, n, i, i - d);
    int64_t lmax = 2;
    while (delta(keys, n, i, i + lmax * d) > dmin) lmax *= 2;
    int64_t l = 0;
    for (int64_t t = lmax / 2; t >= 1; t /= 2)
        if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int64_t j = i + l * d;
    const int dnode = delta(keys, n, i, j);
    int64_t s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
    const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    int32_t left, right;
    if (lo == gamma) {
        left = ~(int32_t)gamma;
        parent_leaf[gamma] = (int32_t)i;
    } else {
        left = (int32_t)gamma;
        parent_node[gamma] = (int32_t)i;
    }
    if (hi == gamma + 1) {
        right = ~(int32_t)(gamma + 1);
        parent_leaf[gamma + 1] = (int32_t)i;
    } else {
        right = (int32_t)(gamma + 1);
        parent_node[gamma + 1] = (int32_t)i;
    }
    nodes[4 * i + 3] = make_float4(__int_as_float(left), __int_as_float(right), 0.f, 0.f);
}

// Structural check of the radix tree before anything climbs it: every child
// ref is in range, the root is nobody's child, and every other node and every
// leaf has exactly one parent.  Failures set bit 16 of the error word and the
// kernels that follow return at once.
__global__ void k_validate_refs(int64_t n, const float4 *nodes, int32_t *pc_node, int32_t *pc_leaf,
                                uint32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const float4 n3 = nodes[4 * i + 3];
    const int32_t c[2] = {__float_as_int(n3.x), __float_as_int(n3.y)};
    for (int k = 0; k < 2; ++k) {
        if (c[k] >= 0) {
            if (c[k] == 0 || c[k] >= n - 1) atomicOr(err, 16u);
            else atomicAdd(&pc_node[c[k]], 1);
        } else {
            const int64_t leaf = ~c[k];
            if (leaf >= n) atomicOr(err, 16u);
            else atomicAdd(&pc_leaf[leaf], 1);
        }
    }
}

__global__ void k_validate_counts(int64_t n, const int32_t *pc_node, const int32_t *pc_leaf, uint32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && pc_leaf[i] != 1) atomicOr(err, 16u);
    if (i < n - 1 && pc_node[i] != (i == 0 ? 0 : 1)) atomicOr(err, 16u);
}

// Boxes of the binary radix tree, level by level from the deepest: launch L
// fills the two child boxes of every node at depth L from its leaves' boxes
// or from its internal children's boxes (filled by the launch before), so
// kernel boundaries order the levels and no node waits on another thread.
// (A climb from each leaf with a flag per node needs device-wide fences at
// every step, and each fence writes back and invalidates the per-XCD L2.)
__global__ void k_node_depth(int64_t ni, const int32_t *parent_node, int32_t *ndepth, int32_t *maxd,
                             uint32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni || (*err & 16u)) return;
    int d = 0;
    for (int32_t p = (int32_t)i; p != 0; p = parent_node[p]) {
        if (++d > 4096) {  // a cycle: not a tree
            atomicOr(err, 16u);
            return;
        }
    }
    ndepth[i] = d;
    atomicMax(maxd, d);
}

__global__ void k_refit_level(int64_t ni, int32_t level, const int32_t *ndepth, const int32_t *sorted_orig,
                              const float *boxes, float4 *nodes) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni || ndepth[i] != level) return;
    float *nd = reinterpret_cast<float *>(nodes + 4 * i);
    const int32_t ref[2] = {__float_as_int(nd[12]), __float_as_int(nd[13])};
    for (int side = 0; side < 2; ++side) {
        float b[6];
        if (ref[side] < 0) {
            const float *lb = boxes + 6 * (int64_t)sorted_orig[~ref[side]];
            for (int c = 0; c < 6; ++c) b[c] = lb[c];
        } else {
            const float *cn = reinterpret_cast<const float *>(nodes + 4 * (int64_t)ref[side]);
            for (int c = 0; c < 3; ++c) {
                b[c] = fminf(cn[c], cn[6 + c]);
                b[3 + c] = fmaxf(cn[3 + c], cn[9 + c]);
            }
        }
        for (int c = 0; c < 6; ++c) nd[6 * side + c] = b[c];
    }
}

__global__ void k_depth(int64_t n, const int32_t *parent_node, const int32_t *parent_leaf, int32_t *depth,
                        uint32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (*err & 16u)) return;
    int d = 1;
    int32_t p = parent_leaf[i];
    while (true) {
        ++d;
        if (p == 0) break;
        if (d > 4096) {  // a cycle: not a tree
            atomicOr(err, 16u);
            break;
        }
        p = parent_node[p];
    }
    atomicMax(depth, d);
}

// The binary radix tree is collapsed into a 4-wide hierarchy (below).  A
// 4-wide node is 128 B: lo.x[4], lo.y[4], lo.z[4], hi.x[4], hi.y[4], hi.z[4],
// ref[4], pad; a ref >= 0 is a 4-wide node, < 0 the leaf primitive ~ref,
// kEmptySlot unused.
__device__ __forceinline__ void node_child(const float4 *nodes, int32_t b, int side, float box[6], int32_t &ref) {
    const float *nd = reinterpret_cast<const float *>(nodes + 4 * (int64_t)b);
    const int o = side ? 6 : 0;
    for (int c = 0; c < 6; ++c) box[c] = nd[o + c];
    ref = side ? __float_as_int(nd[13]) : __float_as_int(nd[12]);
}

// Greedy collapse, one level of the 4-wide hierarchy per launch: a 4-wide
// node rooted at binary node b starts with b's two children and repeatedly
// opens its internal child of largest surface area (the child a ray is most
// likely to enter) until it holds four children or only leaves.  Its internal
// children become the roots of the next level's nodes: each gets an output
// slot (atomic counter) and a place in the next frontier.
__global__ void k_collapse_greedy(const float4 *nodes, const int32_t *fin, const int32_t *fout, int32_t nf,
                                  int32_t *gin, int32_t *gout, int32_t *ng, int32_t *n4, float4 *nodes4) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    float lo[3][4], hi[3][4];
    int32_t ref[4];
    int ns = 0;
    for (int side = 0; side < 2; ++side) {
        float box[6];
        node_child(nodes, fin[i], side, box, ref[ns]);
        for (int k = 0; k < 3; ++k) { lo[k][ns] = box[k]; hi[k][ns] = box[3 + k]; }
        ++ns;
    }
    while (ns < 4) {
        int best = -1;
        float best_area = -1.f;
        for (int k = 0; k < ns; ++k) {
            if (ref[k] < 0) continue;
            const float ex = hi[0][k] - lo[0][k], ey = hi[1][k] - lo[1][k], ez = hi[2][k] - lo[2][k];
            const float area = ex * ey + ey * ez + ez * ex;
            if (area > best_area) {
                best_area = area;
                best = k;
            }
        }
        if (best < 0) break;
        const int32_t c = ref[best];
        float box[6];
        node_child(nodes, c, 0, box, ref[best]);
        for (int k = 0; k < 3; ++k) { lo[k][best] = box[k]; hi[k][best] = box[3 + k]; }
        node_child(nodes, c, 1, box, ref[ns]);
        for (int k = 0; k < 3; ++k) { lo[k][ns] = box[k]; hi[k][ns] = box[3 + k]; }
        ++ns;
    }
    for (int k = 0; k < ns; ++k) {
        if (ref[k] < 0) continue;
        const int32_t slot = atomicAdd(n4, 1);
        const int32_t q = atomicAdd(ng, 1);
        gin[q] = ref[k];
        gout[q] = slot;
        ref[k] = slot;
    }
    for (; ns < 4; ++ns) {
        for (int k = 0; k < 3; ++k) { lo[k][ns] = 3.0e38f; hi[k][ns] = -3.0e38f; }
        ref[ns] = kEmptySlot;
    }
    float4 *o = nodes4 + 8 * (int64_t)fout[i];
    o[0] = make_float4(lo[0][0], lo[0][1], lo[0][2], lo[0][3]);
    o[1] = make_float4(lo[1][0], lo[1][1], lo[1][2], lo[1][3]);
    o[2] = make_float4(lo[2][0], lo[2][1], lo[2][2], lo[2][3]);
    o[3] = make_float4(hi[0][0], hi[0][1], hi[0][2], hi[0][3]);
    o[4] = make_float4(hi[1][0], hi[1][1], hi[1][2], hi[1][3]);
    o[5] = make_float4(hi[2][0], hi[2][1], hi[2][2], hi[2][3]);
    o[6] = make_float4(__int_as_float(ref[0]), __int_as_float(ref[1]), __int_as_float(ref[2]),
                       __int_as_float(ref[3]));
    o[7] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// hot record of leaf i (reference sorted_ref[i]); inv[o] = the leaf of the
// first slab of primitive o
// the hot record of a leaf: primitive o, slab info (slab | count << 8 | long axis << 16)
__device__ __forceinline__ void write_hot(const PackIn &in, const float *mtmp, int64_t o, int info, float4 *h) {
    const float *M = mtmp + 9 * o;
    h[0] = make_float4(in.mean[3 * o], in.mean[3 * o + 1], in.mean[3 * o + 2], in.dens[o]);
    h[1] = make_float4(M[0], M[1], M[2], M[3]);
    h[2] = make_float4(M[4], M[5], M[6], M[7]);
    // largest row norm of M, 1 / min(s): bounds how M magnifies an offset
    const float smin = fminf(in.scale[3 * o], fminf(in.scale[3 * o + 1], in.scale[3 * o + 2]));
    h[3] = make_float4(M[8], __int_as_float((int)o), 1.0f / smin, __int_as_float(info));
}

__global__ void k_scatter(int64_t nr, const int32_t *sorted_ref, const int32_t *rprim, const int32_t *rinfo,
                          PackIn in, const float *mtmp, float4 *hot, int32_t *inv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    const int32_t j = sorted_ref[i];
    const int64_t o = rprim[j];
    const int info = rinfo[j];
    write_hot(in, mtmp, o, info, hot + 4 * i);
    if ((info & 255) == 0) inv[o] = (int32_t)i;
}

// Refit, leaves: each leaf keeps its primitive and slab (the layout of the
// build: slab count and long axis as recorded) and takes the new parameters'
// record and box.  Slabs of a fixed count along a fixed axis still cover the
// ellipsoid, whatever its new shape; only their tightness changes.
__global__ void k_refit_leaves(int64_t nr, PackIn in, const float *mtmp, const float *boxes, float4 *hot,
                               float *lbox) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    const float4 h3 = hot[4 * i + 3];
    const int64_t o = __float_as_int(h3.y);
    const int info = __float_as_int(h3.w);
    write_hot(in, mtmp, o, info, hot + 4 * i);
    const int m = (info >> 8) & 255;
    if (m <= 1) {
        for (int c = 0; c < 6; ++c) lbox[6 * i + c] = boxes[6 * o + c];
    } else {
        double R[3][3];
        quat_to_R(in, o, R);
        slab_box(in, o, R, info & 255, m, (info >> 16) & 3, boxes, lbox + 6 * i);
    }
}

// Refit, one level of 4-wide nodes [q0, q1): every child box from its leaf's
// box or from the union of its node's four (already refitted) child boxes.
__global__ void k_refit_nodes(int32_t q0, int32_t q1, float4 *nodes4, const float *lbox) {
    const int64_t q = q0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= q1) return;
    float4 *nd = nodes4 + 8 * q;
    const float4 rf = nd[6];
    const int32_t ref[4] = {__float_as_int(rf.x), __float_as_int(rf.y), __float_as_int(rf.z), __float_as_int(rf.w)};
    float lo[3][4], hi[3][4];
    for (int c = 0; c < 4; ++c) {
        float b[6] = {3.0e38f, 3.0e38f, 3.0e38f, -3.0e38f, -3.0e38f, -3.0e38f};
        if (ref[c] != kEmptySlot && ref[c] < 0) {
            for (int k = 0; k < 6; ++k) b[k] = lbox[6 * (int64_t)~ref[c] + k];
        } else if (ref[c] != kEmptySlot) {
            const float4 *ch = nodes4 + 8 * (int64_t)ref[c];
            for (int k = 0; k < 3; ++k) {
                const float4 l = ch[k], h = ch[3 + k];
                b[k] = fminf(fminf(l.x, l.y), fminf(l.z, l.w));
                b[3 + k] = fmaxf(fmaxf(h.x, h.y), fmaxf(h.z, h.w));
            }
        }
        for (int k = 0; k < 3; ++k) { lo[k][c] = b[k]; hi[k][c] = b[3 + k]; }
    }
    for (int k = 0; k < 3; ++k) {
        nd[k] = make_float4(lo[k][0], lo[k][1], lo[k][2], lo[k][3]);
        nd[3 + k] = make_float4(hi[k][0], hi[k][1], hi[k][2], hi[k][3]);
    }
}

__global__ void k_compact(int64_t n, const int32_t *flag, const int32_t *pos, int32_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) out[pos[i]] = (int32_t)i;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

void free_scene(SceneDev &sc) {
    hipFree(sc.hot);
    hipFree(sc.cold);
    hipFree(sc.sggx);
    hipFree(sc.nodes);
    hipFree(sc.inv);
    hipFree(sc.emit);
    sc = SceneDev{};
}

#define UGP_CHECK(x)                      \
    do {                                  \
        hipError_t e_ = (x);              \
        if (e_ != hipSuccess) goto fail;  \
    } while (0)

hipError_t build_scene(ugp_ctx ctx, const ugp_scene *s, float eps) {
    hipStream_t st = ctx->stream;
    const int64_t n = s->n;
    SceneDev sc;
    sc.n = n;
    const double r = sqrt(-2.0 * log((double)eps));
    sc.r2 = (float)(r * r);
    sc.r_cut = r;
    std::vector<int32_t> levels4{0, 1};  // level L of the 4-wide nodes: [levels4[L], levels4[L + 1])
    PackIn in{n, s->mean, s->scale, s->rotation, s->density, s->albedo, s->roughness, s->emission,
              s->material, s->sggx, s->metallic, r};
    float *boxes = nullptr, *rbox = nullptr;
    float *mtmp = nullptr;
    uint32_t *bounds = nullptr, *keys = nullptr, *tk = nullptr;
    int32_t *vals = nullptr, *tv = nullptr, *pnode = nullptr, *pleaf = nullptr, *flags = nullptr;
    int32_t *pc_node = nullptr, *pc_leaf = nullptr, *pieces = nullptr, *roff = nullptr, *rprim = nullptr,
            *rinfo = nullptr;
    int32_t *emit_flag = nullptr, *emit_pos = nullptr, *depth = nullptr;
    uint32_t *berr = nullptr;  // the build's own validation flags (not the context's query errors)
    int32_t *maxd = nullptr;   // deepest internal node of the radix tree
    int32_t h_maxd = 0;
    hipError_t e = hipSuccess;
    uint32_t h_err = 0;
    int32_t h_depth = 0, h_nemit = 0, h_last_flag = 0, h_roff_last = 0, h_pieces_last = 0;
    int64_t nr = 0, ni = 1;

    // pack, slab counts, reference offsets
    UGP_CHECK(hipMalloc((void **)&sc.cold, sizeof(float4) * 3 * n));
    UGP_CHECK(hipMalloc((void **)&sc.inv, sizeof(int32_t) * n));
    UGP_CHECK(hipMallocAsync((void **)&boxes, sizeof(float) * 6 * n, st));
    UGP_CHECK(hipMallocAsync((void **)&mtmp, sizeof(float) * 9 * n, st));
    UGP_CHECK(hipMallocAsync((void **)&bounds, sizeof(uint32_t) * 8, st));
    UGP_CHECK(hipMallocAsync((void **)&pieces, sizeof(int32_t) * n, st));
    UGP_CHECK(hipMallocAsync((void **)&roff, sizeof(int32_t) * n, st));
    UGP_CHECK(hipMallocAsync((void **)&emit_flag, sizeof(int32_t) * n, st));
    UGP_CHECK(hipMallocAsync((void **)&emit_pos, sizeof(int32_t) * n, st));
    UGP_CHECK(hipMallocAsync((void **)&depth, sizeof(int32_t), st));
    UGP_CHECK(hipMallocAsync((void **)&berr, sizeof(uint32_t), st));
    UGP_CHECK(hipMallocAsync((void **)&maxd, sizeof(int32_t), st));
    UGP_CHECK(hipMemsetAsync(berr, 0, sizeof(uint32_t), st));
    UGP_CHECK(hipMemsetAsync(depth, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_init_bounds, dim3(1), dim3(64), 0, st, bounds);
    if (s->sggx) UGP_CHECK(hipMalloc((void **)&sc.sggx, sizeof(float4) * 8 * n));
    hipLaunchKernelGGL(k_pack, dim3(blocks(n)), dim3(kThreads), 0, st, in, boxes, sc.cold, mtmp, bounds, pieces,
                       sc.sggx, berr);
    UGP_CHECK(hipGetLastError());
    UGP_CHECK(exclusive_scan(pieces, roff, n, st));
    UGP_CHECK(hipMemcpyAsync(&h_roff_last, roff + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st));
    UGP_CHECK(hipMemcpyAsync(&h_pieces_last, pieces + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st));
    UGP_CHECK(hipMemcpyAsync(&h_err, berr, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    UGP_CHECK(hipStreamSynchronize(st));
    if (h_err & 8u) {
        e = hipErrorInvalidValue;
        goto fail;
    }
    sc.has_mat3 = (h_err & 32u) != 0;
    nr = (int64_t)h_roff_last + h_pieces_last;
    if (nr >= (int64_t(1) << 31) - 1) {
        e = hipErrorNotSupported;
        goto fail;
    }
    ni = nr > 1 ? nr - 1 : 1;
    sc.n_refs = nr;
    UGP_CHECK(hipMalloc((void **)&sc.hot, sizeof(float4) * 4 * nr));
    UGP_CHECK(hipMalloc((void **)&sc.nodes, sizeof(float4) * 4 * ni));
    UGP_CHECK(hipMallocAsync((void **)&rbox, sizeof(float) * 6 * nr, st));
    UGP_CHECK(hipMallocAsync((void **)&rprim, sizeof(int32_t) * nr, st));
    UGP_CHECK(hipMallocAsync((void **)&rinfo, sizeof(int32_t) * nr, st));
    UGP_CHECK(hipMallocAsync((void **)&keys, sizeof(uint32_t) * nr, st));
    UGP_CHECK(hipMallocAsync((void **)&tk, sizeof(uint32_t) * nr, st));
    UGP_CHECK(hipMallocAsync((void **)&vals, sizeof(int32_t) * nr, st));
    UGP_CHECK(hipMallocAsync((void **)&tv, sizeof(int32_t) * nr, st));
    UGP_CHECK(hipMallocAsync((void **)&pnode, sizeof(int32_t) * ni, st));
    UGP_CHECK(hipMallocAsync((void **)&pleaf, sizeof(int32_t) * nr, st));
    UGP_CHECK(hipMallocAsync((void **)&flags, sizeof(int32_t) * ni, st));
    UGP_CHECK(hipMallocAsync((void **)&pc_node, sizeof(int32_t) * ni, st));
    UGP_CHECK(hipMallocAsync((void **)&pc_leaf, sizeof(int32_t) * nr, st));
    UGP_CHECK(hipMemsetAsync(flags, 0, sizeof(int32_t) * ni, st));
    hipLaunchKernelGGL(k_refs, dim3(blocks(n)), dim3(kThreads), 0, st, in, (const int32_t *)pieces,
                       (const int32_t *)roff, (const float *)boxes, rbox, rprim, rinfo);
    hipLaunchKernelGGL(k_morton, dim3(blocks(nr)), dim3(kThreads), 0, st, nr, rbox, bounds, keys, vals);
    UGP_CHECK(hipGetLastError());
    UGP_CHECK(radix_sort(keys, vals, tk, tv, nr, st));
    if (nr > 1) {
        hipLaunchKernelGGL(k_karras, dim3(blocks(nr - 1)), dim3(kThreads), 0, st, keys, nr, sc.nodes, pnode, pleaf);
        UGP_CHECK(hipMemsetAsync(pc_leaf, 0, sizeof(int32_t) * nr, st));
        UGP_CHECK(hipMemsetAsync(pc_node, 0, sizeof(int32_t) * ni, st));
        hipLaunchKernelGGL(k_validate_refs, dim3(blocks(nr - 1)), dim3(kThreads), 0, st, nr, sc.nodes, pc_node,
                           pc_leaf, berr);
        hipLaunchKernelGGL(k_validate_counts, dim3(blocks(nr)), dim3(kThreads), 0, st, nr, pc_node, pc_leaf,
                           berr);
        // node depths (into `flags`), then the boxes level by level
        UGP_CHECK(hipMemsetAsync(maxd, 0, sizeof(int32_t), st));
        hipLaunchKernelGGL(k_node_depth, dim3(blocks(nr - 1)), dim3(kThreads), 0, st, nr - 1, (const int32_t *)pnode,
                           flags, maxd, berr);
        UGP_CHECK(hipMemcpyAsync(&h_maxd, maxd, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        UGP_CHECK(hipMemcpyAsync(&h_err, berr, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        UGP_CHECK(hipStreamSynchronize(st));
        if (h_err & 16u) {
            e = hipErrorUnknown;
            goto fail;
        }
        for (int32_t L = h_maxd; L >= 0; --L)
            hipLaunchKernelGGL(k_refit_level, dim3(blocks(nr - 1)), dim3(kThreads), 0, st, nr - 1, L,
                               (const int32_t *)flags, (const int32_t *)vals, (const float *)rbox, sc.nodes);
        UGP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_depth, dim3(blocks(nr)), dim3(kThreads), 0, st, nr, pnode, pleaf, depth, berr);
    }
    hipLaunchKernelGGL(k_scatter, dim3(blocks(nr)), dim3(kThreads), 0, st, nr, vals, (const int32_t *)rprim,
                       (const int32_t *)rinfo, in, mtmp, sc.hot, sc.inv);
    hipLaunchKernelGGL(k_emit_flags, dim3(blocks(n)), dim3(kThreads), 0, st, n, (const float4 *)sc.cold, emit_flag);
    UGP_CHECK(hipGetLastError());
    UGP_CHECK(exclusive_scan(emit_flag, emit_pos, n, st));
    UGP_CHECK(hipMemcpyAsync(&h_nemit, emit_pos + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st));
    UGP_CHECK(hipMemcpyAsync(&h_last_flag, emit_flag + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st));
    UGP_CHECK(hipMemcpyAsync(&h_depth, depth, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    UGP_CHECK(hipMemcpyAsync(&h_err, berr, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    {
        float rootb[12];
        if (nr > 1) UGP_CHECK(hipMemcpyAsync(rootb, sc.nodes, sizeof(float) * 12, hipMemcpyDeviceToHost, st));
        else UGP_CHECK(hipMemcpyAsync(rootb, rbox, sizeof(float) * 6, hipMemcpyDeviceToHost, st));
        UGP_CHECK(hipStreamSynchronize(st));
        if (nr > 1) {
            for (int c = 0; c < 3; ++c) {
                sc.lo[c] = std::min(rootb[c], rootb[6 + c]);
                sc.hi[c] = std::max(rootb[3 + c], rootb[9 + c]);
            }
        } else {
            for (int c = 0; c < 3; ++c) { sc.lo[c] = rootb[c]; sc.hi[c] = rootb[3 + c]; }
        }
    }
    if (h_err & 8u) {
        e = hipErrorInvalidValue;
        goto fail;
    }
    if (h_err & 16u) {
        e = hipErrorUnknown;
        goto fail;
    }
    h_nemit += h_last_flag;
    sc.n_emit = h_nemit;
    sc.depth = nr > 1 ? h_depth : 1;
    sc.root = nr > 1 ? 0 : ~0;
    if (nr > 1) {
        // greedy 4-wide collapse, level by level (keys / tk / vals / tv reused as frontiers)
        int32_t *fin = (int32_t *)keys, *fout = (int32_t *)tk, *gin = (int32_t *)vals, *gout = (int32_t *)tv;
        int32_t *cnt = nullptr;  // [0] next frontier, [1] 4-wide nodes
        float4 *big = nullptr;
        UGP_CHECK(hipMalloc((void **)&cnt, sizeof(int32_t) * 2));
        e = hipMalloc((void **)&big, sizeof(float4) * 8 * (size_t)(nr - 1));
        if (e != hipSuccess) {
            hipFree(cnt);
            goto fail;
        }
        const int32_t init[2] = {0, 1};
        UGP_CHECK(hipMemcpyAsync(cnt, init, sizeof(init), hipMemcpyHostToDevice, st));
        UGP_CHECK(hipMemsetAsync(fin, 0, sizeof(int32_t), st));
        UGP_CHECK(hipMemsetAsync(fout, 0, sizeof(int32_t), st));
        int32_t nf = 1, levels = 0;
        while (nf > 0) {
            UGP_CHECK(hipMemsetAsync(cnt, 0, sizeof(int32_t), st));
            hipLaunchKernelGGL(k_collapse_greedy, dim3(blocks(nf)), dim3(kThreads), 0, st,
                               (const float4 *)sc.nodes, (const int32_t *)fin, (const int32_t *)fout, nf, gin,
                               gout, cnt, cnt + 1, big);
            UGP_CHECK(hipGetLastError());
            int32_t h_cnt[2] = {0, 0};
            UGP_CHECK(hipMemcpyAsync(h_cnt, cnt, sizeof(h_cnt), hipMemcpyDeviceToHost, st));
            UGP_CHECK(hipStreamSynchronize(st));
            nf = h_cnt[0];
            levels4.push_back(h_cnt[1]);
            std::swap(fin, gin);
            std::swap(fout, gout);
            if (++levels > 4096) {
                hipFree(big);
                hipFree(cnt);
                e = hipErrorUnknown;
                goto fail;
            }
        }
        int32_t h_n4 = 0;
        e = hipMemcpy(&h_n4, cnt + 1, sizeof(int32_t), hipMemcpyDeviceToHost);
        hipFree(cnt);
        float4 *nodes4 = nullptr;
        if (e == hipSuccess) e = hipMalloc((void **)&nodes4, sizeof(float4) * 8 * (size_t)h_n4);
        if (e != hipSuccess) {
            hipFree(big);
            goto fail;
        }
        UGP_CHECK(hipMemcpyAsync(nodes4, big, sizeof(float4) * 8 * (size_t)h_n4, hipMemcpyDeviceToDevice, st));
        UGP_CHECK(hipStreamSynchronize(st));
        hipFree(big);
        hipFree(sc.nodes);
        sc.nodes = nodes4;
        sc.n_nodes4 = h_n4;
        sc.depth = levels;
        // a 4-wide node pushes at most three entries
        if (3 * sc.depth > kStackSize + kStackSpill) {
            e = hipErrorNotSupported;
            goto fail;
        }
    }
    if (h_nemit > 0) {
        UGP_CHECK(hipMalloc((void **)&sc.emit, sizeof(int32_t) * h_nemit));
        hipLaunchKernelGGL(k_compact, dim3(blocks(n)), dim3(kThreads), 0, st, n, emit_flag, emit_pos, sc.emit);
        UGP_CHECK(hipGetLastError());
    }
    hipFreeAsync(boxes, st); hipFreeAsync(rbox, st); hipFreeAsync(mtmp, st); hipFreeAsync(bounds, st);
    hipFreeAsync(keys, st); hipFreeAsync(tk, st); hipFreeAsync(vals, st); hipFreeAsync(tv, st);
    hipFreeAsync(pnode, st); hipFreeAsync(pleaf, st); hipFreeAsync(flags, st);
    hipFreeAsync(pc_node, st); hipFreeAsync(pc_leaf, st); hipFreeAsync(pieces, st); hipFreeAsync(roff, st);
    hipFreeAsync(rprim, st); hipFreeAsync(rinfo, st);
    hipFreeAsync(emit_flag, st); hipFreeAsync(emit_pos, st); hipFreeAsync(depth, st); hipFreeAsync(berr, st);
    hipFreeAsync(maxd, st);
    UGP_CHECK(hipStreamSynchronize(st));
    free_scene(ctx->scene);
    ctx->scene = sc;
    ctx->node_levels = sc.n_nodes4 > 0 ? levels4 : std::vector<int32_t>{};
    return hipSuccess;
fail:
    hipStreamSynchronize(st);
    hipFree(boxes); hipFree(rbox); hipFree(mtmp); hipFree(bounds); hipFree(keys); hipFree(tk);
    hipFree(vals); hipFree(tv); hipFree(pnode); hipFree(pleaf); hipFree(flags);
    hipFree(pc_node); hipFree(pc_leaf); hipFree(pieces); hipFree(roff); hipFree(rprim); hipFree(rinfo);
    hipFree(emit_flag); hipFree(emit_pos); hipFree(depth); hipFree(berr); hipFree(maxd);
    free_scene(sc);
    return e == hipSuccess ? hipErrorUnknown : e;
}

hipError_t refit_scene(ugp_ctx ctx, const ugp_scene *s) {
    hipStream_t st = ctx->stream;
    SceneDev &sc = ctx->scene;
    const int64_t n = s->n, nr = sc.n_refs;
    PackIn in{n, s->mean, s->scale, s->rotation, s->density, s->albedo, s->roughness, s->emission,
              s->material, s->sggx, s->metallic, sc.r_cut};
    float *boxes = nullptr, *mtmp = nullptr, *lbox = nullptr;
    float4 *cold = nullptr, *sggx = nullptr;
    uint32_t *bounds = nullptr;
    int32_t *pieces = nullptr, *emit_flag = nullptr, *emit_pos = nullptr;
    uint32_t *berr = nullptr;
    hipError_t e = hipSuccess;
    uint32_t h_err = 0;
    int32_t h_nemit = 0, h_last_flag = 0;
    float rootb[24];
    const std::vector<int32_t> &lv = ctx->node_levels;
    // pack into temporaries and validate: on bad parameters the scene is left as it was
    UGP_CHECK(hipMallocAsync((void **)&boxes, sizeof(float) * 6 * n, st));
    UGP_CHECK(hipMallocAsync((void **)&mtmp, sizeof(float) * 9 * n, st));
    UGP_CHECK(hipMallocAsync((void **)&cold, sizeof(float4) * 3 * n, st));
    UGP_CHECK(hipMallocAsync((void **)&bounds, sizeof(uint32_t) * 8, st));
    UGP_CHECK(hipMallocAsync((void **)&pieces, sizeof(int32_t) * n, st));
    UGP_CHECK(hipMallocAsync((void **)&lbox, sizeof(float) * 6 * nr, st));
    UGP_CHECK(hipMallocAsync((void **)&emit_flag, sizeof(int32_t) * n, st));
    UGP_CHECK(hipMallocAsync((void **)&emit_pos, sizeof(int32_t) * n, st));
    UGP_CHECK(hipMallocAsync((void **)&berr, sizeof(uint32_t), st));
    UGP_CHECK(hipMemsetAsync(berr, 0, sizeof(uint32_t), st));
    hipLaunchKernelGGL(k_init_bounds, dim3(1), dim3(64), 0, st, bounds);
    if (s->sggx) UGP_CHECK(hipMallocAsync((void **)&sggx, sizeof(float4) * 8 * n, st));
    hipLaunchKernelGGL(k_pack, dim3(blocks(n)), dim3(kThreads), 0, st, in, boxes, cold, mtmp, bounds, pieces,
                       sggx, berr);
    UGP_CHECK(hipGetLastError());
    UGP_CHECK(hipMemcpyAsync(&h_err, berr, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    UGP_CHECK(hipStreamSynchronize(st));
    if (h_err & 8u) {
        e = hipErrorInvalidValue;
        goto fail;
    }
    sc.has_mat3 = (h_err & 32u) != 0;
    // records and leaf boxes, then the 4-wide nodes from the deepest level up
    UGP_CHECK(hipMemcpyAsync(sc.cold, cold, sizeof(float4) * 3 * n, hipMemcpyDeviceToDevice, st));
    if (sggx) {
        if (!sc.sggx) UGP_CHECK(hipMalloc((void **)&sc.sggx, sizeof(float4) * 8 * n));
        UGP_CHECK(hipMemcpyAsync(sc.sggx, sggx, sizeof(float4) * 8 * n, hipMemcpyDeviceToDevice, st));
    } else if (sc.sggx) {  // no material 2 or 3 any more (validated): drop the records
        UGP_CHECK(hipStreamSynchronize(st));
        hipFree(sc.sggx);
        sc.sggx = nullptr;
    }
    hipLaunchKernelGGL(k_refit_leaves, dim3(blocks(nr)), dim3(kThreads), 0, st, nr, in, (const float *)mtmp,
                       (const float *)boxes, sc.hot, lbox);
    for (int64_t L = (int64_t)lv.size() - 2; L >= 0; --L)
        if (lv[L + 1] > lv[L])
            hipLaunchKernelGGL(k_refit_nodes, dim3(blocks(lv[L + 1] - lv[L])), dim3(kThreads), 0, st, lv[L],
                               lv[L + 1], sc.nodes, (const float *)lbox);
    UGP_CHECK(hipGetLastError());
    // emitters and the scene bounds
    hipLaunchKernelGGL(k_emit_flags, dim3(blocks(n)), dim3(kThreads), 0, st, n, (const float4 *)sc.cold, emit_flag);
    UGP_CHECK(hipGetLastError());
    UGP_CHECK(exclusive_scan(emit_flag, emit_pos, n, st));
    UGP_CHECK(hipMemcpyAsync(&h_nemit, emit_pos + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st));
    UGP_CHECK(hipMemcpyAsync(&h_last_flag, emit_flag + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (sc.n_nodes4 > 0)
        UGP_CHECK(hipMemcpyAsync(rootb, sc.nodes, sizeof(float) * 24, hipMemcpyDeviceToHost, st));
    else
        UGP_CHECK(hipMemcpyAsync(rootb, lbox, sizeof(float) * 6, hipMemcpyDeviceToHost, st));
    UGP_CHECK(hipStreamSynchronize(st));
    h_nemit += h_last_flag;
    if (h_nemit != sc.n_emit) {
        hipFree(sc.emit);
        sc.emit = nullptr;
        sc.n_emit = 0;
        if (h_nemit > 0) UGP_CHECK(hipMalloc((void **)&sc.emit, sizeof(int32_t) * h_nemit));
    }
    if (h_nemit > 0) {
        hipLaunchKernelGGL(k_compact, dim3(blocks(n)), dim3(kThreads), 0, st, n, emit_flag, emit_pos, sc.emit);
        UGP_CHECK(hipGetLastError());
    }
    sc.n_emit = h_nemit;
    for (int c = 0; c < 3; ++c) {
        if (sc.n_nodes4 > 0) {  // the root's four child boxes (lo.c[4] at 4 c, hi.c[4] at 12 + 4 c)
            sc.lo[c] = std::min(std::min(rootb[4 * c], rootb[4 * c + 1]), std::min(rootb[4 * c + 2], rootb[4 * c + 3]));
            sc.hi[c] = std::max(std::max(rootb[12 + 4 * c], rootb[12 + 4 * c + 1]),
                                std::max(rootb[12 + 4 * c + 2], rootb[12 + 4 * c + 3]));
        } else {
            sc.lo[c] = rootb[c];
            sc.hi[c] = rootb[3 + c];
        }
    }
    hipFreeAsync(boxes, st); hipFreeAsync(mtmp, st); hipFreeAsync(cold, st); hipFreeAsync(sggx, st);
    hipFreeAsync(bounds, st);
    hipFreeAsync(pieces, st); hipFreeAsync(lbox, st); hipFreeAsync(emit_flag, st); hipFreeAsync(emit_pos, st);
    hipFreeAsync(berr, st);
    return hipSuccess;
fail:
    hipStreamSynchronize(st);
    hipFree(boxes); hipFree(mtmp); hipFree(cold); hipFree(sggx); hipFree(bounds); hipFree(pieces); hipFree(lbox);
    hipFree(emit_flag); hipFree(emit_pos); hipFree(berr);
    return e == hipSuccess ? hipErrorUnknown : e;
}

}  // namespace ugp
