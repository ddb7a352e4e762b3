// nrc.hip -- neural radiance cache: the learned part of the path tracer.
//
// A fully fused MLP 96 -> 64 -> 64 -> 64 -> 64 -> 3 (ReLU, no biases) with
// bf16 weights and activations and FP32 accumulation on the gfx950 matrix
// cores (v_mfma_f32_16x16x32_bf16), trained online with a relative-L2 loss
// and Adam on FP32 master weights.
//
// Input encoding (per query, 96 features): the position normalised to the
// scene box as sin / cos(2^j pi x) for j = 0..11 per axis (72), the outgoing
// direction as real spherical harmonics of bands 0..3 (16), the facet normal
// (3), roughness (1) and albedo (3), one zero pad.
//
// MFMA lane layout (16x16x32 bf16, wave64): lane l supplies A[row l%16][k =
// 8(l/16) .. +8], B[k = 8(l/16) .. +8][col l%16] and receives C[rows
// 4(l/16) .. +4][col l%16].  Activations are staged in LDS between layers
// (row-major 16 x K tiles per wave), weights sit in LDS for the whole kernel.
#include <hip/hip_runtime.h>

#include "ugp_internal.hpp"
#include "ugp_math.hpp"

namespace ugp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kNIn = 96, kNH = 64, kNOut = 3;
constexpr int kNParam = kNH * kNIn + 3 * kNH * kNH + kNOut * kNH;  // 18624
// forward-layout bf16 weights: per layer [n_out][n_in]; the output layer is
// padded to 16 rows
constexpr int kWfOff[5] = {0, 6144, 10240, 14336, 18432};
constexpr int kWfSize = 18432 + 16 * 64;
// backward-layout bf16 weights (transposed, layers 1..4): [n_in][n_out_pad]
// with n_out_pad = 64 (layers 1..3) or 32 (the output layer)
constexpr int kWbOff[5] = {0, 0, 4096, 8192, 12288};
constexpr int kWbSize = 12288 + 64 * 32;
constexpr int kMOff[5] = {0, 6144, 10240, 14336, 18432};  // master weight offsets

struct NrcState {
    float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    float *scale = nullptr;    // radiance unit of the network's output (device; <= 0: not set yet)
    int32_t *bcnt = nullptr;   // per-batch record counts of a render's training steps
    __bf16 *wf = nullptr, *wb = nullptr;
    int step = 0;
    // training buffers for up to cap records
    int64_t cap = 0;
    __bf16 *act[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // inputs of the 5 layers
    __bf16 *delta[5] = {nullptr, nullptr, nullptr, nullptr, nullptr}; // dL/d(pre-activation) per layer
    float *y = nullptr, *part = nullptr, *loss = nullptr;
    void *block = nullptr;
};

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kActStride = 104;  // bf16 per LDS activation row (96 + 8 pad)

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 ld8(const __bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

// encode one quarter of a query's features: group g = 0,1,2 the sinusoids of
// one axis (24 values), g = 3 the harmonics, normal, roughness, albedo, pad
__device__ __forceinline__ void encode_group(const float *in, int g, const double *lo, const double *inv_ext,
                                             float f[24]) {
    if (g < 3) {
        // x_hat in double so that 2^11 pi x_hat keeps its phase; the argument
        // 2^j x_hat is reduced exactly modulo 2 (units of pi) before sincospi
        const double xh = ((double)in[g] - lo[g]) * inv_ext[g];
#pragma unroll
        for (int j = 0; j < 12; ++j) {
            const double a = ldexp(xh, j);
            const float fr = (float)(a - 2.0 * floor(0.5 * a));  // in [0, 2]
            float s, c;
            sincospif(fr, &s, &c);
            f[2 * j] = s;
            f[2 * j + 1] = c;
        }
        return;
    }
    const float x = in[3], y = in[4], z = in[5];
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    f[0] = 0.28209479177387814f;
    f[1] = -0.48860251190291987f * y;
    f[2] = 0.48860251190291987f * z;
    f[3] = -0.48860251190291987f * x;
    f[4] = 1.0925484305920792f * x * y;
    f[5] = -1.0925484305920792f * y * z;
    f[6] = 0.31539156525252005f * (3.f * z2 - 1.f);
    f[7] = -1.0925484305920792f * x * z;
    f[8] = 0.5462742152960396f * (x2 - y2);
    f[9] = -0.5900435899266435f * y * (3.f * x2 - y2);
    f[10] = 2.890611442640554f * x * y * z;
    f[11] = -0.4570457994644658f * y * (5.f * z2 - 1.f);
    f[12] = 0.3731763325901154f * z * (5.f * z2 - 3.f);
    f[13] = -0.4570457994644658f * x * (5.f * z2 - 1.f);
    f[14] = 1.445305721320277f * z * (x2 - y2);
    f[15] = -0.5900435899266435f * x * (x2 - 3.f * y2);
#pragma unroll
    for (int k = 0; k < 7; ++k) f[16 + k] = in[6 + k];
    f[23] = 0.f;
}

struct EncodeBox {
    double lo[3], inv_ext[3];
};

// device-side record count: min(*dev, host) when dev is given
__device__ __forceinline__ int64_t rec_count(int64_t n_host, const int32_t *n_dev) {
    if (!n_dev) return n_host;
    const int64_t d = (int64_t)*n_dev;
    return d < n_host ? d : n_host;
}

__global__ void k_nrc_encode(int64_t n, const float *inputs, int stride, EncodeBox box, float *feat) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * n) return;
    const int64_t r = t >> 2;
    const int g = (int)(t & 3);
    float f[24];
    encode_group(inputs + (int64_t)stride * r, g, box.lo, box.inv_ext, f);
    for (int k = 0; k < 24; ++k) feat[96 * r + 24 * g + k] = f[k];
}

// copy the forward weights (bf16) into LDS
__device__ __forceinline__ void load_weights(const __bf16 *wf, __bf16 *sw) {
    const uint4 *src = reinterpret_cast<const uint4 *>(wf);
    uint4 *dst = reinterpret_cast<uint4 *>(sw);
    for (int i = threadIdx.x; i < kWfSize / 8; i += blockDim.x) dst[i] = src[i];
}

// one hidden layer on a 16-row tile: out[16][64] = relu(in[16][K] W^T)
template <int K>
__device__ __forceinline__ void layer_relu(const __bf16 *in, const __bf16 *W, __bf16 *out, int lane) {
    const int col = lane & 15, grp = lane >> 4;
    f32x4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < K / 32; ++ks) {
        const bf16x8 a = ld8(in + col * kActStride + ks * 32 + grp * 8);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma(a, ld8(W + (nt * 16 + col) * K + ks * 32 + grp * 8), acc[nt]);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            out[(grp * 4 + i) * kActStride + nt * 16 + col] = (__bf16)fmaxf(acc[nt][i], 0.f);
}

struct SavePtrs {
    __bf16 *p[5];  // layer inputs: [n][96], then [n][64] x 4; p[0] == nullptr: nothing saved
};

// Forward pass over n records.  MODE 0: raw inputs (16 floats at src + stride
// * r) encoded here, y[n][3] written; MODE 1: features [n][96] given, y
// written; MODE 2: raw inputs as MODE 0 followed by a weight (rgb) and path
// index (int bits) at floats 16..19 of the record -- the prediction, clamped
// at 0, times the radiance unit *scale (1 if unset) and the weight, is added
// to L[path] (one record per path).
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_nrc_forward(int64_t n_host, const int32_t *n_dev, const float *src,
                                                          int stride, EncodeBox box, const __bf16 *wf, float *y,
                                                          float4 *L, SavePtrs save, const float *scale) {
    __shared__ __attribute__((aligned(16))) __bf16 sw[kWfSize];
    __shared__ __attribute__((aligned(16))) __bf16 sact[kWaves][2][16 * kActStride];
    const int64_t n = rec_count(n_host, n_dev);
    const int64_t ntiles = (n + 15) / 16;
    // every wave of a block runs the same number of iterations (barriers)
    const int64_t per_block = (ntiles + (int64_t)gridDim.x * kWaves - 1) / ((int64_t)gridDim.x * kWaves);
    if (per_block == 0) return;
    load_weights(wf, sw);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, grp = lane >> 4;
    const bool do_save = save.p[0] != nullptr;
    for (int64_t it = 0; it < per_block; ++it) {
        const int64_t tile = ((int64_t)blockIdx.x * per_block + it) * kWaves + wave;
        const bool live = tile < ntiles;
        __bf16 *a0 = sact[wave][0], *a1 = sact[wave][1];
        if (live) {
            // stage the 16 x 96 input tile: lane (row col, quarter grp)
            const int64_t r = tile * 16 + col;
            float f[24];
            if (r < n) {
                if (MODE != 1) {
                    encode_group(src + (int64_t)stride * r, grp, box.lo, box.inv_ext, f);
                } else {
#pragma unroll
                    for (int k = 0; k < 24; ++k) f[k] = src[96 * r + 24 * grp + k];
                }
            } else {
#pragma unroll
                for (int k = 0; k < 24; ++k) f[k] = 0.f;
            }
#pragma unroll
            for (int k = 0; k < 24; ++k) a0[col * kActStride + 24 * grp + k] = (__bf16)f[k];
        }
        __syncthreads();
        if (live && do_save) {
            for (int e = lane; e < 16 * 96; e += 64) {
                const int rr = e / 96, c = e % 96;
                if (tile * 16 + rr < n) save.p[0][(tile * 16 + rr) * 96 + c] = a0[rr * kActStride + c];
            }
        }
        if (live) layer_relu<96>(a0, sw + kWfOff[0], a1, lane);
        __syncthreads();
#pragma unroll
        for (int l = 1; l < 4; ++l) {
            __bf16 *in = (l & 1) ? a1 : a0, *out = (l & 1) ? a0 : a1;
            if (live && do_save) {
                for (int e = lane; e < 16 * 64; e += 64) {
                    const int rr = e / 64, c = e % 64;
                    if (tile * 16 + rr < n) save.p[l][(tile * 16 + rr) * 64 + c] = in[rr * kActStride + c];
                }
            }
            if (live) layer_relu<64>(in, sw + kWfOff[l], out, lane);
            __syncthreads();
        }
        // output layer: 64 -> 3 (16 padded columns), no activation
        if (live) {
            const __bf16 *in = a0;
            if (do_save) {
                for (int e = lane; e < 16 * 64; e += 64) {
                    const int rr = e / 64, c = e % 64;
                    if (tile * 16 + rr < n) save.p[4][(tile * 16 + rr) * 64 + c] = in[rr * kActStride + c];
                }
            }
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                acc = mfma(ld8(in + col * kActStride + ks * 32 + grp * 8),
                           ld8(sw + kWfOff[4] + col * 64 + ks * 32 + grp * 8), acc);
            if (col < 3) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t r = tile * 16 + grp * 4 + i;
                    if (r < n) {
                        if (MODE == 2) {
                            const float *rec = src + (int64_t)stride * r;
                            const int pix = __float_as_int(rec[19]) & 0x3fffffff;
                            const float unit = (scale && *scale > 0.f) ? *scale : 1.f;
                            float *lp = reinterpret_cast<float *>(L + pix) + col;
                            *lp += rec[16 + col] * unit * fmaxf(acc[i], 0.f);
                        } else {
                            y[3 * r + col] = acc[i];
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Relative L2 loss, mean over records and channels of (y - t)^2 / (y^2 +
// 0.01) with the denominator held constant, targets in units of *tscale (if
// given and set) and clamped at tclamp (if > 0); writes dL/dy as bf16 [n][32]
// (columns >= 3 zero) and per-block loss partial sums.
__global__ void k_nrc_loss(int64_t n_host, const int32_t *n_dev, const float *y, const float *t, const float *tscale,
                           float tclamp, __bf16 *d4, float *loss_part) {
    __shared__ float red[256];
    const int64_t n = rec_count(n_host, n_dev);
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (r < n) {
        const float scale = 1.f / (3.f * (float)n);
        const float tinv = (tscale && *tscale > 0.f) ? 1.f / *tscale : 1.f;
        for (int c = 0; c < 32; ++c) {
            float g = 0.f;
            if (c < 3) {
                float tt = t[3 * r + c] * tinv;
                if (tclamp > 0.f) tt = fminf(tt, tclamp);
                const float yy = y[3 * r + c], e = yy - tt;
                const float den = yy * yy + 0.01f;
                l += e * e / den * scale;
                g = 2.f * e / den * scale;
            }
            d4[32 * r + c] = (__bf16)g;
        }
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// delta_{l-1} = (delta_l W_l) * [act_l > 0] on 16-row tiles; KO is the padded
// n_out of layer l (the row stride of delta_l)
template <int KO>
__global__ __launch_bounds__(kThreads) void k_nrc_backprop(int64_t n_host, const int32_t *n_dev, const __bf16 *dl,
                                                           const __bf16 *wbl, const __bf16 *actl, __bf16 *dprev) {
    __shared__ __attribute__((aligned(16))) __bf16 sw[64 * KO];
    for (int i = threadIdx.x; i < 64 * KO / 8; i += blockDim.x)
        reinterpret_cast<uint4 *>(sw)[i] = reinterpret_cast<const uint4 *>(wbl)[i];
    __syncthreads();
    const int64_t n = rec_count(n_host, n_dev);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, grp = lane >> 4;
    const int64_t ntiles = (n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < ntiles; tile += (int64_t)gridDim.x * kWaves) {
        const int64_t r = tile * 16 + col;
        f32x4 acc[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KO / 32; ++ks) {
            bf16x8 a = bf16x8{};
            if (r < n) a = ld8(dl + r * KO + ks * 32 + grp * 8);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[nt] = mfma(a, ld8(sw + (nt * 16 + col) * KO + ks * 32 + grp * 8), acc[nt]);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t rr = tile * 16 + grp * 4 + i;
                if (rr < n) {
                    const int c = nt * 16 + col;
                    const bool on = (float)actl[rr * 64 + c] > 0.f;
                    dprev[rr * 64 + c] = (__bf16)(on ? acc[nt][i] : 0.f);
                }
            }
    }
}

// Weight-gradient partials of one layer, dW[o][i] = sum_r delta[r][o] act[r][i]
// over this block's slice of records, on the matrix cores with the records as
// the contraction dimension.  NO: row stride of delta (64 or 32); NOUT: real
// outputs; NIN: inputs.
template <int NO, int NOUT, int NIN>
__global__ __launch_bounds__(64) void k_nrc_wgrad(int64_t n_host, const int32_t *n_dev, const __bf16 *delta,
                                                   const __bf16 *act, int64_t rows_per_block, float *part) {
    constexpr int OT = (NOUT + 15) / 16, IT = NIN / 16;
    __shared__ __attribute__((aligned(16))) __bf16 sd[32 * NO];
    __shared__ __attribute__((aligned(16))) __bf16 sa[32 * NIN];
    const int64_t n = rec_count(n_host, n_dev);
    const int lane = threadIdx.x;
    const int col = lane & 15, grp = lane >> 4;
    f32x4 acc[OT][IT];
#pragma unroll
    for (int a = 0; a < OT; ++a)
#pragma unroll
        for (int b = 0; b < IT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = r0 + rows_per_block < n ? r0 + rows_per_block : n;
    for (int64_t rb = r0; rb < r1; rb += 32) {
        // stage 32 records of delta and of the layer input (zero past the end)
        for (int e = lane; e < 32 * NO / 8; e += 64) {
            const int rr = e / (NO / 8);
            uint4 v = make_uint4(0, 0, 0, 0);
            if (rb + rr < r1) v = reinterpret_cast<const uint4 *>(delta + (rb + rr) * NO)[e % (NO / 8)];
            reinterpret_cast<uint4 *>(sd)[e] = v;
        }
        for (int e = lane; e < 32 * NIN / 8; e += 64) {
            const int rr = e / (NIN / 8);
            uint4 v = make_uint4(0, 0, 0, 0);
            if (rb + rr < r1) v = reinterpret_cast<const uint4 *>(act + (rb + rr) * NIN)[e % (NIN / 8)];
            reinterpret_cast<uint4 *>(sa)[e] = v;
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < OT; ++a) {
            bf16x8 fa;
#pragma unroll
            for (int j = 0; j < 8; ++j) fa[j] = sd[(grp * 8 + j) * NO + a * 16 + col];
#pragma unroll
            for (int b = 0; b < IT; ++b) {
                bf16x8 fb;
#pragma unroll
                for (int j = 0; j < 8; ++j) fb[j] = sa[(grp * 8 + j) * NIN + b * 16 + col];
                acc[a][b] = mfma(fa, fb, acc[a][b]);
            }
        }
        __syncthreads();
    }
    // C tile (a, b): rows o = a*16 + grp*4 + i, column i_in = b*16 + col
    float *out = part + (int64_t)blockIdx.x * NOUT * NIN;
#pragma unroll
    for (int a = 0; a < OT; ++a)
#pragma unroll
        for (int b = 0; b < IT; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = a * 16 + grp * 4 + i;
                if (o < NOUT) out[o * NIN + b * 16 + col] = acc[a][b][i];
            }
}

// Weight gradient of every layer from its record-slice partials ([slice][layer
// params] per layer): grad[p] = sum over the nb slices, in a fixed order --
// row y of a block sums slices y, y + 16, y + 32, ... in turn, then the 16
// rows are added in row order.  64 parameters x 16 rows per block, one launch
// for all layers (the slices are independent loads, summed 16 at a time).
__global__ __launch_bounds__(1024) void k_nrc_reduce_grad(int nb, const float *part, float *grad) {
    __shared__ float red[16][64];
    const int x = threadIdx.x & 63, y = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + x;
    float s = 0.f;
    if (p < kNParam) {
        const int l = p < kMOff[1] ? 0 : p < kMOff[2] ? 1 : p < kMOff[3] ? 2 : p < kMOff[4] ? 3 : 4;
        const int np = (l == 4 ? kNParam : kMOff[l + 1]) - kMOff[l];
        const float *base = part + (int64_t)nb * kMOff[l] + (p - kMOff[l]);
        for (int b = y; b < nb; b += 16) s += base[(int64_t)b * np];
    }
    red[y][x] = s;
    __syncthreads();
    if (y == 0 && p < kNParam) {
        float t = 0.f;
        for (int k = 0; k < 16; ++k) t += red[k][x];
        grad[p] = t;
    }
}

// out[p] = sum over b < nblocks of part[b][p], in block order
__global__ void k_nrc_reduce(int nblocks, int np, const float *part, float *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * np + p];
    out[p] = s;
}

// bf16 copies of the master weights in the forward layout ([n_out][n_in] per
// layer, output layer padded to 16 rows) and the transposed layout of layers
// 1..4 ([n_in][n_out_pad]).  Every index is written by exactly one thread.
__global__ void k_nrc_publish(const float *master, __bf16 *wf, __bf16 *wb) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    // padding: rows 3..15 of the forward output layer, columns 3..31 of the
    // transposed output layer
    if (p >= kWfOff[4] + 3 * 64 && p < kWfSize) wf[p] = (__bf16)0.f;
    if (p >= kWbOff[4] && p < kWbSize && ((p - kWbOff[4]) & 31) >= 3) wb[p] = (__bf16)0.f;
    if (p >= kNParam) return;
    const int l = p < kMOff[1] ? 0 : p < kMOff[2] ? 1 : p < kMOff[3] ? 2 : p < kMOff[4] ? 3 : 4;
    const int nin = l == 0 ? kNIn : kNH;
    const int o = (p - kMOff[l]) / nin, i = (p - kMOff[l]) % nin;
    const __bf16 w = (__bf16)master[p];
    wf[kWfOff[l] + o * nin + i] = w;
    if (l >= 1) wb[kWbOff[l] + i * (l == 4 ? 32 : 64) + o] = w;
}

// Adam (Kingma and Ba 2015) with bias correction on the FP32 master weights;
// c1, c2 = 1 - beta^t
__global__ void k_nrc_adam(int np, float *master, float *m, float *v, const float *g, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const float gg = g[p];
    const float mm = b1 * m[p] + (1.f - b1) * gg;
    const float vv = b2 * v[p] + (1.f - b2) * gg * gg;
    m[p] = mm;
    v[p] = vv;
    master[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// training targets of collected path records: (L[pixel] - L_prefix) / beta per
// channel (0 where beta is 0); record layout in nrc_build_targets
__global__ void k_nrc_targets(int64_t n_host, const int32_t *n_dev, const float *rec, const float4 *L,
                              float *targets) {
    const int64_t n = rec_count(n_host, n_dev);
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const float *q = rec + (int64_t)kNrcRecordFloats * r;
    const int pix = __float_as_int(q[19]) & 0x3fffffff;
    const float4 l = L[pix];
    const float tot[3] = {l.x, l.y, l.z};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float b = q[16 + c];
        targets[3 * r + c] = b > 0.f ? fmaxf(0.f, tot[c] - q[20 + c]) / b : 0.f;
    }
}

__global__ void k_nrc_adapt(const int32_t *attempted, int32_t cap, float *frac) {
    const float a = (float)*attempted;
    float f = *frac;
    f = a > 0.f ? f * fminf(4.f, fmaxf(0.25f, (float)cap / a)) : f * 4.f;
    *frac = fminf(1.f, fmaxf(1e-5f, f));
}

// radiance unit from the first training batch: the mean target (once)
__global__ void k_nrc_scale_init(int64_t n_host, const int32_t *n_dev, const float *targets, float *scale) {
    __shared__ float red[256];
    if (*scale > 0.f) return;
    const int64_t n = rec_count(n_host, n_dev);
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < 3 * n; i += blockDim.x) s += targets[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0 && n > 0 && red[0] > 0.f) *scale = red[0] / (3.f * (float)n);
}

// record count of each of `steps` batches of `per` records
__global__ void k_nrc_batches(const int32_t *n_dev, int64_t cap, int steps, int64_t per, int32_t *bcnt) {
    const int b = threadIdx.x;
    if (b >= steps) return;
    const int64_t n = (int64_t)*n_dev < cap ? (int64_t)*n_dev : cap;
    const int64_t left = n - (int64_t)b * per;
    bcnt[b] = (int32_t)(left < 0 ? 0 : (left > per ? per : left));
}

__global__ void k_nrc_set(float *p, float v) { *p = v; }

EncodeBox make_box(ugp_ctx ctx, const float *box) {
    EncodeBox b;
    for (int k = 0; k < 3; ++k) {
        const double lo = box ? (double)box[k] : (double)ctx->scene.lo[k];
        const double hi = box ? (double)box[3 + k] : (double)ctx->scene.hi[k];
        b.lo[k] = lo;
        b.inv_ext[k] = hi > lo ? 1.0 / (hi - lo) : 0.0;
    }
    return b;
}

unsigned fwd_grid(int64_t n) {
    const int64_t tiles = (n + 15) / 16;
    const int64_t g = (tiles + kWaves - 1) / kWaves;
    return (unsigned)(g < 2048 ? (g > 0 ? g : 1) : 2048);
}

constexpr int kParts = 1024;  // record slices of the weight gradient

}  // namespace

int nrc_num_params() { return kNParam; }

hipError_t nrc_ensure(ugp_ctx ctx) {
    if (ctx->nrc) return hipSuccess;
    NrcState *s = new NrcState();
    hipError_t e = hipMalloc((void **)&s->master, sizeof(float) * kNParam * 4 + 1024);
    if (e != hipSuccess) {
        delete s;
        return e;
    }
    s->m = s->master + kNParam;
    s->v = s->m + kNParam;
    s->grad = s->v + kNParam;
    s->scale = s->grad + kNParam;
    s->bcnt = reinterpret_cast<int32_t *>(s->scale + 64);
    e = hipMalloc((void **)&s->wf, sizeof(__bf16) * (kWfSize + kWbSize));
    if (e != hipSuccess) {
        hipFree(s->master);
        delete s;
        return e;
    }
    s->wb = s->wf + kWfSize;
    hipMemsetAsync(s->master, 0, sizeof(float) * kNParam * 4 + 1024, ctx->stream);
    hipMemsetAsync(s->wf, 0, sizeof(__bf16) * (kWfSize + kWbSize), ctx->stream);
    ctx->nrc = s;
    return hipSuccess;
}

void nrc_free(ugp_ctx ctx) {
    if (!ctx->nrc) return;
    hipFree(ctx->nrc->master);
    hipFree(ctx->nrc->wf);
    hipFree(ctx->nrc->block);
    delete ctx->nrc;
    ctx->nrc = nullptr;
}

bool nrc_ready(ugp_ctx ctx) { return ctx->nrc != nullptr; }

hipError_t nrc_set_weights(ugp_ctx ctx, const float *w) {
    hipError_t e = nrc_ensure(ctx);
    if (e != hipSuccess) return e;
    NrcState *s = ctx->nrc;
    e = hipMemcpyAsync(s->master, w, sizeof(float) * kNParam, hipMemcpyDeviceToDevice, ctx->stream);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(s->m, 0, sizeof(float) * kNParam * 2, ctx->stream);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(s->scale, 0, sizeof(float), ctx->stream);  // radiance unit: set by the next training
    if (e != hipSuccess) return e;
    s->step = 0;
    ctx->nrc_frac_pixels = 0;  // the next training render starts the training-path probability afresh
    hipLaunchKernelGGL(k_nrc_publish, dim3((kWfSize + 255) / 256), dim3(256), 0, ctx->stream, (const float *)s->master,
                       s->wf, s->wb);
    return hipGetLastError();
}

hipError_t nrc_get_weights(ugp_ctx ctx, float *w) {
    if (!ctx->nrc) return hipErrorNotReady;
    return hipMemcpyAsync(w, ctx->nrc->master, sizeof(float) * kNParam, hipMemcpyDeviceToDevice, ctx->stream);
}

hipError_t nrc_encode(ugp_ctx ctx, int64_t n, const float *inputs, int stride, const float *box, float *feat) {
    const EncodeBox b = make_box(ctx, box);
    hipLaunchKernelGGL(k_nrc_encode, dim3((unsigned)((4 * n + 255) / 256)), dim3(256), 0, ctx->stream, n, inputs,
                       stride, b, feat);
    return hipGetLastError();
}

hipError_t nrc_forward(ugp_ctx ctx, int64_t n, const int32_t *n_dev, const float *src, int stride, int src_kind,
                       const float *box, float *y, float4 *L, const float *scale) {
    if (!ctx->nrc) return hipErrorNotReady;
    const EncodeBox b = make_box(ctx, box);
    const SavePtrs none{{nullptr, nullptr, nullptr, nullptr, nullptr}};
    const __bf16 *wf = ctx->nrc->wf;
    const dim3 g(fwd_grid(n)), t(kThreads);
    if (src_kind == 0)
        hipLaunchKernelGGL((k_nrc_forward<0>), g, t, 0, ctx->stream, n, n_dev, src, stride, b, wf, y, L, none, scale);
    else if (src_kind == 1)
        hipLaunchKernelGGL((k_nrc_forward<1>), g, t, 0, ctx->stream, n, n_dev, src, stride, b, wf, y, L, none, scale);
    else
        hipLaunchKernelGGL((k_nrc_forward<2>), g, t, 0, ctx->stream, n, n_dev, src, stride, b, wf, y, L, none, scale);
    return hipGetLastError();
}

static hipError_t nrc_train_buffers(ugp_ctx ctx, int64_t n) {
    NrcState *s = ctx->nrc;
    if (s->cap >= n) return hipSuccess;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return e;
    hipFree(s->block);
    s->block = nullptr;
    s->cap = 0;
    const int64_t cap = n < 4096 ? 4096 : n;
    const int64_t loss_parts = (cap + 255) / 256;
    const size_t bytes = sizeof(__bf16) * (size_t)cap * (96 + 4 * 64)  // layer inputs
                         + sizeof(__bf16) * (size_t)cap * (4 * 64 + 32)  // deltas
                         + sizeof(float) * (size_t)cap * 3              // outputs
                         + sizeof(float) * (size_t)kParts * kNParam     // gradient partials
                         + sizeof(float) * (size_t)loss_parts + 16 * 256;
    e = hipMalloc(&s->block, bytes);
    if (e != hipSuccess) return e;
    char *p = (char *)s->block;
    auto take = [&](size_t b) {
        void *r = p;
        p += (b + 255) & ~(size_t)255;
        return r;
    };
    s->act[0] = (__bf16 *)take(sizeof(__bf16) * cap * 96);
    for (int l = 1; l < 5; ++l) s->act[l] = (__bf16 *)take(sizeof(__bf16) * cap * 64);
    for (int l = 0; l < 4; ++l) s->delta[l] = (__bf16 *)take(sizeof(__bf16) * cap * 64);
    s->delta[4] = (__bf16 *)take(sizeof(__bf16) * cap * 32);
    s->y = (float *)take(sizeof(float) * cap * 3);
    s->part = (float *)take(sizeof(float) * kParts * kNParam);
    s->loss = (float *)take(sizeof(float) * loss_parts);
    s->cap = cap;
    return hipSuccess;
}

// One optimisation step on n records (at most *n_dev when given): forward with
// saved layer inputs, loss and its gradient, back-propagation, weight
// gradients (per-slice partials reduced in a fixed order), Adam, new bf16
// copies.  grad_out / loss_out (device, optional) receive the gradient and
// the loss of this step.
static hipError_t train_step_impl(ugp_ctx ctx, int64_t n, const int32_t *n_dev, const float *src, int stride,
                                  int src_kind, const float *box, const float *targets, const float *tscale,
                                  float tclamp, float lr, float *loss_out, float *grad_out) {
    if (!ctx->nrc) return hipErrorNotReady;
    NrcState *s = ctx->nrc;
    hipError_t e = nrc_train_buffers(ctx, n);
    if (e != hipSuccess) return e;
    hipStream_t st = ctx->stream;
    const EncodeBox b = make_box(ctx, box);
    SavePtrs save;
    for (int l = 0; l < 5; ++l) save.p[l] = s->act[l];
    const dim3 g(fwd_grid(n)), t(kThreads);
    if (src_kind == 1)
        hipLaunchKernelGGL((k_nrc_forward<1>), g, t, 0, st, n, n_dev, src, stride, b, (const __bf16 *)s->wf, s->y,
                           (float4 *)nullptr, save, (const float *)nullptr);
    else
        hipLaunchKernelGGL((k_nrc_forward<0>), g, t, 0, st, n, n_dev, src, stride, b, (const __bf16 *)s->wf, s->y,
                           (float4 *)nullptr, save, (const float *)nullptr);
    const unsigned lb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_nrc_loss, dim3(lb), dim3(256), 0, st, n, n_dev, (const float *)s->y, targets, tscale,
                       tclamp, s->delta[4], s->loss);
    hipLaunchKernelGGL((k_nrc_backprop<32>), g, t, 0, st, n, n_dev, (const __bf16 *)s->delta[4],
                       (const __bf16 *)(s->wb + kWbOff[4]), (const __bf16 *)s->act[4], s->delta[3]);
    for (int l = 3; l >= 1; --l)
        hipLaunchKernelGGL((k_nrc_backprop<64>), g, t, 0, st, n, n_dev, (const __bf16 *)s->delta[l],
                           (const __bf16 *)(s->wb + kWbOff[l]), (const __bf16 *)s->act[l], s->delta[l - 1]);
    // weight gradients: up to kParts record slices (multiples of 32 records),
    // stored per layer as [slice][layer params]
    const int64_t rpb = ((n + kParts - 1) / kParts + 31) / 32 * 32;
    const int nb = (int)((n + rpb - 1) / rpb);
    hipLaunchKernelGGL((k_nrc_wgrad<64, 64, 96>), dim3(nb), dim3(64), 0, st, n, n_dev, (const __bf16 *)s->delta[0],
                       (const __bf16 *)s->act[0], rpb, s->part + (int64_t)nb * kMOff[0]);
    for (int l = 1; l < 4; ++l)
        hipLaunchKernelGGL((k_nrc_wgrad<64, 64, 64>), dim3(nb), dim3(64), 0, st, n, n_dev, (const __bf16 *)s->delta[l],
                           (const __bf16 *)s->act[l], rpb, s->part + (int64_t)nb * kMOff[l]);
    hipLaunchKernelGGL((k_nrc_wgrad<32, 3, 64>), dim3(nb), dim3(64), 0, st, n, n_dev, (const __bf16 *)s->delta[4],
                       (const __bf16 *)s->act[4], rpb, s->part + (int64_t)nb * kMOff[4]);
    hipLaunchKernelGGL(k_nrc_reduce_grad, dim3((kNParam + 63) / 64), dim3(1024), 0, st, nb, (const float *)s->part,
                       s->grad);
    if (grad_out) {
        e = hipMemcpyAsync(grad_out, s->grad, sizeof(float) * kNParam, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    if (loss_out)
        hipLaunchKernelGGL(k_nrc_reduce, dim3(1), dim3(256), 0, st, (int)lb, 1, (const float *)s->loss, loss_out);
    s->step += 1;
    const float b1 = 0.9f, b2 = 0.99f;
    const float c1 = (float)(1.0 - pow((double)b1, (double)s->step));
    const float c2 = (float)(1.0 - pow((double)b2, (double)s->step));
    hipLaunchKernelGGL(k_nrc_adam, dim3((kNParam + 255) / 256), dim3(256), 0, st, kNParam, s->master, s->m, s->v,
                       (const float *)s->grad, lr, b1, b2, 1e-8f, c1, c2);
    hipLaunchKernelGGL(k_nrc_publish, dim3((kWfSize + 255) / 256), dim3(256), 0, st, (const float *)s->master, s->wf,
                       s->wb);
    return hipGetLastError();
}

hipError_t nrc_train_step(ugp_ctx ctx, int64_t n, const int32_t *n_dev, const float *src, int stride, int src_kind,
                          const float *box, const float *targets, float lr, float *loss_out, float *grad_out) {
    return train_step_impl(ctx, n, n_dev, src, stride, src_kind, box, targets, nullptr, 0.f, lr, loss_out, grad_out);
}

// Training of a render: the radiance unit is set from the first batch's
// targets (unless given), then `steps` Adam steps on consecutive batches of
// the records (targets in that unit).
hipError_t nrc_train_render(ugp_ctx ctx, int64_t cap, const int32_t *n_dev, const float *rec, const float *box,
                            const float *targets, float lr, int steps, float tclamp, float *loss_out) {
    NrcState *s = ctx->nrc;
    if (!s) return hipErrorNotReady;
    if (steps > 64) steps = 64;
    hipLaunchKernelGGL(k_nrc_scale_init, dim3(1), dim3(256), 0, ctx->stream, cap, n_dev, targets, s->scale);
    const int64_t per = (cap + steps - 1) / steps;
    hipLaunchKernelGGL(k_nrc_batches, dim3(1), dim3(64), 0, ctx->stream, n_dev, cap, steps, per, s->bcnt);
    hipError_t e = hipGetLastError();
    for (int b = 0; b < steps && e == hipSuccess; ++b)
        e = train_step_impl(ctx, per, s->bcnt + b, rec + (int64_t)kNrcRecordFloats * per * b, kNrcRecordFloats, 0,
                            box, targets + 3 * per * b, s->scale, tclamp, lr, loss_out, nullptr);
    return e;
}

hipError_t nrc_set_scale(ugp_ctx ctx, float value) {
    if (!ctx->nrc) return hipErrorNotReady;
    if (value > 0.f) hipLaunchKernelGGL(k_nrc_set, dim3(1), dim3(1), 0, ctx->stream, ctx->nrc->scale, value);
    return hipGetLastError();
}

const float *nrc_scale_ptr(ugp_ctx ctx) { return ctx->nrc ? ctx->nrc->scale : nullptr; }

hipError_t nrc_targets(ugp_ctx ctx, int64_t cap, const int32_t *n_dev, const float *rec, const float4 *L,
                       float *targets) {
    hipLaunchKernelGGL(k_nrc_targets, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, ctx->stream, cap, n_dev, rec,
                       L, targets);
    return hipGetLastError();
}

hipError_t nrc_adapt(ugp_ctx ctx, const int32_t *attempted, int32_t cap, float *frac) {
    hipLaunchKernelGGL(k_nrc_adapt, dim3(1), dim3(1), 0, ctx->stream, attempted, cap, frac);
    return hipGetLastError();
}

}  // namespace ugp
