// Learned correction network: forward, backward and optimiser kernels.
//
// The two 32 -> 32 convolutions (94% of the arithmetic) run on the gfx950 matrix
// cores as implicit GEMMs: one wavefront computes 32 consecutive pixels of an
// image row times the 32 output channels with v_mfma_f32_32x32x16_bf16, the
// reduction running over 9 taps x 2 chunks of 16 input channels.  Operand
// fragments are 16-byte LDS reads (8 consecutive channels of one pixel per lane)
// of an input tile and of the [tap][n][k] BF16 weights, both staged per workgroup;
// accumulation is FP32.  The weights are the A operand, so each lane ends
// with runs of four consecutive output channels of one pixel, stored 8 bytes at a
// time.  The weight gradient of those layers is the same contraction with the pixel
// index as the reduction, also on MFMA.  The
// 3 -> 32 input layer, the 32 -> 1 output layer and their gradients are small
// and run on the vector ALUs in FP32.
//
// MFMA 32x32x16 operand layout (lane l of the wavefront): A[m][k] with m = l % 32,
// k = 8 (l / 32) + j, j = 0..7 in the lane's 8 BF16 values; B[k][n] with n = l % 32,
// same k; result D[m][n] in 16 FP32 registers, n = l % 32,
// m = 8 (i / 4) + 4 (l / 32) + i % 4 for register i.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "net.h"

namespace hpadi {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr float kGeluC = 0.7978845608028654f;  // sqrt(2/pi)
constexpr float kGeluA = 0.044715f;

// tanh(u) = 1 - 2 / (1 + e^(2u)) with the hardware exponential (saturates to +-1 for large |u|)
__device__ inline float fast_tanh(float u) { return 1.0f - __fdividef(2.0f, 1.0f + __expf(2.0f * u)); }
__device__ inline float gelu(float x) {
    return 0.5f * x * (1.0f + fast_tanh(kGeluC * (x + kGeluA * x * x * x)));
}
__device__ inline float gelu_grad(float x) {
    const float t = fast_tanh(kGeluC * (x + kGeluA * x * x * x));
    return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * kGeluC * (1.0f + 3.0f * kGeluA * x * x);
}
// round to nearest even (finite inputs)
__device__ inline bf16_t f2bf(float f) {
    const unsigned u = __float_as_uint(f);
    return (bf16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf2f(bf16_t h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ inline void pix_of(long p, const ImgShape& s, int& b, int& h, int& w) {
    w = (int)(p % s.W);
    const long t = p / s.W;
    h = (int)(t % s.H);
    b = (int)(t / s.H);
}

// ---- first layer: 3 -> 32 -------------------------------------------------
// A workgroup computes 4 rows x 64 pixels; the 3-channel input of the tile plus a
// one-pixel halo (6 x 66 pixels, zero outside the image) is staged in LDS as float4.
constexpr int kInRows = 4, kInCols = 64;
constexpr int kInTileW = kInCols + 2, kInTileH = kInRows + 2;

__global__ void __launch_bounds__(256) conv_in_kernel(const float* __restrict__ x, ImgShape s,
                                                      const float* __restrict__ P, float* __restrict__ pre,
                                                      bf16_t* __restrict__ act) {
    __shared__ float wsh[9 * kNetCin * kNetC + kNetC];
    __shared__ float4 tin[kInTileH * kInTileW];
    for (int i = threadIdx.x; i < 9 * kNetCin * kNetC + kNetC; i += blockDim.x) wsh[i] = P[kOffW0 + i];
    const int tiles_w = (s.W + kInCols - 1) / kInCols, tiles_h = (s.H + kInRows - 1) / kInRows;
    long t = blockIdx.x;
    const int tw = (int)(t % tiles_w);
    t /= tiles_w;
    const int th = (int)(t % tiles_h);
    const int b = (int)(t / tiles_h);
    const int h0 = th * kInRows, w0 = tw * kInCols;
    for (int i = threadIdx.x; i < kInTileH * kInTileW; i += blockDim.x) {
        const int r = i / kInTileW, px = i % kInTileW;
        const int hh = h0 - 1 + r, ww = w0 - 1 + px;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (hh >= 0 && hh < s.H && ww >= 0 && ww < s.W) {
            const float* src = x + (((long)b * s.H + hh) * s.W + ww) * kNetCin;
            v = make_float4(src[0], src[1], src[2], 0.0f);
        }
        tin[i] = v;
    }
    __syncthreads();
    const int r = threadIdx.x / kInCols, cc = threadIdx.x % kInCols;
    const int h = h0 + r, w = w0 + cc;
    if (h >= s.H || w >= s.W) return;
    const long p = ((long)b * s.H + h) * s.W + w;
    float acc[kNetC];
#pragma unroll
    for (int c = 0; c < kNetC; ++c) acc[c] = wsh[9 * kNetCin * kNetC + c];
    for (int tap = 0; tap < 9; ++tap) {
        const float4 v4 = tin[(r + tap / 3) * kInTileW + cc + tap % 3];
        const float vin[kNetCin] = {v4.x, v4.y, v4.z};
#pragma unroll
        for (int ci = 0; ci < kNetCin; ++ci) {
            const float v = vin[ci];
            const float* wr = wsh + (tap * kNetCin + ci) * kNetC;
#pragma unroll
            for (int c = 0; c < kNetC; ++c) acc[c] += v * wr[c];
        }
    }
    // 16-byte stores: a pixel's 32 channels are 64 contiguous bytes of act (128 of pre)
    if (pre) {
        float4* pd = reinterpret_cast<float4*>(pre + p * kNetC);
#pragma unroll
        for (int q = 0; q < kNetC / 4; ++q) pd[q] = make_float4(acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]);
    }
    u32x4* ad = reinterpret_cast<u32x4*>(act + p * kNetC);
#pragma unroll
    for (int q = 0; q < kNetC / 8; ++q) {
        u32x4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            v[e] = (unsigned)f2bf(gelu(acc[8 * q + 2 * e])) | ((unsigned)f2bf(gelu(acc[8 * q + 2 * e + 1])) << 16);
        ad[q] = v;
    }
}

// ---- hidden layers: 32 -> 32 on MFMA --------------------------------------
// A workgroup of eight wavefronts computes a tile of eight image rows x 32 pixels: the
// input rows of the tile plus a one-pixel halo (10 x 34 pixels) and the 9 x 32 x 32
// weights are staged in LDS once, then each wavefront runs its row's 18 MFMAs from
// LDS.  Staged pixels and weight rows are padded to 80 bytes, so the 16-byte LDS
// reads of 16 consecutive lanes fall on distinct banks.
constexpr int kConvRows = 8;                 // output rows per workgroup (one per wavefront)
constexpr int kConvCols = 32;                // output pixels per row (the MFMA's 32)
constexpr int kStage = 40;                   // BF16 per staged pixel or weight row (32 + 8 padding)
constexpr int kTileW = kConvCols + 2, kTileH = kConvRows + 2;

__global__ void __launch_bounds__(64 * kConvRows) conv32_kernel(const bf16_t* __restrict__ in, ImgShape s,
                                                     const bf16_t* __restrict__ wt, const float* __restrict__ bias,
                                                     const float* __restrict__ pre_prev, float* __restrict__ pre,
                                                     bf16_t* __restrict__ act, int mode) {
    __shared__ __attribute__((aligned(16))) bf16_t tile[kTileH * kTileW * kStage];
    __shared__ __attribute__((aligned(16))) bf16_t wsh[9 * kNetC * kStage];
    const int tiles_w = (s.W + kConvCols - 1) / kConvCols, tiles_h = (s.H + kConvRows - 1) / kConvRows;
    long t = blockIdx.x;
    const int tw = (int)(t % tiles_w);
    t /= tiles_w;
    const int th = (int)(t % tiles_h);
    const int b = (int)(t / tiles_h);
    const int h0 = th * kConvRows, w0 = tw * kConvCols;
    // weights [tap][n][k]: 9 x 32 rows of 4 16-byte chunks
    for (int i = threadIdx.x; i < 9 * kNetC * 4; i += blockDim.x) {
        const int row = i >> 2, q = i & 3;
        *reinterpret_cast<u32x4*>(wsh + row * kStage + 8 * q) =
            *reinterpret_cast<const u32x4*>(wt + row * kNetC + 8 * q);
    }
    // input tile: rows h0-1 .. h0+4, pixels w0-1 .. w0+32, zero outside the image
    for (int i = threadIdx.x; i < kTileH * kTileW * 4; i += blockDim.x) {
        const int q = i & 3, px = (i >> 2) % kTileW, r = (i >> 2) / kTileW;
        const int hh = h0 - 1 + r, ww = w0 - 1 + px;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (hh >= 0 && hh < s.H && ww >= 0 && ww < s.W)
            v = *reinterpret_cast<const u32x4*>(in + (((long)b * s.H + hh) * s.W + ww) * kNetC + 8 * q);
        *reinterpret_cast<u32x4*>(tile + (r * kTileW + px) * kStage + 8 * q) = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int h = h0 + wv;
    if (h >= s.H) return;  // uniform per wavefront; no barrier follows
    const int m = lane & 31, kh = lane >> 5;
    f32x16 acc = {};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const bf16_t* src = tile + ((wv + tap / 3) * kTileW + m + tap % 3) * kStage + 8 * kh;
        const bf16_t* wsrc = wsh + (tap * kNetC + m) * kStage + 8 * kh;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const u32x4 av = *reinterpret_cast<const u32x4*>(src + 16 * c);
            const u32x4 bv = *reinterpret_cast<const u32x4*>(wsrc + 16 * c);
            // weights as A (rows: output channels), activations as B (columns: pixels)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, bv),
                                                          __builtin_bit_cast(bf16x8, av), acc, 0, 0, 0);
        }
    }
    // D[channel][pixel]: lane l holds pixel w0 + l % 32 and, in registers 4g..4g+3, the four
    // consecutive channels 8 g + 4 (l / 32) + 0..3: 8-byte BF16 and 16-byte FP32 stores
    const int w = w0 + m;
    if (w >= s.W) return;
    const long base = (((long)b * s.H + h) * s.W + w) * kNetC;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int c0 = 8 * g + 4 * kh;
        float v[4];
        if (mode == 0) {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = acc[4 * g + e] + (bias ? bias[c0 + e] : 0.0f);
            if (pre) *reinterpret_cast<float4*>(pre + base + c0) = make_float4(v[0], v[1], v[2], v[3]);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = gelu(v[e]);
        } else {
            const float4 pp = *reinterpret_cast<const float4*>(pre_prev + base + c0);
            v[0] = acc[4 * g + 0] * gelu_grad(pp.x);
            v[1] = acc[4 * g + 1] * gelu_grad(pp.y);
            v[2] = acc[4 * g + 2] * gelu_grad(pp.z);
            v[3] = acc[4 * g + 3] * gelu_grad(pp.w);
        }
        uint2 o;
        o.x = (unsigned)f2bf(v[0]) | ((unsigned)f2bf(v[1]) << 16);
        o.y = (unsigned)f2bf(v[2]) | ((unsigned)f2bf(v[3]) << 16);
        *reinterpret_cast<uint2*>(act + base + c0) = o;
    }
}

// ---- last layer: 32 -> 1 --------------------------------------------------
// A workgroup computes 4 rows x 64 pixels from an LDS tile of the input (6 x 66 pixels,
// zero outside the image, pixels padded to 80 bytes); each thread sums its pixel's
// 9 taps x 32 channels in FP32, in the same order as a direct loop.
constexpr int kOutRows = 4, kOutCols = 64;
constexpr int kOutTileW = kOutCols + 2, kOutTileH = kOutRows + 2;

__global__ void __launch_bounds__(256) conv_out_kernel(const bf16_t* __restrict__ a, ImgShape s,
                                                       const float* __restrict__ P, float* __restrict__ out) {
    __shared__ float wsh[9 * kNetC + 1];
    __shared__ __attribute__((aligned(16))) bf16_t tile[kOutTileH * kOutTileW * kStage];
    for (int i = threadIdx.x; i < 9 * kNetC + 1; i += blockDim.x) wsh[i] = P[kOffW3 + i];
    const int tiles_w = (s.W + kOutCols - 1) / kOutCols, tiles_h = (s.H + kOutRows - 1) / kOutRows;
    long t = blockIdx.x;
    const int tw = (int)(t % tiles_w);
    t /= tiles_w;
    const int th = (int)(t % tiles_h);
    const int b = (int)(t / tiles_h);
    const int h0 = th * kOutRows, w0 = tw * kOutCols;
    for (int i = threadIdx.x; i < kOutTileH * kOutTileW * 4; i += blockDim.x) {
        const int q = i & 3, px = (i >> 2) % kOutTileW, r = (i >> 2) / kOutTileW;
        const int hh = h0 - 1 + r, ww = w0 - 1 + px;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (hh >= 0 && hh < s.H && ww >= 0 && ww < s.W)
            v = *reinterpret_cast<const u32x4*>(a + (((long)b * s.H + hh) * s.W + ww) * kNetC + 8 * q);
        *reinterpret_cast<u32x4*>(tile + (r * kOutTileW + px) * kStage + 8 * q) = v;
    }
    __syncthreads();
    const int r = threadIdx.x / kOutCols, c = threadIdx.x % kOutCols;
    const int h = h0 + r, w = w0 + c;
    if (h >= s.H || w >= s.W) return;
    float acc = wsh[9 * kNetC];
    for (int tap = 0; tap < 9; ++tap) {
        const bf16_t* src = tile + ((r + tap / 3) * kOutTileW + c + tap % 3) * kStage;
        const float* wr = wsh + tap * kNetC;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const u32x4 v = *reinterpret_cast<const u32x4*>(src + 8 * q);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                acc += __uint_as_float(v[e] << 16) * wr[8 * q + 2 * e];
                acc += __uint_as_float(v[e] & 0xFFFF0000u) * wr[8 * q + 2 * e + 1];
            }
        }
    }
    out[((long)b * s.H + h) * s.W + w] = acc;
}

// ---- loss -----------------------------------------------------------------
__device__ inline double block_sum_d(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    __syncthreads();
    return s;
}

// num_den[2 b] += sum w (zn + o - t)^2, num_den[2 b + 1] += sum w t^2 over image b (grid.y = b)
__global__ void __launch_bounds__(256) loss_sums_kernel(const float* o, const float* zn, const float* t,
                                                        const float* w, int hw, double* num_den) {
    __shared__ double red[4];
    const int b = blockIdx.y;
    double sn = 0.0, sd = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < hw; i += gridDim.x * blockDim.x) {
        const long p = (long)b * hw + i;
        const double d = (double)zn[p] + o[p] - t[p];
        sn += (double)w[p] * d * d;
        sd += (double)w[p] * t[p] * t[p];
    }
    sn = block_sum_d(sn, red);
    sd = block_sum_d(sd, red);
    if (threadIdx.x == 0) {
        atomicAdd(&num_den[2 * b], sn);
        atomicAdd(&num_den[2 * b + 1], sd);
    }
}

__global__ void loss_grad_kernel(const float* o, const float* zn, const float* t, const float* w, int hw, int B,
                                 const double* num_den, float* g) {
    const long np = (long)B * hw;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (long)gridDim.x * blockDim.x) {
        const int b = (int)(p / hw);
        const double den = num_den[2 * b + 1];
        g[p] = den > 0.0 ? (float)(2.0 / B * w[p] * ((double)zn[p] + o[p] - t[p]) / den) : 0.0f;
    }
}

// ---- backward of the last layer ---------------------------------------------
__global__ void __launch_bounds__(256) conv_out_bwd_data_kernel(const float* __restrict__ g, const float* __restrict__ pre2,
                                                                ImgShape s, const float* __restrict__ P,
                                                                bf16_t* __restrict__ gact) {
    __shared__ float wsh[9 * kNetC];
    for (int i = threadIdx.x; i < 9 * kNetC; i += blockDim.x) wsh[i] = P[kOffW3 + i];
    __syncthreads();
    const long np = (long)s.B * s.H * s.W;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    int b, h, w;
    pix_of(p, s, b, h, w);
    float acc[kNetC];
#pragma unroll
    for (int c = 0; c < kNetC; ++c) acc[c] = 0.0f;
    for (int tap = 0; tap < 9; ++tap) {
        // out[q] uses a[q + off]; a[p] feeds out[p - off]
        const int hh = h - (tap / 3 - 1), ww = w - (tap % 3 - 1);
        if (hh < 0 || hh >= s.H || ww < 0 || ww >= s.W) continue;
        const float gv = g[((long)b * s.H + hh) * s.W + ww];
#pragma unroll
        for (int c = 0; c < kNetC; ++c) acc[c] += gv * wsh[tap * kNetC + c];
    }
#pragma unroll
    for (int c = 0; c < kNetC; ++c) gact[p * kNetC + c] = f2bf(acc[c] * gelu_grad(pre2[p * kNetC + c]));
}

// grads[W3[tap][ci]] += sum_p a[p + off][ci] g[p]; grads[b3] += sum_p g[p]  (tiles of 256 pixels)
__global__ void __launch_bounds__(320) conv_out_bwd_w_kernel(const bf16_t* __restrict__ a, const float* __restrict__ g,
                                                             ImgShape s, float* __restrict__ grads) {
    __shared__ float gs[256];
    const long np = (long)s.B * s.H * s.W;
    const long p0 = (long)blockIdx.x * 256;
    for (int i = threadIdx.x; i < 256; i += blockDim.x) gs[i] = p0 + i < np ? g[p0 + i] : 0.0f;
    __syncthreads();
    const int t = threadIdx.x;
    if (t < 9 * kNetC) {
        const int tap = t / kNetC, ci = t % kNetC;
        float acc = 0.0f;
        for (int i = 0; i < 256 && p0 + i < np; ++i) {
            int b, h, w;
            pix_of(p0 + i, s, b, h, w);
            const int hh = h + tap / 3 - 1, ww = w + tap % 3 - 1;
            if (hh < 0 || hh >= s.H || ww < 0 || ww >= s.W) continue;
            acc += bf2f(a[(((long)b * s.H + hh) * s.W + ww) * kNetC + ci]) * gs[i];
        }
        atomicAdd(&grads[kOffW3 + t], acc);
    } else if (t == 9 * kNetC) {
        float acc = 0.0f;
        for (int i = 0; i < 256; ++i) acc += gs[i];
        atomicAdd(&grads[kOffB3], acc);
    }
}

// ---- weight gradient of the hidden layers on MFMA ----------------------------
// wave -> (tap, part); part covers kChunks chunks of 16 pixels of one image row (W % 16 == 0)
constexpr int kWgChunks = 64;
__global__ void __launch_bounds__(256) conv32_wgrad_kernel(const bf16_t* __restrict__ a, const bf16_t* __restrict__ g,
                                                           ImgShape s, float* __restrict__ dW, long nparts) {
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wave >= 9 * nparts) return;
    const int tap = (int)(wave % 9);
    const long part = wave / 9;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int segs = s.W / 16;
    const long nchunks = (long)s.B * s.H * segs;
    const int mn = lane & 31, kh = lane >> 5;
    f32x16 acc = {};
    for (long ch = part * kWgChunks; ch < (part + 1) * kWgChunks && ch < nchunks; ++ch) {
        const int seg = (int)(ch % segs);
        const long bh = ch / segs;
        const int h = (int)(bh % s.H), b = (int)(bh / s.H);
        const int hh = h + dy;
        const bool rowok = hh >= 0 && hh < s.H;
        bf16x8 av, bv;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int w = seg * 16 + 8 * kh + j;
            const int ww = w + dx;
            const bool ok = rowok && ww >= 0 && ww < s.W;
            // A[m = ci][k = pixel]: shifted activation; B[k = pixel][n = co]: output gradient
            const bf16_t ua = ok ? a[(((long)b * s.H + hh) * s.W + ww) * kNetC + mn] : (bf16_t)0;
            const bf16_t ub = g[(((long)b * s.H + h) * s.W + w) * kNetC + mn];
            av[j] = __builtin_bit_cast(__bf16, ua);
            bv[j] = __builtin_bit_cast(__bf16, ub);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int ci = 8 * (i / 4) + 4 * kh + (i % 4);
        atomicAdd(&dW[(tap * kNetC + ci) * kNetC + mn], acc[i]);
    }
}

// first-layer weight gradient: dW0[tap][ci][co] += sum_p x[p + off][ci] g[p][co], tiles of 512 pixels
__global__ void __launch_bounds__(256) conv_in_wgrad_kernel(const float* __restrict__ x, const bf16_t* __restrict__ g,
                                                            ImgShape s, float* __restrict__ dW0) {
    const long np = (long)s.B * s.H * s.W;
    const long p0 = (long)blockIdx.x * 512;
    for (int o = threadIdx.x; o < 9 * kNetCin * kNetC; o += blockDim.x) {
        const int co = o % kNetC, ci = (o / kNetC) % kNetCin, tap = o / (kNetC * kNetCin);
        float acc = 0.0f;
        for (int i = 0; i < 512 && p0 + i < np; ++i) {
            int b, h, w;
            pix_of(p0 + i, s, b, h, w);
            const int hh = h + tap / 3 - 1, ww = w + tap % 3 - 1;
            if (hh < 0 || hh >= s.H || ww < 0 || ww >= s.W) continue;
            acc += x[(((long)b * s.H + hh) * s.W + ww) * kNetCin + ci] * bf2f(g[(p0 + i) * kNetC + co]);
        }
        atomicAdd(&dW0[o], acc);
    }
}

// db[c] += sum_p g[p][c]; 256 threads = 8 pixel lanes x 32 channels, tiles of 2048 pixels
__global__ void __launch_bounds__(256) bias_grad_kernel(const bf16_t* __restrict__ g, long np, float* __restrict__ db) {
    __shared__ float red[256];
    const int c = threadIdx.x % kNetC, r = threadIdx.x / kNetC;
    const long p0 = (long)blockIdx.x * 2048;
    float acc = 0.0f;
    for (long p = p0 + r; p < p0 + 2048 && p < np; p += 8) acc += bf2f(g[p * kNetC + c]);
    red[threadIdx.x] = acc;
    __syncthreads();
    if (r == 0) {
        float s = 0.0f;
        for (int k = 0; k < 8; ++k) s += red[k * kNetC + c];
        atomicAdd(&db[c], s);
    }
}

// ---- optimiser ---------------------------------------------------------------
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void pack_weights_kernel(const float* P, bf16_t* wf1, bf16_t* wb1, bf16_t* wf2, bf16_t* wb2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // over 9 * 32 * 32
    if (i >= 9 * kNetC * kNetC) return;
    const int tap = i / (kNetC * kNetC), r = i % (kNetC * kNetC);
    const int n = r / kNetC, k = r % kNetC;
    // forward [tap][n = co][k = ci] = W[tap][ci][co]; data gradient [tap][n = ci][k = co] = W[8 - tap][ci][co]
    wf1[i] = f2bf(P[kOffW1 + (tap * kNetC + k) * kNetC + n]);
    wf2[i] = f2bf(P[kOffW2 + (tap * kNetC + k) * kNetC + n]);
    wb1[i] = f2bf(P[kOffW1 + ((8 - tap) * kNetC + n) * kNetC + k]);
    wb2[i] = f2bf(P[kOffW2 + ((8 - tap) * kNetC + n) * kNetC + k]);
}

__global__ void zero_f32_kernel(float* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// ---- coefficient <-> image ----------------------------------------------------
// The scale of z: isz, or (zz != NULL) 1 / sqrt(zz[0] inv_n) with zz[0] the device sum of
// squares of z (0 for a zero z).
__device__ inline double inv_rms(double isz, const double* zz, double inv_n) {
    if (!zz) return isz;
    const double ms = zz[0] * inv_n;
    return ms > 0.0 ? 1.0 / sqrt(ms) : 0.0;
}

__global__ void pack_image_kernel(SlotMap mp, const double* z, long ld, double isz_h, const double* zz, double inv_n,
                                  float* x) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= mp.W) return;
    const double isz = inv_rms(isz_h, zz, inv_n);
    const int gi = mp.sx[i], gj = mp.sy[j];
    const bool ok = gi >= 0 && gj >= 0;
    const long p = (long)i * mp.W + j;
    x[3 * p + 0] = ok ? (float)(z[(long)gi * ld + gj] * isz) : 0.0f;
    x[3 * p + 1] = ok ? (float)(z[(long)gi * ld + gj] * isz * exp(-(double)mp.loga[p])) : 0.0f;
    x[3 * p + 2] = mp.loga[p];
}

__global__ void unpack_add_kernel(SlotMap mp, const float* o, double sz_h, const double* zz, double inv_n, double* z,
                                  long ld) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= mp.W) return;
    // scale sz_h, or (zz != NULL) sz_h times the root-mean-square value of z
    const double sz = zz ? sz_h * sqrt(fmax(zz[0] * inv_n, 0.0)) : sz_h;
    const int gi = mp.sx[i], gj = mp.sy[j];
    if (gi < 0 || gj < 0) return;
    z[(long)gi * ld + gj] += sz * (double)o[(long)i * mp.W + j];
}

__global__ void target_image_kernel(SlotMap mp, const double* xs, const double* x, const double* z, long ld,
                                    double isz, const float* wx, const float* wy, float* zn, float* t, float* w) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= mp.W) return;
    const int gi = mp.sx[i], gj = mp.sy[j];
    const bool ok = gi >= 0 && gj >= 0;
    const long p = (long)i * mp.W + j;
    const long q = (long)gi * ld + gj;
    zn[p] = ok ? (float)(z[q] * isz) : 0.0f;
    t[p] = ok ? (float)((xs[q] - x[q]) * isz) : 0.0f;
    // diagonal of the energy form a (K (x) M + M (x) K) at the slot
    w[p] = ok ? expf(mp.loga[p]) * (wx[mp.H + i] * wy[j] + wx[i] * wy[mp.W + j]) : 0.0f;
}

__global__ void crop_kernel(const float* x, const float* zn, const float* t, const float* w, int H, int W, int c,
                            const int* pos, float* cx, float* czn, float* ct, float* cw) {
    const int n = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= c * c) return;
    const int yy = pos[2 * n] + k / c, xx = pos[2 * n + 1] + k % c;
    const long src = (long)yy * W + xx;
    const long dst = (long)n * c * c + k;
    for (int ch = 0; ch < 3; ++ch) cx[3 * dst + ch] = x[3 * src + ch];
    czn[dst] = zn[src];
    ct[dst] = t[src];
    cw[dst] = w[src];
}

__global__ void gather_batch_kernel(const float* X, const float* ZN, const float* T, const float* Wt, int cc,
                                    const int* idx, float* x, float* zn, float* t, float* w) {
    const int b = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cc) return;
    const long src = (long)idx[b] * cc + k, dst = (long)b * cc + k;
    for (int ch = 0; ch < 3; ++ch) x[3 * dst + ch] = X[3 * src + ch];
    zn[dst] = ZN[src];
    t[dst] = T[src];
    w[dst] = Wt[src];
}

inline unsigned blocks_for(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_conv_in(const float* x, ImgShape s, const float* params, float* pre, bf16_t* act, hipStream_t st) {
    const long tiles = (long)s.B * ((s.H + kInRows - 1) / kInRows) * ((s.W + kInCols - 1) / kInCols);
    hipLaunchKernelGGL(conv_in_kernel, dim3((unsigned)tiles), dim3(256), 0, st, x, s, params, pre, act);
    return hipGetLastError();
}

hipError_t launch_conv32(const bf16_t* in, ImgShape s, const bf16_t* wt, const float* bias, const float* pre_prev,
                         float* pre, bf16_t* act, int mode, hipStream_t st) {
    const long tiles = (long)s.B * ((s.H + kConvRows - 1) / kConvRows) * ((s.W + kConvCols - 1) / kConvCols);
    hipLaunchKernelGGL(conv32_kernel, dim3((unsigned)tiles), dim3(64 * kConvRows), 0, st, in, s, wt, bias, pre_prev,
                       pre, act, mode);
    return hipGetLastError();
}

hipError_t launch_conv_out(const bf16_t* a, ImgShape s, const float* params, float* out, hipStream_t st) {
    const long tiles = (long)s.B * ((s.H + kOutRows - 1) / kOutRows) * ((s.W + kOutCols - 1) / kOutCols);
    hipLaunchKernelGGL(conv_out_kernel, dim3((unsigned)tiles), dim3(256), 0, st, a, s, params, out);
    return hipGetLastError();
}

hipError_t launch_loss(const float* o, const float* zn, const float* t, const float* w, ImgShape s, float* g,
                       double* num_den, hipStream_t st) {
    const int hw = s.H * s.W;
    hipLaunchKernelGGL(loss_sums_kernel, dim3(std::min<unsigned>(blocks_for(hw, 256), 64), s.B), dim3(256), 0, st,
                       o, zn, t, w, hw, num_den);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !g) return e;
    const long np = (long)s.B * hw;
    hipLaunchKernelGGL(loss_grad_kernel, dim3(std::min<unsigned>(blocks_for(np, 256), 4096)), dim3(256), 0, st, o,
                       zn, t, w, hw, s.B, num_den, g);
    return hipGetLastError();
}

hipError_t launch_conv_out_backward(const bf16_t* a, const float* g, const float* pre2, ImgShape s,
                                    const float* params, float* grads, bf16_t* gact, hipStream_t st) {
    const long np = (long)s.B * s.H * s.W;
    hipLaunchKernelGGL(conv_out_bwd_data_kernel, dim3(blocks_for(np, 256)), dim3(256), 0, st, g, pre2, s, params,
                       gact);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(conv_out_bwd_w_kernel, dim3(blocks_for(np, 256)), dim3(320), 0, st, a, g, s, grads);
    return hipGetLastError();
}

hipError_t launch_conv32_wgrad(const bf16_t* a, const bf16_t* g, ImgShape s, float* dW, hipStream_t st) {
    if (s.W % 16 != 0) return hipErrorInvalidValue;
    const long nchunks = (long)s.B * s.H * (s.W / 16);
    const long nparts = (nchunks + kWgChunks - 1) / kWgChunks;
    hipLaunchKernelGGL(conv32_wgrad_kernel, dim3(blocks_for(9 * nparts, 4)), dim3(256), 0, st, a, g, s, dW, nparts);
    return hipGetLastError();
}

hipError_t launch_conv_in_wgrad(const float* x, const bf16_t* g, ImgShape s, float* dW0, hipStream_t st) {
    const long np = (long)s.B * s.H * s.W;
    hipLaunchKernelGGL(conv_in_wgrad_kernel, dim3(blocks_for(np, 512)), dim3(256), 0, st, x, g, s, dW0);
    return hipGetLastError();
}

hipError_t launch_bias_grad(const bf16_t* g, ImgShape s, float* db, hipStream_t st) {
    const long np = (long)s.B * s.H * s.W;
    hipLaunchKernelGGL(bias_grad_kernel, dim3(blocks_for(np, 2048)), dim3(256), 0, st, g, np, db);
    return hipGetLastError();
}

hipError_t launch_adam(float* params, const float* grads, float* m, float* v, int n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t st) {
    const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, params, grads, m, v, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_pack_weights(const float* params, bf16_t* wf1, bf16_t* wb1, bf16_t* wf2, bf16_t* wb2,
                               hipStream_t st) {
    hipLaunchKernelGGL(pack_weights_kernel, dim3(blocks_for(9 * kNetC * kNetC, 256)), dim3(256), 0, st, params, wf1,
                       wb1, wf2, wb2);
    return hipGetLastError();
}

hipError_t launch_zero_f32(float* p, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(zero_f32_kernel, dim3(std::min<unsigned>(blocks_for((long)n, 256), 4096)), dim3(256), 0, st,
                       p, n);
    return hipGetLastError();
}

hipError_t launch_pack_image(const SlotMap& m, const double* z, long ld, double inv_sz, float* x, hipStream_t st,
                             const double* zz, double inv_n) {
    hipLaunchKernelGGL(pack_image_kernel, dim3(blocks_for(m.W, 256), m.H), dim3(256), 0, st, m, z, ld, inv_sz, zz,
                       inv_n, x);
    return hipGetLastError();
}

hipError_t launch_unpack_add(const SlotMap& m, const float* o, double sz, double* z, long ld, hipStream_t st,
                             const double* zz, double inv_n) {
    hipLaunchKernelGGL(unpack_add_kernel, dim3(blocks_for(m.W, 256), m.H), dim3(256), 0, st, m, o, sz, zz, inv_n, z,
                       ld);
    return hipGetLastError();
}

hipError_t launch_target_image(const SlotMap& m, const double* xs, const double* x, const double* z, long ld,
                               double inv_sz, const float* wx, const float* wy, float* zn, float* t, float* w,
                               hipStream_t st) {
    hipLaunchKernelGGL(target_image_kernel, dim3(blocks_for(m.W, 256), m.H), dim3(256), 0, st, m, xs, x, z, ld,
                       inv_sz, wx, wy, zn, t, w);
    return hipGetLastError();
}

hipError_t launch_crop(const float* x, const float* zn, const float* t, const float* w, int H, int W, int c,
                       const int* pos, int n, float* cx, float* czn, float* ct, float* cw, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(crop_kernel, dim3(blocks_for((long)c * c, 256), n), dim3(256), 0, st, x, zn, t, w, H, W, c,
                       pos, cx, czn, ct, cw);
    return hipGetLastError();
}

hipError_t launch_gather_batch(const float* X, const float* ZN, const float* T, const float* Wt, int c,
                               const int* idx, int B, float* x, float* zn, float* t, float* w, hipStream_t st) {
    hipLaunchKernelGGL(gather_batch_kernel, dim3(blocks_for((long)c * c, 256), B), dim3(256), 0, st, X, ZN, T, Wt,
                       c * c, idx, x, zn, t, w);
    return hipGetLastError();
}

}  // namespace hpadi
