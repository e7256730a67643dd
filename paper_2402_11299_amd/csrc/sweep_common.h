// Device helpers shared by the half-sweep kernels (sweep.hip, sweep_uni.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace hpadi {
namespace sweep_detail {

__device__ __forceinline__ bool vhat(int bc, int n, int v) { return bc == 0 ? (v >= 1 && v <= n - 1) : (v >= 0 && v <= n); }
__device__ __forceinline__ int hov(int bc, int v) { return bc == 0 ? v - 1 : v; }
__device__ __forceinline__ int voh(int bc, int h) { return bc == 0 ? h + 1 : h; }

__device__ __forceinline__ long addr(const Layout& L, int i, int j) {
    const int ii = i >= L.nhr ? i + L.offr : i;
    const int jj = j >= L.nhc ? j + L.offc : j;
    if (L.panel == 8) return (long)(jj >> 3) * L.ld + (long)ii * 8 + (jj & 7);
    if (L.panel == 4) return (long)(jj >> 2) * L.ld + (long)ii * 4 + (jj & 3);
    return (long)ii * L.ld + jj;
}

constexpr int sweep_max_threads(int cl) { return cl <= 32 ? 1024 : 512; }

// Staged hat data of one factor: 1/diag, diag, sub-diagonal of L0, coupling C.
struct HatF {
    double* invd0;
    double* d0;
    double* link0;  // link0[h] = L0[h][h-1]; link0[nh] = 0 (sentinel)
    double* cpl;    // 4n
};

// Suffix scan over lanes of affine maps z = a + b z_next (lane k composes with
// lane k+1, k+2, ...): afterwards a = value of the recurrence run from the last
// lane down to k with terminal value 0.
__device__ __forceinline__ void suffix_scan(double& a, double& b, int lane, int nl) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double a2 = __shfl_down(a, d, 64);
        const double b2 = __shfl_down(b, d, 64);
        if (lane + d < nl) {
            a = a + b * a2;
            b = b * b2;
        }
    }
}
// Prefix scan: x = a + b x_prev, composed with lanes k-1, k-2, ...
__device__ __forceinline__ void prefix_scan(double& a, double& b, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double a2 = __shfl_up(a, d, 64);
        const double b2 = __shfl_up(b, d, 64);
        if (lane >= d) {
            a = a + b * a2;
            b = b * b2;
        }
    }
}

// Hat-block backward solve L0^T z = r for one line, by one full wavefront.
// r: LDS hat array (nh <= 65), overwritten with z.  Lane k owns hat k; lane 63
// also owns hat 64 when nh = 65.
__device__ __forceinline__ void hat_backward(double* r, const HatF& F, int nh, int lane) {
    const int nl = nh < 64 ? nh : 64;
    double a = 0.0, b = 1.0;
    double a64 = 0.0;
    if (lane < nl) {
        a = r[lane] * F.invd0[lane];
        b = -F.link0[lane + 1] * F.invd0[lane];
        if (lane == 63 && nh == 65) {
            a64 = r[64] * F.invd0[64];
            a = a + b * a64;  // compose with hat 64 (whose own map is constant)
            b = 0.0;
        }
    }
    suffix_scan(a, b, lane, nl);
    if (lane < nl) r[lane] = a;
    if (lane == 63 && nh == 65) r[64] = a64;
}

// Hat-block forward solve L0 x = z for one line (in place on r).
__device__ __forceinline__ void hat_forward(double* r, const HatF& F, int nh, int lane) {
    const int nl = nh < 64 ? nh : 64;
    double a = 0.0, b = 0.0;
    if (lane < nl) {
        a = r[lane] * F.invd0[lane];
        b = -F.link0[lane] * F.invd0[lane];
    }
    prefix_scan(a, b, lane);
    if (lane < nl) r[lane] = a;
    if (nh == 65) {
        const double x63 = __shfl(a, 63, 64);
        if (lane == 0) r[64] = (r[64] - F.link0[64] * x63) * F.invd0[64];
    }
}

// Coupling of the chain heads of the two elements adjacent to hat h:
// sum_{(e,pi) adjacent} C[(pi,e)][h] * heads[pi n + e].
__device__ __forceinline__ double head_coupling(const double* C, const double* heads, int bc, int n, int h) {
    const int v = voh(bc, h);
    double acc = 0.0;
    if (v >= 1) {
        const int q = v - 1;
        acc += C[4 * q + 1] * heads[q] + C[4 * q + 3] * heads[n + q];
    }
    if (v <= n - 1) {
        const int q = v;
        acc += C[4 * q + 0] * heads[q] + C[4 * q + 2] * heads[n + q];
    }
    return acc;
}


// Adds the sum of v over the workgroup to *acc (one atomic per workgroup).  Every thread
// of the workgroup calls it; red is LDS of at least blockDim.x / 64 doubles, free once
// every thread has reached the call.
__device__ __forceinline__ void block_sum_atomic(double v, double* red, double* acc) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        atomicAdd(acc, t);
    }
}

size_t sweep_lds_bytes(const DimDev& d, int threads, int mode);

}  // namespace sweep_detail
}  // namespace hpadi
