// Device helpers shared by the half-sweep kernels (sweep.hip, sweep_uni.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace hpadi {
namespace sweep_detail {

// bc is the hat mask of DimDev: bit 0 vertex 0 carries a hat, bit 1 vertex n.
__device__ __forceinline__ bool vhat(int bc, int n, int v) { return v >= ((bc & 1) ? 0 : 1) && v <= ((bc & 2) ? n : n - 1); }
__device__ __forceinline__ int hov(int bc, int v) { return v - ((bc & 1) ? 0 : 1); }
__device__ __forceinline__ int voh(int bc, int h) { return h + ((bc & 1) ? 0 : 1); }
// Robin coefficient of the end at vertex v (0 elsewhere), on the stiffness diagonal of its hat
__device__ __forceinline__ double robin_at(const DimDev& d, int v) {
    return (v == 0 ? d.rob0 : 0.0) + (v == d.n ? d.rob1 : 0.0);
}

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

// One step of an inclusive scan of affine maps over the 64 lanes: (a, b) of this lane is
// composed with the (a', b') that the DPP control CTRL moves in (identity (0, 1) where the
// move has no source or the row is masked off): a <- a + b a', b <- b b'.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v, double identity) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(identity), __double2loint(v), CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(identity), __double2hiint(v), CTRL, ROWMASK, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ void compose_from(double& a, double& b) {
    const double a2 = dpp_move<CTRL, ROWMASK>(a, 0.0);
    const double b2 = dpp_move<CTRL, ROWMASK>(b, 1.0);
    a = a + b * a2;
    b = b * b2;
}
// Inclusive prefix composition over the wavefront: lane k ends with f_k o f_{k-1} o ... o f_0,
// f_j(z) = a_j + b_j z.  Row shifts by 1, 2, 4, 8 within each 16-lane row, then the last
// lane of row 0 (2) into row 1 (3), then lane 31 into rows 2 and 3 (DPP row broadcasts):
// register moves only, no LDS round trips.  Every lane of the wavefront must be active.
__device__ __forceinline__ void prefix_compose(double& a, double& b) {
    compose_from<0x111, 0xF>(a, b);  // row_shr:1
    compose_from<0x112, 0xF>(a, b);  // row_shr:2
    compose_from<0x114, 0xF>(a, b);  // row_shr:4
    compose_from<0x118, 0xF>(a, b);  // row_shr:8
    compose_from<0x142, 0xA>(a, b);  // row_bcast:15 into rows 1 and 3
    compose_from<0x143, 0xC>(a, b);  // row_bcast:31 into rows 2 and 3
}

// Hat-block backward solve L0^T z = r for one line, by one full wavefront.
// r: LDS hat array (nh <= 65), overwritten with z.  z_h = (r_h - L0[h+1][h] z_{h+1}) /
// L0[h][h] runs from the last hat down, so lane k takes hat nl - 1 - k and the suffix
// becomes a prefix over lanes; hat 64 (nh = 65) is folded into hat 63's map.
__device__ __forceinline__ void hat_backward(double* r, const HatF& F, int nh, int lane) {
    const int nl = nh < 64 ? nh : 64;
    const int h = nl - 1 - lane;
    double a = 0.0, b = 1.0;
    double a64 = 0.0;
    if (h >= 0) {
        a = r[h] * F.invd0[h];
        b = -F.link0[h + 1] * F.invd0[h];
        if (h == 63 && nh == 65) {
            a64 = r[64] * F.invd0[64];
            a = a + b * a64;  // compose with hat 64 (whose own map is constant)
            b = 0.0;
        }
    }
    prefix_compose(a, b);
    if (h >= 0) r[h] = a;
    if (h == 63 && nh == 65) r[64] = a64;
}

// Hat-block forward solve L0 x = z for one line (in place on r): lane k takes hat k.
__device__ __forceinline__ void hat_forward(double* r, const HatF& F, int nh, int lane) {
    const int nl = nh < 64 ? nh : 64;
    double a = 0.0, b = 0.0;
    if (lane < nl) {
        a = r[lane] * F.invd0[lane];
        b = -F.link0[lane] * F.invd0[lane];
    }
    prefix_compose(a, b);
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
