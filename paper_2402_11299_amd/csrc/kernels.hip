// HIP kernels of hpadi for gfx950 (MI355X).
//
// Everything here is bandwidth-bound banded work: no matrix cores.
//  * factor_kernel   reverse Cholesky of kappa K + sigma M (Sec. 4, Alg. 1), one
//                    workgroup per matrix, one thread per (element, parity) chain,
//                    the hat Schur complement in FP64 by one thread.
//  * the ADI half-sweeps themselves are in sweep.hip.
//  * op_apply, residual, load: elementwise gathers of the banded operators.
//
// Coefficient order (per dimension, Sec. 2.2): hats 0..nh-1, then bubble (m, e)
// at nh + m n + e.  Element e has left vertex e and right vertex e+1; vertex v
// is hat v-1 (Dirichlet, v = 1..n-1) or hat v (Neumann, v = 0..n).

#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace hpadi {

namespace {

// bc is the hat mask: bit 0 set when vertex 0 carries a hat, bit 1 when vertex n does.
__device__ __forceinline__ bool vertex_is_hat(int bc, int n, int v) {
    return v >= ((bc & 1) ? 0 : 1) && v <= ((bc & 2) ? n : n - 1);
}
__device__ __forceinline__ int hat_of_vertex(int bc, int v) { return v - ((bc & 1) ? 0 : 1); }
__device__ __forceinline__ int vertex_of_hat(int bc, int h) { return h + ((bc & 1) ? 0 : 1); }
// Robin coefficient of the end at vertex v (0 elsewhere): Sec. 3.3's boundary term on K
__device__ __forceinline__ double robin_at(const DimDev& d, int v) {
    return (v == 0 ? d.rob0 : 0.0) + (v == d.n ? d.rob1 : 0.0);
}

// ---------------------------------------------------------------------------
// Factorisation (Alg. 1) of S = kappa K + sigma M, FP64.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) factor_kernel(DimDev d, const double* __restrict__ kappa,
                                                     const double* __restrict__ sigma, double* fac64,
                                                     float* fac32, FactorLayout fl, int* status) {
    const int f = blockIdx.x;
    const double kap = kappa[f], sig = sigma[f];
    double* F = fac64 + (size_t)f * fl.stride;
    const int n = d.n, p = d.p, nh = d.nh;
    const double* kd = d.tab64;
    const double* md = d.tab64 + d.tabstride;
    const double* mo = d.tab64 + 2 * d.tabstride;
    int bad = 0;
    // Step 1: reverse Cholesky of each element's bubble block.  Degrees m and m+-2
    // couple, odd offsets vanish, so each block splits into an even and an odd
    // tridiagonal chain, factorised from the highest degree down.
    for (int t = threadIdx.x; t < 2 * n; t += blockDim.x) {
        const int e = t >> 1, pi = t & 1;
        const int len = pi ? (p - 1) / 2 : p / 2;
        const double de = d.delta[e], ide = d.invdelta[e];
        double dup = 0.0, dhead = 1.0;
        for (int s = len - 1; s >= 0; --s) {
            const int m = pi + 2 * s;
            double a = kap * kd[m] * ide + sig * md[m] * de;
            if (s + 1 < len) {
                const double l = sig * mo[m] * de / dup;  // S[(m),(m+2)] / d_{m+2}
                F[fl.off_link + (m + 2) * n + e] = l;
                a -= l * l;
            }
            if (!(a > 0.0)) {
                bad = 1;
                a = 1.0;
            }
            const double dd = sqrt(a);
            F[fl.off_invd + m * n + e] = 1.0 / dd;
            F[fl.off_d + m * n + e] = dd;
            dup = dd;
            if (s == 0) dhead = dd;
        }
        if (pi < p - 1) F[fl.off_link + pi * n + e] = 0.0;
        // Step 2: coupling of the chain head (degree pi) to the hats of element e:
        // L[(pi,e), hat] = S[hat, (pi,e)] / d_(pi,e).  Only W_0 and W_1 touch hats.
        double sl, sr;
        if (pi == 0) {
            sl = sr = sig * de / 6.0;
        } else {
            sl = -sig * de / 30.0;
            sr = sig * de / 30.0;
        }
        const bool has = len > 0;
        F[fl.off_cpl + 4 * e + 2 * pi + 0] = (has && vertex_is_hat(d.bc, n, e)) ? sl / dhead : 0.0;
        F[fl.off_cpl + 4 * e + 2 * pi + 1] = (has && vertex_is_hat(d.bc, n, e + 1)) ? sr / dhead : 0.0;
    }
    __syncthreads();
    // Steps 3-4: hat Schur complement A0 - C^T C (tridiagonal) and its reverse
    // Cholesky, sequential over the hats, FP64.
    if (threadIdx.x == 0) {
        const double* C = F + fl.off_cpl;
        double dup = 0.0;
        for (int h = nh - 1; h >= 0; --h) {
            const int v = vertex_of_hat(d.bc, h);
            double a = kap * robin_at(d, v);
            if (v >= 1) {  // element v-1 lies left of v: v is its right vertex
                const int e = v - 1;
                a += kap * d.invdelta[e] + sig * d.delta[e] / 3.0;
                a -= C[4 * e + 1] * C[4 * e + 1] + C[4 * e + 3] * C[4 * e + 3];
            }
            if (v <= n - 1) {  // element v lies right of v: v is its left vertex
                const int e = v;
                a += kap * d.invdelta[e] + sig * d.delta[e] / 3.0;
                a -= C[4 * e + 0] * C[4 * e + 0] + C[4 * e + 2] * C[4 * e + 2];
            }
            if (h + 1 < nh) {
                const int e = v;  // element between vertices v and v+1
                double b = -kap * d.invdelta[e] + sig * d.delta[e] / 6.0;
                b -= C[4 * e + 0] * C[4 * e + 1] + C[4 * e + 2] * C[4 * e + 3];
                const double l = b / dup;
                F[fl.off_link0 + h + 1] = l;
                a -= l * l;
            }
            if (!(a > 0.0)) {
                bad = 1;
                a = 1.0;
            }
            const double dd = sqrt(a);
            F[fl.off_invd0 + h] = 1.0 / dd;
            F[fl.off_d0 + h] = dd;
            dup = dd;
        }
        if (nh > 0) F[fl.off_link0] = 0.0;
    }
    if (bad) atomicOr(status + f, 1);
    __syncthreads();
    if (fac32) {
        float* F32 = fac32 + (size_t)f * fl.stride;
        for (int i = threadIdx.x; i < fl.size; i += blockDim.x) F32[i] = (float)F[i];
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Elementwise banded operators.
// ---------------------------------------------------------------------------

// K x and M x at position pos of a line x (stride sp), App. A entries (the 1/3, 1/6, 1/30
// factors are multiplications by rounded reciprocals: a divide is a long FP64 sequence).
__device__ __forceinline__ void gather_km(const DimDev& d, const double* x, long sp, int pos, double& Kx,
                                          double& Mx) {
    const int n = d.n, nh = d.nh, p = d.p;
    Kx = 0.0;
    Mx = 0.0;
    if (pos < nh) {
        const int h = pos, v = vertex_of_hat(d.bc, h);
        const double xh = x[(long)h * sp];
        Kx += robin_at(d, v) * xh;
        if (v >= 1) {
            const int q = v - 1;
            const double dq = d.delta[q], idq = d.invdelta[q];
            Kx += idq * xh;
            Mx += dq * (1.0 / 3.0) * xh;
            if (vertex_is_hat(d.bc, n, v - 1)) {
                const double xn = x[(long)(h - 1) * sp];
                Kx -= idq * xn;
                Mx += dq * (1.0 / 6.0) * xn;
            }
            if (p >= 2) Mx += dq * (1.0 / 6.0) * x[(long)(nh + q) * sp];
            if (p >= 3) Mx += dq * (1.0 / 30.0) * x[(long)(nh + n + q) * sp];
        }
        if (v <= n - 1) {
            const int q = v;
            const double dq = d.delta[q], idq = d.invdelta[q];
            Kx += idq * xh;
            Mx += dq * (1.0 / 3.0) * xh;
            if (vertex_is_hat(d.bc, n, v + 1)) {
                const double xn = x[(long)(h + 1) * sp];
                Kx -= idq * xn;
                Mx += dq * (1.0 / 6.0) * xn;
            }
            if (p >= 2) Mx += dq * (1.0 / 6.0) * x[(long)(nh + q) * sp];
            if (p >= 3) Mx -= dq * (1.0 / 30.0) * x[(long)(nh + n + q) * sp];
        }
    } else {
        const int b = pos - nh, m = b / n, e = b - m * n;
        const double de = d.delta[e], ide = d.invdelta[e];
        const double* kd = d.tab64;
        const double* md = d.tab64 + d.tabstride;
        const double* mo = d.tab64 + 2 * d.tabstride;
        const double xm = x[(long)pos * sp];
        Kx = kd[m] * ide * xm;
        Mx = md[m] * de * xm;
        if (m >= 2) Mx += mo[m - 2] * de * x[(long)(pos - 2 * n) * sp];
        if (m + 2 <= p - 2) Mx += mo[m] * de * x[(long)(pos + 2 * n) * sp];
        if (m <= 1) {
            double xl = 0.0, xr = 0.0;
            if (vertex_is_hat(d.bc, n, e)) xl = x[(long)hat_of_vertex(d.bc, e) * sp];
            if (vertex_is_hat(d.bc, n, e + 1)) xr = x[(long)hat_of_vertex(d.bc, e + 1) * sp];
            Mx += (m == 0) ? de * (1.0 / 6.0) * (xl + xr) : de * (1.0 / 30.0) * (xr - xl);
        }
    }
}

// The stencil of K and M at one position of a line as a fixed number of taps (App. A
// entries): K x = sum_t kc[t] x[idx[t]], M x = sum_t mc[t] x[idx[t]].  Absent taps point at
// the position itself with zero coefficients, and every choice is a select, not a branch,
// so that the loads of several positions can be in flight together.  Hat rows have 7 taps
// (itself, the neighbouring hats, W_0 and W_1 of both adjacent elements), bubble rows 5
// (itself, degrees m -/+ 2, and for m <= 1 the hats of the element's two vertices).
template <int NT>
struct Taps {
    int idx[NT];
    double kc[NT], mc[NT];
};

__device__ __forceinline__ void hat_taps(const DimDev& d, int h, Taps<7>& t) {
    const int n = d.n, nh = d.nh, p = d.p;
    const int v = vertex_of_hat(d.bc, h);
    const bool has_l = v >= 1, has_r = v <= n - 1;
    const int ql = has_l ? v - 1 : 0, qr = has_r ? v : 0;
    const double dl = has_l ? d.delta[ql] : 0.0, il = has_l ? d.invdelta[ql] : 0.0;
    const double dr = has_r ? d.delta[qr] : 0.0, ir = has_r ? d.invdelta[qr] : 0.0;
    const bool hl = has_l && vertex_is_hat(d.bc, n, v - 1), hr = has_r && vertex_is_hat(d.bc, n, v + 1);
    t.idx[0] = h;
    t.kc[0] = il + ir + robin_at(d, v);
    t.mc[0] = (dl + dr) * (1.0 / 3.0);
    t.idx[1] = hl ? h - 1 : h;
    t.kc[1] = hl ? -il : 0.0;
    t.mc[1] = hl ? dl * (1.0 / 6.0) : 0.0;
    t.idx[2] = hr ? h + 1 : h;
    t.kc[2] = hr ? -ir : 0.0;
    t.mc[2] = hr ? dr * (1.0 / 6.0) : 0.0;
    const bool w0 = p >= 2, w1 = p >= 3;
    t.idx[3] = (has_l && w0) ? nh + ql : h;
    t.mc[3] = (has_l && w0) ? dl * (1.0 / 6.0) : 0.0;
    t.idx[4] = (has_l && w1) ? nh + n + ql : h;
    t.mc[4] = (has_l && w1) ? dl * (1.0 / 30.0) : 0.0;
    t.idx[5] = (has_r && w0) ? nh + qr : h;
    t.mc[5] = (has_r && w0) ? dr * (1.0 / 6.0) : 0.0;
    t.idx[6] = (has_r && w1) ? nh + n + qr : h;
    t.mc[6] = (has_r && w1) ? -dr * (1.0 / 30.0) : 0.0;
    t.kc[3] = t.kc[4] = t.kc[5] = t.kc[6] = 0.0;
}

__device__ __forceinline__ void bubble_taps(const DimDev& d, int pos, Taps<5>& t) {
    const int n = d.n, nh = d.nh, p = d.p;
    const int b = pos - nh, m = b / n, e = b - m * n;
    const double de = d.delta[e], ide = d.invdelta[e];
    const double* kd = d.tab64;
    const double* md = d.tab64 + d.tabstride;
    const double* mo = d.tab64 + 2 * d.tabstride;
    t.idx[0] = pos;
    t.kc[0] = kd[m] * ide;
    t.mc[0] = md[m] * de;
    const bool lo = m >= 2, hi = m + 2 <= p - 2;
    t.idx[1] = lo ? pos - 2 * n : pos;
    t.mc[1] = lo ? mo[lo ? m - 2 : 0] * de : 0.0;
    t.idx[2] = hi ? pos + 2 * n : pos;
    t.mc[2] = hi ? mo[m] * de : 0.0;
    const bool hl = m <= 1 && vertex_is_hat(d.bc, n, e), hr = m <= 1 && vertex_is_hat(d.bc, n, e + 1);
    const double cl = m == 0 ? de * (1.0 / 6.0) : -de * (1.0 / 30.0);
    const double cr = m == 0 ? de * (1.0 / 6.0) : de * (1.0 / 30.0);
    t.idx[3] = hl ? hat_of_vertex(d.bc, e) : pos;
    t.mc[3] = hl ? cl : 0.0;
    t.idx[4] = hr ? hat_of_vertex(d.bc, e + 1) : pos;
    t.mc[4] = hr ? cr : 0.0;
    t.kc[1] = t.kc[2] = t.kc[3] = t.kc[4] = 0.0;
}

__device__ __forceinline__ void make_taps(const DimDev& d, int pos, Taps<7>& t) { hat_taps(d, pos, t); }
__device__ __forceinline__ void make_taps(const DimDev& d, int pos, Taps<5>& t) { bubble_taps(d, pos, t); }

// Row operator: lines are rows (contiguous positions); thread x -> position, and a block
// takes kRowLines consecutive lines.  The position's stencil taps are computed once (they do
// not depend on the line) and every load of a line is independent of the others.
constexpr int kRowLines = 8;
template <int NT>
__device__ __forceinline__ void apply_rows_taps(const DimDev& d, const OpApply& a, int pos, int l0) {
    Taps<NT> t;
    make_taps(d, pos, t);
    const int l1 = min(l0 + kRowLines, a.nlines);
    for (int line = l0; line < l1; ++line) {
        const double* x = a.in + (long)line * a.in_sl;
        double Kx = 0.0, Mx = 0.0;
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const double v = x[(long)t.idx[q] * a.in_sp];
            Kx += t.kc[q] * v;
            Mx += t.mc[q] * v;
        }
        a.out1[(long)line * a.o1_sl + (long)pos * a.o1_sp] = a.k1 * Kx + a.t1 * Mx;
        if (a.out2) a.out2[(long)line * a.o2_sl + (long)pos * a.o2_sp] = a.k2 * Kx + a.t2 * Mx;
    }
}
__global__ void __launch_bounds__(256) op_apply_rows(DimDev d, OpApply a) {
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    const int l0 = blockIdx.y * kRowLines;
    if (pos >= d.N) return;
    if (pos < d.nh) apply_rows_taps<7>(d, a, pos, l0);
    else apply_rows_taps<5>(d, a, pos, l0);
}

// Column operator: lines are columns; thread x -> line (contiguous), y -> position.
__global__ void __launch_bounds__(256) op_apply_cols(DimDev d, OpApply a) {
    const int line = blockIdx.x * blockDim.x + threadIdx.x;
    const int pos = blockIdx.y;
    if (pos >= d.N || line >= a.nlines) return;
    double Kx, Mx;
    gather_km(d, a.in + (long)line * a.in_sl, a.in_sp, pos, Kx, Mx);
    a.out1[(long)line * a.o1_sl + (long)pos * a.o1_sp] = a.k1 * Kx + a.t1 * Mx;
    if (a.out2) a.out2[(long)line * a.o2_sl + (long)pos * a.o2_sp] = a.k2 * Kx + a.t2 * Mx;
}


// r[i][j] = alpha G[i][j] + beta ((ax_k K + ax_t M) T1 + M T2)[i][j], operators along x.
// A block owns 256 columns and a band of rows, all hats (7-tap rows) or all bubbles (5-tap
// rows); a thread takes RU rows at a time, whose taps are the same for every lane, and
// issues all their loads before any store, so that RU rows of gathers are in flight at
// once.  The weighted sums of squares are reduced per block (one atomic per sum).
template <int NT, bool PAIRS>
__device__ __forceinline__ void residual_rows(const DimDev& dx, const Residual& a, int j, int ibeg, int iend,
                                              double& sr, double& sg, double& su) {
    constexpr int RU = 4;
    for (int i0 = ibeg; i0 < iend; i0 += RU) {
        double rv[RU], gv[RU], uv[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int i = min(i0 + u, iend - 1);  // a repeated row past the band end is not stored
            Taps<NT> t;
            make_taps(dx, i, t);
            double K1 = 0.0, M1 = 0.0, M2 = 0.0;
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                double x1, x2;
                if constexpr (PAIRS) {
                    // (T1, T2) interleaved: one 16-byte load per tap
                    const double2 v = reinterpret_cast<const double2*>(a.T1)[(long)t.idx[q] * a.t_ld + j];
                    x1 = v.x;
                    x2 = v.y;
                } else {
                    x1 = a.T1[(long)t.idx[q] * a.t_ld + j];
                    x2 = a.T2[(long)t.idx[q] * a.t_ld + j];
                }
                K1 += t.kc[q] * x1;
                M1 += t.mc[q] * x1;
                M2 += t.mc[q] * x2;
            }
            gv[u] = a.G ? a.G[(long)i * a.g_ld + j] : 0.0;
            rv[u] = a.alpha * gv[u] + a.beta * (a.ax_k * K1 + a.ax_t * M1 + M2);
            uv[u] = a.U ? a.U[(long)i * a.u_ld + j] * M1 : 0.0;
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int i = i0 + u;
            if (i >= iend) continue;
            const double r = rv[u], g = gv[u];
            if (a.r64) a.r64[(long)i * a.r64_ld + j] = r;
            if (a.r32) a.r32[(long)i * a.r32_ld + j] = (float)r;
            if (a.norm_acc) {
                const double w = dx.mdiag[i] * a.wcol[j];
                sr += w * r * r;
                sg += w * g * g;
                su += uv[u];
            }
        }
    }
}

constexpr int kResRows = 4;  // rows per block: short-lived blocks, every load of a block in flight at once
template <bool PAIRS>
__global__ void __launch_bounds__(256) residual_kernel(DimDev dx, Residual a) {
    __shared__ double red[3][4];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    // bands of kResRows rows: first the hat rows, then the bubble rows, in address order.
    // (Bands ordered element block by element block, all degrees of a block in turn, cut the
    // HBM reads of the m -/+ 2 rows from 1.67x to 1.05x of the algorithmic bytes but took 377
    // instead of 305 us at N = 4095: consecutive workgroups then touch rows 2 MB apart.)
    const int hb = (dx.nh + kResRows - 1) / kResRows;
    double sr = 0.0, sg = 0.0, su = 0.0;
    if (j < a.ncols) {
        if ((int)blockIdx.y < hb) {
            const int ibeg = blockIdx.y * kResRows;
            residual_rows<7, PAIRS>(dx, a, j, ibeg, min(dx.nh, ibeg + kResRows), sr, sg, su);
        } else {
            const int ibeg = dx.nh + (blockIdx.y - hb) * kResRows;
            residual_rows<5, PAIRS>(dx, a, j, ibeg, min(dx.N, ibeg + kResRows), sr, sg, su);
        }
    }
    if (a.norm_acc) {
        sr = wave_sum(sr);
        sg = wave_sum(sg);
        su = wave_sum(su);
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[0][w] = sr;
            red[1][w] = sg;
            red[2][w] = su;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            const int k = threadIdx.x;
            const double t = red[k][0] + red[k][1] + red[k][2] + red[k][3];
            if (a.partials) {
                // one slot per block, summed by residual_reduce (thousands of same-address
                // atomics serialise at the L2 and dominated the kernel's time)
                const int nblk = gridDim.x * gridDim.y, b = blockIdx.y * gridDim.x + blockIdx.x;
                a.partials[(long)k * nblk + b] = t;
            } else if (k < 2 || a.U) {
                atomicAdd(a.norm_acc + k, t);
            }
        }
    }
}

// Two-stage sum of the residual's per-block partial sums (fixed order, deterministic):
// stage 1, block g of kReduceBlocks: out[k * kReduceBlocks + g] = sum over b = g (mod
// kReduceBlocks) of partials[k][b]; stage 2 (one block): norm_acc[k] += sum over g.
constexpr int kReduceBlocks = 128;
__global__ void __launch_bounds__(256) residual_reduce1(const double* __restrict__ partials, int nblk, int nk,
                                                        double* __restrict__ out) {
    __shared__ double red[4];
    for (int k = 0; k < nk; ++k) {
        double t = 0.0;
        for (int b = blockIdx.x + kReduceBlocks * threadIdx.x; b < nblk; b += kReduceBlocks * blockDim.x)
            t += partials[(long)k * nblk + b];
        t = wave_sum(t);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x == 0) out[k * kReduceBlocks + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
        __syncthreads();
    }
}
__global__ void __launch_bounds__(kReduceBlocks) residual_reduce2(const double* __restrict__ part1, int nk,
                                                                  double* norm_acc) {
    __shared__ double red[2];
    for (int k = 0; k < nk; ++k) {
        double t = wave_sum(part1[k * kReduceBlocks + threadIdx.x]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x == 0) norm_acc[k] += red[0] + red[1];
        __syncthreads();
    }
}

// (T f)[pos] for the load operator T = R^T M_P (App. A via eq. app:1, R_00, R_10).
__device__ __forceinline__ double gather_load(const DimDev& d, const double* f, long sp, int pos) {
    const int n = d.n, nh = d.nh;
    if (pos < nh) {
        const int v = vertex_of_hat(d.bc, pos);
        double acc = 0.0;
        if (v >= 1) {
            const int q = v - 1;
            const double dq = d.delta[q];
            acc += dq * 0.5 * f[(long)q * sp] + dq / 6.0 * f[(long)(n + q) * sp];
        }
        if (v <= n - 1) {
            const int q = v;
            const double dq = d.delta[q];
            acc += dq * 0.5 * f[(long)q * sp] - dq / 6.0 * f[(long)(n + q) * sp];
        }
        return acc;
    }
    const int b = pos - nh, m = b / n, e = b - m * n;
    const double de = d.delta[e];
    const double c0 = de / ((2.0 * m + 1.0) * (2.0 * m + 3.0));
    const double c2 = -de / ((2.0 * m + 3.0) * (2.0 * m + 5.0));
    return c0 * f[(long)(m * n + e) * sp] + c2 * f[(long)((m + 2) * n + e) * sp];
}

// H[i][j - j0] = (T_y F[i, :])[j] for the columns j0 <= j < j0 + ncols, i < Nleg_x.
__global__ void __launch_bounds__(256) load_rows(DimDev dy, const double* F, long ldf, double* H, long ldh,
                                                 int nrows, int j0, int ncols) {
    const int jj = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (jj >= ncols || i >= nrows) return;
    H[(long)i * ldh + jj] = gather_load(dy, F + (long)i * ldf, 1, j0 + jj);
}

// G[i][j0 + jj] = scale (T_x H[:, jj])[i], jj < ncols.
__global__ void __launch_bounds__(256) load_cols(DimDev dx, const double* H, long ldh, double* G, long ldg,
                                                 int j0, int ncols, double scale) {
    const int jj = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (jj >= ncols || i >= dx.N) return;
    G[(long)i * ldg + j0 + jj] = scale * gather_load(dx, H + jj, ldh, i);
}

__global__ void __launch_bounds__(256) convert_kernel(const double* src, long lds, float* dst, long ldd,
                                                      int rows, int cols, double* acc, const double* wr,
                                                      const double* wc) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    double s = 0.0;
    if (j < cols && i < rows) {
        const double v = src[(long)i * lds + j];
        dst[(long)i * ldd + j] = (float)v;
        if (acc) s = wr[i] * wc[j] * v * v;
    }
    if (acc) {
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0) atomicAdd(acc, s);
    }
}

__global__ void __launch_bounds__(256) zero_kernel(double* dst, long ld, int rows, int cols) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j < cols && i < rows) dst[(long)i * ld + j] = 0.0;
}

inline dim3 grid2(int inner, int outer) { return dim3((inner + 255) / 256, outer); }

}  // namespace

hipError_t launch_factor(const DimDev& d, int nf, const double* kappa_dev, const double* sigma_dev, double* fac64,
                         float* fac32, int stride, int* status_dev, hipStream_t s) {
    FactorLayout fl = make_factor_layout(d.n, d.p, d.nh);
    fl.stride = stride;
    hipLaunchKernelGGL(factor_kernel, dim3(nf), dim3(256), 0, s, d, kappa_dev, sigma_dev, fac64, fac32, fl,
                       status_dev);
    return hipGetLastError();
}

hipError_t launch_op_apply(const DimDev& d, const OpApply& a, bool column, hipStream_t s) {
    if (a.nlines <= 0 || d.N <= 0) return hipSuccess;
    if (column)
        hipLaunchKernelGGL(op_apply_cols, grid2(a.nlines, d.N), dim3(256), 0, s, d, a);
    else
        hipLaunchKernelGGL(op_apply_rows, grid2(d.N, (a.nlines + kRowLines - 1) / kRowLines), dim3(256), 0, s, d,
                           a);
    return hipGetLastError();
}

// Bands of kResRows hat rows, then of kResRows bubble rows; 256 columns per block.
static dim3 residual_grid(const DimDev& dx, int ncols) {
    const int nb = dx.N - dx.nh;
    const int bands = (dx.nh + kResRows - 1) / kResRows + (nb + kResRows - 1) / kResRows;
    return dim3((unsigned)((ncols + 255) / 256), (unsigned)bands);
}

long residual_partials(const DimDev& dx, int ncols) {
    const dim3 g = residual_grid(dx, ncols);
    return 3L * g.x * g.y + 3L * kReduceBlocks;  // per-block sums, then the first reduction stage
}

hipError_t launch_residual(const DimDev& dx, const Residual& a, hipStream_t s) {
    if (a.ncols <= 0 || dx.N <= 0) return hipSuccess;
    const dim3 g = residual_grid(dx, a.ncols);
    if (a.T2) hipLaunchKernelGGL(residual_kernel<false>, g, dim3(256), 0, s, dx, a);
    else hipLaunchKernelGGL(residual_kernel<true>, g, dim3(256), 0, s, dx, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.norm_acc || !a.partials) return e;
    const int nblk = (int)(g.x * g.y), nk = a.U ? 3 : 2;
    double* stage1 = a.partials + 3L * nblk;
    hipLaunchKernelGGL(residual_reduce1, dim3(kReduceBlocks), dim3(256), 0, s, a.partials, nblk, nk, stage1);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(residual_reduce2, dim3(1), dim3(kReduceBlocks), 0, s, stage1, nk, a.norm_acc);
    return hipGetLastError();
}

hipError_t launch_load(const DimDev& dx, const DimDev& dy, const double* F, long ldf, double* H, long ldh, double* G,
                       long ldg, hipStream_t s, double scale) {
    return launch_load_cols(dx, dy, F, ldf, H, ldh, G, ldg, 0, dy.N, s, scale);
}

hipError_t launch_load_cols(const DimDev& dx, const DimDev& dy, const double* F, long ldf, double* H, long ldh,
                            double* G, long ldg, int j0, int ncols, hipStream_t s, double scale) {
    if (ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(load_rows, grid2(ncols, dx.Nleg), dim3(256), 0, s, dy, F, ldf, H, ldh, dx.Nleg, j0, ncols);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(load_cols, grid2(ncols, dx.N), dim3(256), 0, s, dx, H, ldh, G, ldg, j0, ncols, scale);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed scratch for callers that cannot allocate: one array per device, holding a
// column block of the intermediate H = F T_y^T of the load.  In host code the name
// `scratch` is only a host-side stand-in; the device address comes from
// hipGetSymbolAddress, once per device, and only that address is passed to kernels.
// ---------------------------------------------------------------------------
namespace {
__device__ __align__(256) double scratch[kLoadScratchWords];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t load_scratch(double** out) {
    *out = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_convert_f64_f32(const double* src, long ld_src, float* dst, long ld_dst, int rows, int cols,
                                  double* norm_acc, const double* wr, const double* wc, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(convert_kernel, grid2(cols, rows), dim3(256), 0, s, src, ld_src, dst, ld_dst, rows, cols,
                       norm_acc, wr, wc);
    return hipGetLastError();
}

hipError_t launch_zero_f64(double* dst, long ld, int rows, int cols, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, grid2(cols, rows), dim3(256), 0, s, dst, ld, rows, cols);
    return hipGetLastError();
}

namespace {
__global__ void gather_acc_kernel(const double* const* accs, int count, double* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    // squared norms of the last correction and of U before it (lemma bound inputs)
    out[2 * i] = accs[i][0];
    out[2 * i + 1] = accs[i][4];
}
}  // namespace

namespace {
__global__ void zero_acc_kernel(double* const* accs, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    accs[i][0] = 0.0;
    accs[i][1] = 0.0;
}
}  // namespace

hipError_t launch_zero_accs(double* const* accs, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_acc_kernel, dim3((count + 255) / 256), dim3(256), 0, s, accs, count);
    return hipGetLastError();
}

hipError_t launch_gather_acc(const double* const* accs, int count, double* out, hipStream_t s) {
    hipLaunchKernelGGL(gather_acc_kernel, dim3((count + 255) / 256), dim3(256), 0, s, accs, count, out);
    return hipGetLastError();
}

}  // namespace hpadi
