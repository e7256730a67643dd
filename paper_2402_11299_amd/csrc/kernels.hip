// HIP kernels of hpadi for gfx950 (MI355X).
//
// Everything here is bandwidth-bound banded work: no matrix cores.
//  * factor_kernel   reverse Cholesky of kappa K + sigma M (Sec. 4, Alg. 1), one
//                    workgroup per matrix, one thread per (element, parity) chain,
//                    the hat Schur complement in FP64 by one thread.
//  * line_pass       one ADI half-sweep (Sec. 5, Alg. 2): per line a solve with the
//                    structured factor (corollary of Sec. 4) fused with the banded
//                    product of the next half-step.  One thread owns one element of
//                    one line and keeps both of its bubble chains in registers; the
//                    hat system is solved per line through LDS.
//  * op_apply, residual, load: elementwise gathers of the banded operators.
//
// Coefficient order (per dimension, Sec. 2.2): hats 0..nh-1, then bubble (m, e)
// at nh + m n + e.  Element e has left vertex e and right vertex e+1; vertex v
// is hat v-1 (Dirichlet, v = 1..n-1) or hat v (Neumann, v = 0..n).

#include <hip/hip_runtime.h>

#include "internal.h"

namespace hpadi {

namespace {

__device__ __forceinline__ bool vertex_is_hat(int bc, int n, int v) {
    return bc == 0 ? (v >= 1 && v <= n - 1) : (v >= 0 && v <= n);
}
__device__ __forceinline__ int hat_of_vertex(int bc, int v) { return bc == 0 ? v - 1 : v; }
__device__ __forceinline__ int vertex_of_hat(int bc, int h) { return bc == 0 ? h + 1 : h; }

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
            double a = 0.0;
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

// ---------------------------------------------------------------------------
// ADI half-sweep over lines.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ const T* tables(const DimDev& d);
template <>
__device__ __forceinline__ const double* tables<double>(const DimDev& d) {
    return d.tab64;
}
template <>
__device__ __forceinline__ const float* tables<float>(const DimDev& d) {
    return d.tab32;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

constexpr int max_threads_for(int cl, int tsize) {
    return (2 * cl * tsize / 4) <= 64 ? 1024 : ((2 * cl * tsize / 4) <= 128 ? 512 : 256);
}

template <typename T, int CL, int MODE, bool COL>
__global__ void __launch_bounds__(max_threads_for(CL, sizeof(T)))
    line_pass_kernel(DimDev d, LinePass a, int lpb) {
    extern __shared__ unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int n = d.n, p = d.p, nh = d.nh;
    const int hs = nh + 1;
    T* hb = sm;             // [lpb][hs]: hat right-hand side, then hat solution
    T* hd = sm + lpb * hs;  // [lpb][n][2]: chain heads (y, then x)

    const int t = threadIdx.x;
    int l, e;
    if (COL) {
        l = t % lpb;
        e = t / lpb;
    } else {
        e = t % n;
        l = t / n;
    }
    const int line = blockIdx.x * lpb + l;
    const bool act = line < a.nlines;
    const int le = p / 2, lo = (p - 1) / 2;

    const T* fac = reinterpret_cast<const T*>(a.fac);
    const T* invd = fac + a.fl.off_invd;
    const T* link = fac + a.fl.off_link;
    const T* cpl = fac + a.fl.off_cpl;
    const T* invd0 = fac + a.fl.off_invd0;
    const T* link0 = fac + a.fl.off_link0;

    T ev[CL], od[CL];
    T* hbl = hb + l * hs;
    T* hdl = hd + l * 2 * n;

    // ---- load the line: both chains of element e into registers, hats into LDS
    if (act) {
        const T* in = reinterpret_cast<const T*>(a.in) + (long)line * a.in_sl;
#pragma unroll
        for (int s = 0; s < CL; ++s) {
            if (s < le) ev[s] = in[(long)(nh + (2 * s) * n + e) * a.in_sp];
            if (s < lo) od[s] = in[(long)(nh + (2 * s + 1) * n + e) * a.in_sp];
        }
        if (e < nh) hbl[e] = in[(long)e * a.in_sp];
        if (e == 0 && nh == n + 1) hbl[n] = in[(long)n * a.in_sp];
        // ---- L~^T y = b along each chain, highest degree first
#pragma unroll
        for (int s = CL - 1; s >= 0; --s) {
            if (s < le) {
                T v = ev[s];
                if (s + 1 < CL) {
                    if (s + 1 < le) v -= link[(2 * s + 2) * n + e] * ev[s + 1];
                }
                ev[s] = v * invd[(2 * s) * n + e];
            }
            if (s < lo) {
                T v = od[s];
                if (s + 1 < CL) {
                    if (s + 1 < lo) v -= link[(2 * s + 3) * n + e] * od[s + 1];
                }
                od[s] = v * invd[(2 * s + 1) * n + e];
            }
        }
        hdl[2 * e + 0] = le > 0 ? ev[0] : T(0);
        hdl[2 * e + 1] = lo > 0 ? od[0] : T(0);
    }
    __syncthreads();
    // ---- hat right-hand side b_h - (C^T y)_h
    if (act) {
        for (int h = e; h < nh; h += n) {
            const int v = vertex_of_hat(d.bc, h);
            T acc = hbl[h];
            if (v >= 1) {
                const int q = v - 1;
                acc -= cpl[4 * q + 1] * hdl[2 * q] + cpl[4 * q + 3] * hdl[2 * q + 1];
            }
            if (v <= n - 1) {
                const int q = v;
                acc -= cpl[4 * q + 0] * hdl[2 * q] + cpl[4 * q + 2] * hdl[2 * q + 1];
            }
            hbl[h] = acc;
        }
    }
    __syncthreads();
    // ---- hat block: L0^T z = bhat (last hat first), then L0 x = z
    if (act && e == 0) {
        T z = T(0);
        for (int h = nh - 1; h >= 0; --h) {
            T v = hbl[h];
            if (h + 1 < nh) v -= link0[h + 1] * z;
            z = v * invd0[h];
            hbl[h] = z;
        }
        T x = T(0);
        for (int h = 0; h < nh; ++h) {
            T v = hbl[h];
            if (h > 0) v -= link0[h] * x;
            x = v * invd0[h];
            hbl[h] = x;
        }
    }
    __syncthreads();
    // ---- L~ x = y - C x_h along each chain, lowest degree first
    T xl = T(0), xr = T(0);
    if (act) {
        if (vertex_is_hat(d.bc, n, e)) xl = hbl[hat_of_vertex(d.bc, e)];
        if (vertex_is_hat(d.bc, n, e + 1)) xr = hbl[hat_of_vertex(d.bc, e + 1)];
        if (le > 0) ev[0] = (ev[0] - cpl[4 * e + 0] * xl - cpl[4 * e + 1] * xr) * invd[e];
        if (lo > 0) od[0] = (od[0] - cpl[4 * e + 2] * xl - cpl[4 * e + 3] * xr) * invd[n + e];
#pragma unroll
        for (int s = 1; s < CL; ++s) {
            if (s < le) ev[s] = (ev[s] - link[(2 * s) * n + e] * ev[s - 1]) * invd[(2 * s) * n + e];
            if (s < lo) od[s] = (od[s] - link[(2 * s + 1) * n + e] * od[s - 1]) * invd[(2 * s + 1) * n + e];
        }
        hdl[2 * e + 0] = le > 0 ? ev[0] : T(0);
        hdl[2 * e + 1] = lo > 0 ? od[0] : T(0);
    }
    __syncthreads();

    // ---- outputs
    if (act && MODE == MODE_PRODUCT) {
        // out = G - (kappa K + tau M) x   (App. A entries)
        const T* G = reinterpret_cast<const T*>(a.g) + (long)line * a.g_sl;
        T* out = reinterpret_cast<T*>(a.out) + (long)line * a.out_sl;
        const T* tb = tables<T>(d);
        const T* kd = tb;
        const T* md = tb + d.tabstride;
        const T* mo = tb + 2 * d.tabstride;
        const T kap = (T)a.kappa, tau = (T)a.tau;
        const T de = (T)d.delta[e], ide = (T)d.invdelta[e];
        const T tde = tau * de;
#pragma unroll
        for (int s = 0; s < CL; ++s) {
            if (s < le) {
                const int m = 2 * s;
                T y = (kap * kd[m] * ide + tde * md[m]) * ev[s];
                if (s > 0) y += tde * mo[m - 2] * ev[s - 1];
                if (s + 1 < CL) {
                    if (s + 1 < le) y += tde * mo[m] * ev[s + 1];
                }
                if (s == 0) y += tde * (T(1) / T(6)) * (xl + xr);
                const long pos = nh + m * n + e;
                out[pos * a.out_sp] = G[pos * a.g_sp] - y;
            }
            if (s < lo) {
                const int m = 2 * s + 1;
                T y = (kap * kd[m] * ide + tde * md[m]) * od[s];
                if (s > 0) y += tde * mo[m - 2] * od[s - 1];
                if (s + 1 < CL) {
                    if (s + 1 < lo) y += tde * mo[m] * od[s + 1];
                }
                if (s == 0) y += tde * (T(1) / T(30)) * (xr - xl);
                const long pos = nh + m * n + e;
                out[pos * a.out_sp] = G[pos * a.g_sp] - y;
            }
        }
        for (int h = e; h < nh; h += n) {
            const int v = vertex_of_hat(d.bc, h);
            const T xh = hbl[h];
            T y = T(0);
            if (v >= 1) {
                const int q = v - 1;
                const T dq = (T)d.delta[q], idq = (T)d.invdelta[q];
                y += (kap * idq + tau * dq * (T(1) / T(3))) * xh;
                if (vertex_is_hat(d.bc, n, v - 1)) y += (-kap * idq + tau * dq * (T(1) / T(6))) * hbl[h - 1];
                y += tau * dq * (hdl[2 * q] * (T(1) / T(6)) + hdl[2 * q + 1] * (T(1) / T(30)));
            }
            if (v <= n - 1) {
                const int q = v;
                const T dq = (T)d.delta[q], idq = (T)d.invdelta[q];
                y += (kap * idq + tau * dq * (T(1) / T(3))) * xh;
                if (vertex_is_hat(d.bc, n, v + 1)) y += (-kap * idq + tau * dq * (T(1) / T(6))) * hbl[h + 1];
                y += tau * dq * (hdl[2 * q] * (T(1) / T(6)) - hdl[2 * q + 1] * (T(1) / T(30)));
            }
            out[(long)h * a.out_sp] = G[(long)h * a.g_sp] - y;
        }
    } else if (act && MODE == MODE_SOLVE) {
        T* out = reinterpret_cast<T*>(a.out) + (long)line * a.out_sl;
#pragma unroll
        for (int s = 0; s < CL; ++s) {
            if (s < le) out[(long)(nh + (2 * s) * n + e) * a.out_sp] = ev[s];
            if (s < lo) out[(long)(nh + (2 * s + 1) * n + e) * a.out_sp] = od[s];
        }
        for (int h = e; h < nh; h += n) out[(long)h * a.out_sp] = hbl[h];
    } else if (MODE == MODE_ACCUM) {
        // U += x in FP64, with weighted sums of squares of the update and of U
        double sdx = 0.0, su = 0.0;
        if (act) {
        double* out = reinterpret_cast<double*>(a.out) + (long)line * a.out_sl;
        const double* w = d.mdiag;
#pragma unroll
        for (int s = 0; s < CL; ++s) {
            if (s < le) {
                const long pos = nh + (2 * s) * n + e;
                const double dx = (double)ev[s];
                const double u = out[pos * a.out_sp] + dx;
                out[pos * a.out_sp] = u;
                sdx += w[pos] * dx * dx;
                su += w[pos] * u * u;
            }
            if (s < lo) {
                const long pos = nh + (2 * s + 1) * n + e;
                const double dx = (double)od[s];
                const double u = out[pos * a.out_sp] + dx;
                out[pos * a.out_sp] = u;
                sdx += w[pos] * dx * dx;
                su += w[pos] * u * u;
            }
        }
        for (int h = e; h < nh; h += n) {
            const double dx = (double)hbl[h];
            const double u = out[(long)h * a.out_sp] + dx;
            out[(long)h * a.out_sp] = u;
            sdx += w[h] * dx * dx;
            su += w[h] * u * u;
        }
        if (a.norm_acc) {
            const double wl = a.wline[line];
            sdx *= wl;
            su *= wl;
        }
        }
        if (a.norm_acc) {
            // block reduction through LDS (the launch sizes LDS for 2 doubles per thread)
            __syncthreads();
            double* red = reinterpret_cast<double*>(smem_raw);
            red[2 * t] = sdx;
            red[2 * t + 1] = su;
            __syncthreads();
            for (int w = blockDim.x; w > 1; w = (w + 1) / 2) {
                const int half = (w + 1) / 2;
                if (t + half < w) {
                    red[2 * t] += red[2 * (t + half)];
                    red[2 * t + 1] += red[2 * (t + half) + 1];
                }
                __syncthreads();
            }
            if (t == 0) {
                atomicAdd(a.norm_acc + 0, red[0]);
                atomicAdd(a.norm_acc + 1, red[1]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Elementwise banded operators.
// ---------------------------------------------------------------------------

// K x and M x at position pos of a line x (stride sp), App. A entries.
__device__ __forceinline__ void gather_km(const DimDev& d, const double* x, long sp, int pos, double& Kx,
                                          double& Mx) {
    const int n = d.n, nh = d.nh, p = d.p;
    Kx = 0.0;
    Mx = 0.0;
    if (pos < nh) {
        const int h = pos, v = vertex_of_hat(d.bc, h);
        const double xh = x[(long)h * sp];
        if (v >= 1) {
            const int q = v - 1;
            const double dq = d.delta[q], idq = d.invdelta[q];
            Kx += idq * xh;
            Mx += dq / 3.0 * xh;
            if (vertex_is_hat(d.bc, n, v - 1)) {
                const double xn = x[(long)(h - 1) * sp];
                Kx -= idq * xn;
                Mx += dq / 6.0 * xn;
            }
            if (p >= 2) Mx += dq / 6.0 * x[(long)(nh + q) * sp];
            if (p >= 3) Mx += dq / 30.0 * x[(long)(nh + n + q) * sp];
        }
        if (v <= n - 1) {
            const int q = v;
            const double dq = d.delta[q], idq = d.invdelta[q];
            Kx += idq * xh;
            Mx += dq / 3.0 * xh;
            if (vertex_is_hat(d.bc, n, v + 1)) {
                const double xn = x[(long)(h + 1) * sp];
                Kx -= idq * xn;
                Mx += dq / 6.0 * xn;
            }
            if (p >= 2) Mx += dq / 6.0 * x[(long)(nh + q) * sp];
            if (p >= 3) Mx -= dq / 30.0 * x[(long)(nh + n + q) * sp];
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
            Mx += (m == 0) ? de / 6.0 * (xl + xr) : de / 30.0 * (xr - xl);
        }
    }
}

// Row operator: lines are rows (contiguous positions); thread x -> position.
__global__ void __launch_bounds__(256) op_apply_rows(DimDev d, OpApply a) {
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    const int line = blockIdx.y;
    if (pos >= d.N || line >= a.nlines) return;
    double Kx, Mx;
    gather_km(d, a.in + (long)line * a.in_sl, a.in_sp, pos, Kx, Mx);
    a.out1[(long)line * a.o1_sl + (long)pos * a.o1_sp] = a.k1 * Kx + a.t1 * Mx;
    if (a.out2) a.out2[(long)line * a.o2_sl + (long)pos * a.o2_sp] = a.k2 * Kx + a.t2 * Mx;
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
__global__ void __launch_bounds__(256) residual_kernel(DimDev dx, Residual a) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    double sr = 0.0, sg = 0.0;
    if (j < a.ncols && i < dx.N) {
        double K1, M1, K2, M2;
        gather_km(dx, a.T1 + j, a.t_ld, i, K1, M1);
        gather_km(dx, a.T2 + j, a.t_ld, i, K2, M2);
        const double g = a.G ? a.G[(long)i * a.g_ld + j] : 0.0;
        const double r = a.alpha * g + a.beta * (a.ax_k * K1 + a.ax_t * M1 + M2);
        if (a.r64) a.r64[(long)i * a.r64_ld + j] = r;
        if (a.r32) a.r32[(long)i * a.r32_ld + j] = (float)r;
        if (a.norm_acc) {
            const double w = dx.mdiag[i] * a.wcol[j];
            sr = w * r * r;
            sg = w * g * g;
        }
    }
    if (a.norm_acc) {
        sr = wave_sum(sr);
        sg = wave_sum(sg);
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(a.norm_acc + 0, sr);
            atomicAdd(a.norm_acc + 1, sg);
        }
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

// H[i][j] = (T_y F[i, :])[j], i < Nleg_x.
__global__ void __launch_bounds__(256) load_rows(DimDev dy, const double* F, long ldf, double* H, long ldh,
                                                 int nrows) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= dy.N || i >= nrows) return;
    H[(long)i * ldh + j] = gather_load(dy, F + (long)i * ldf, 1, j);
}

// G[i][j] = (T_x H[:, j])[i].
__global__ void __launch_bounds__(256) load_cols(DimDev dx, const double* H, long ldh, double* G, long ldg,
                                                 int ncols) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= ncols || i >= dx.N) return;
    G[(long)i * ldg + j] = gather_load(dx, H + j, ldh, i);
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

template <typename T, int CL, int MODE, bool COL>
hipError_t launch_lp(const DimDev& d, const LinePass& a, int lpb, hipStream_t s) {
    const int threads = lpb * d.n;
    if (threads > max_threads_for(CL, sizeof(T)) || threads <= 0) return hipErrorInvalidValue;
    const int blocks = (a.nlines + lpb - 1) / lpb;
    size_t shm = (size_t)lpb * (d.nh + 1 + 2 * d.n) * sizeof(T);
    if (MODE == MODE_ACCUM && shm < (size_t)threads * 2 * sizeof(double)) shm = (size_t)threads * 2 * sizeof(double);
    hipLaunchKernelGGL((line_pass_kernel<T, CL, MODE, COL>), dim3(blocks), dim3(threads), shm, s, d, a, lpb);
    return hipGetLastError();
}

template <typename T, int CL>
hipError_t dispatch_mode(const DimDev& d, const LinePass& a, int mode, bool col, int lpb, hipStream_t s) {
    if (mode == MODE_PRODUCT) return col ? launch_lp<T, CL, MODE_PRODUCT, true>(d, a, lpb, s)
                                         : launch_lp<T, CL, MODE_PRODUCT, false>(d, a, lpb, s);
    if (mode == MODE_SOLVE) return col ? launch_lp<T, CL, MODE_SOLVE, true>(d, a, lpb, s)
                                       : launch_lp<T, CL, MODE_SOLVE, false>(d, a, lpb, s);
    return col ? launch_lp<T, CL, MODE_ACCUM, true>(d, a, lpb, s) : launch_lp<T, CL, MODE_ACCUM, false>(d, a, lpb, s);
}

template <typename T>
hipError_t dispatch_cl(const DimDev& d, const LinePass& a, int mode, bool col, int lpb, hipStream_t s) {
    const int need = d.p / 2;
    if (need <= 4) return dispatch_mode<T, 4>(d, a, mode, col, lpb, s);
    if (need <= 8) return dispatch_mode<T, 8>(d, a, mode, col, lpb, s);
    if (need <= 16) return dispatch_mode<T, 16>(d, a, mode, col, lpb, s);
    if (need <= 32) return dispatch_mode<T, 32>(d, a, mode, col, lpb, s);
    if (need <= 64) return dispatch_mode<T, 64>(d, a, mode, col, lpb, s);
    return hipErrorInvalidValue;
}

inline dim3 grid2(int inner, int outer) { return dim3((inner + 255) / 256, outer); }

}  // namespace

int line_pass_max_threads(int p, bool fp32) {
    const int need = p / 2;
    const int cl = need <= 4 ? 4 : need <= 8 ? 8 : need <= 16 ? 16 : need <= 32 ? 32 : 64;
    return max_threads_for(cl, fp32 ? 4 : 8);
}

hipError_t launch_factor(const DimDev& d, int nf, const double* kappa_dev, const double* sigma_dev, double* fac64,
                         float* fac32, int stride, int* status_dev, hipStream_t s) {
    FactorLayout fl = make_factor_layout(d.n, d.p, d.nh);
    fl.stride = stride;
    hipLaunchKernelGGL(factor_kernel, dim3(nf), dim3(256), 0, s, d, kappa_dev, sigma_dev, fac64, fac32, fl,
                       status_dev);
    return hipGetLastError();
}

hipError_t launch_line_pass(const DimDev& d, const LinePass& a, bool fp32, bool /*g_fp32*/, int mode, bool column,
                            int lines_per_block, hipStream_t s) {
    if (a.nlines <= 0) return hipSuccess;
    return fp32 ? dispatch_cl<float>(d, a, mode, column, lines_per_block, s)
                : dispatch_cl<double>(d, a, mode, column, lines_per_block, s);
}

hipError_t launch_op_apply(const DimDev& d, const OpApply& a, bool column, hipStream_t s) {
    if (a.nlines <= 0 || d.N <= 0) return hipSuccess;
    if (column)
        hipLaunchKernelGGL(op_apply_cols, grid2(a.nlines, d.N), dim3(256), 0, s, d, a);
    else
        hipLaunchKernelGGL(op_apply_rows, grid2(d.N, a.nlines), dim3(256), 0, s, d, a);
    return hipGetLastError();
}

hipError_t launch_residual(const DimDev& dx, const Residual& a, hipStream_t s) {
    if (a.ncols <= 0 || dx.N <= 0) return hipSuccess;
    hipLaunchKernelGGL(residual_kernel, grid2(a.ncols, dx.N), dim3(256), 0, s, dx, a);
    return hipGetLastError();
}

hipError_t launch_load(const DimDev& dx, const DimDev& dy, const double* F, long ldf, double* H, long ldh, double* G,
                       long ldg, hipStream_t s) {
    hipLaunchKernelGGL(load_rows, grid2(dy.N, dx.Nleg), dim3(256), 0, s, dy, F, ldf, H, ldh, dx.Nleg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(load_cols, grid2(dy.N, dx.N), dim3(256), 0, s, dx, H, ldh, G, ldg, dy.N);
    return hipGetLastError();
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

}  // namespace hpadi
