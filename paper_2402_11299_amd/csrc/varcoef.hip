// Variable-coefficient operator -div(a grad u) in the hat+bubble basis, and the
// vector kernels of the Krylov iterations that use it (Sec. 7: a CG iteration
// preconditioned by the constant-coefficient ADI solve).
//
// The Galerkin form a_h(u, v) = sum_e sum_(i,j) w_i w_j a(x_i, y_j) grad u . grad v
// is evaluated with q = p + 2 Gauss-Legendre points per element and dimension.
// One workgroup owns one element pair (e_x, e_y): it gathers the (p_x+1) x (p_y+1)
// local coefficients into LDS, forms the x- and y-derivatives at the q_x x q_y
// points by two small dense products each, weights them by a w_i w_j and the
// element's aspect ratio, and maps back by the transposed products.  Element
// results go to an element-major scratch array; a second kernel sums, for every
// global coefficient, the (at most four) element contributions that share it
// (a hat belongs to the two elements of its vertex).  Both passes are FP64 and
// atomic-free, so results are deterministic.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "krylov.h"

namespace hpadi {

namespace {

__global__ void __launch_bounds__(256) vc_element_kernel(VarCoefDev v, const double* __restrict__ U, long ldu) {
    extern __shared__ double sm[];
    const int Lx = v.px + 1, Ly = v.py + 1, qx = v.qx, qy = v.qy;
    double* Ue = sm;                    // Lx x Ly
    double* Tm = Ue + Lx * Ly;          // qx x Ly
    double* Pm = Tm + qx * Ly;          // qx x qy
    double* EyT = Pm + qx * qy;         // Ly x qy (transposed y table of the current term)
    const int ex = blockIdx.x / v.ny, ey = blockIdx.x % v.ny;
    const int tid = threadIdx.x, nt = blockDim.x;

    for (int idx = tid; idx < Lx * Ly; idx += nt) {
        const int lx = idx / Ly, ly = idx - lx * Ly;
        const int gi = v.l2gx[ex * Lx + lx], gj = v.l2gy[ey * Ly + ly];
        Ue[idx] = (gi >= 0 && gj >= 0) ? U[(long)gi * ldu + gj] : 0.0;
    }
    const double ratio = v.dely[ey] / v.delx[ex];
    double* Yout = v.Ye + (size_t)blockIdx.x * Lx * Ly;

    for (int term = 0; term < 2; ++term) {
        // term 0: d/dx u d/dx v (derivative table on x, value table on y); term 1: the y pair
        const double* Ex = term == 0 ? v.Edx : v.Evx;
        const double* Ey = term == 0 ? v.Evy : v.Edy;
        const double scale = term == 0 ? ratio : 1.0 / ratio;
        for (int idx = tid; idx < qy * Ly; idx += nt) {
            const int j = idx / Ly, ly = idx - j * Ly;
            EyT[ly * qy + j] = Ey[idx];
        }
        __syncthreads();
        // Tm = Ex Ue (qx x Ly)
        for (int idx = tid; idx < qx * Ly; idx += nt) {
            const int i = idx / Ly, ly = idx - i * Ly;
            const double* er = Ex + i * Lx;
            double s = 0.0;
            for (int lx = 0; lx < Lx; ++lx) s += er[lx] * Ue[lx * Ly + ly];
            Tm[idx] = s;
        }
        __syncthreads();
        // Pm = (Tm Ey^T) .* (a w_i w_j scale)  (qx x qy)
        for (int idx = tid; idx < qx * qy; idx += nt) {
            const int i = idx / qy, j = idx - i * qy;
            const double* tr = Tm + i * Ly;
            double s = 0.0;
            for (int ly = 0; ly < Ly; ++ly) s += tr[ly] * EyT[ly * qy + j];
            const double a = v.a[(long)(ex * qx + i) * v.lda + (ey * qy + j)];
            Pm[idx] = s * a * v.wx[i] * v.wy[j] * scale;
        }
        __syncthreads();
        // Tm = Pm Ey (qx x Ly)
        for (int idx = tid; idx < qx * Ly; idx += nt) {
            const int i = idx / Ly, ly = idx - i * Ly;
            const double* pr = Pm + i * qy;
            double s = 0.0;
            for (int j = 0; j < qy; ++j) s += pr[j] * Ey[j * Ly + ly];
            Tm[idx] = s;
        }
        __syncthreads();
        // Y (+)= Ex^T Tm (Lx x Ly)
        for (int idx = tid; idx < Lx * Ly; idx += nt) {
            const int lx = idx / Ly, ly = idx - lx * Ly;
            double s = 0.0;
            for (int i = 0; i < qx; ++i) s += Ex[i * Lx + lx] * Tm[i * Ly + ly];
            Yout[idx] = term == 0 ? s : Yout[idx] + s;
        }
        __syncthreads();
    }
}

// Y[i][j] = sum over the element/local pairs owning i and j of the element results.
__global__ void vc_gather_kernel(VarCoefDev v, double* __restrict__ Y, long ldy) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= v.Ny) return;
    const int Lx = v.px + 1, Ly = v.py + 1;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int exi = v.ownx[4 * i + 2 * a], lxi = v.ownx[4 * i + 2 * a + 1];
        if (exi < 0) continue;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int eyj = v.owny[4 * j + 2 * b], lyj = v.owny[4 * j + 2 * b + 1];
            if (eyj < 0) continue;
            s += v.Ye[((size_t)(exi * v.ny + eyj) * Lx + lxi) * Ly + lyj];
        }
    }
    Y[(long)i * ldy + j] = s;
}

// ---- separable terms: four passes of banded-block products per term ---------
// Every pass is a gather along one axis with the local tables: the x-axis maps
// coefficient rows to Gauss-point rows (and back), the y-axis columns likewise.
// They hold no per-element dense block, so any degree fits (the element kernel's
// LDS tile caps p near 80).

// T1[e q + i][j] = sum_l Ex[i][l] U[g_x(e, l)][j]
__global__ void __launch_bounds__(256) sep_rows_to_points(VarCoefDev v, const double* __restrict__ Ex,
                                                          const double* __restrict__ U, long ldu) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (j >= v.Ny) return;
    const int Lx = v.px + 1, e = r / v.qx, i = r - e * v.qx;
    const int* g = v.l2gx + e * Lx;
    const double* er = Ex + i * Lx;
    double s = 0.0;
    for (int l = 0; l < Lx; ++l) {
        const int gi = g[l];
        if (gi >= 0) s += er[l] * U[(long)gi * ldu + j];
    }
    v.T1[(long)r * v.Ny + j] = s;
}

// T2[r][e q + j] = C[r][e q + j] sum_l T1[r][g_y(e, l)] Ey[j][l]
__global__ void __launch_bounds__(256) sep_cols_to_points(VarCoefDev v, const double* __restrict__ Ey,
                                                          const double* __restrict__ C) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const int nqy = v.ny * v.qy;
    if (c >= nqy) return;
    const int Ly = v.py + 1, e = c / v.qy, jj = c - e * v.qy;
    const int* g = v.l2gy + e * Ly;
    const double* t = v.T1 + (long)r * v.Ny;
    const double* er = Ey + jj * Ly;
    double s = 0.0;
    for (int l = 0; l < Ly; ++l) {
        const int gj = g[l];
        if (gj >= 0) s += t[gj] * er[l];
    }
    v.T2[(long)r * nqy + c] = s * C[(long)r * nqy + c];
}

// T1[r][j] = sum over the (element, local) owners of column j of sum_jj T2[r][e q + jj] Ey[jj][l]
__global__ void __launch_bounds__(256) sep_points_to_cols(VarCoefDev v, const double* __restrict__ Ey) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (j >= v.Ny) return;
    const int Ly = v.py + 1, nqy = v.ny * v.qy;
    const double* t = v.T2 + (long)r * nqy;
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int e = v.owny[4 * j + 2 * b], l = v.owny[4 * j + 2 * b + 1];
        if (e < 0) continue;
        for (int jj = 0; jj < v.qy; ++jj) s += t[e * v.qy + jj] * Ey[jj * Ly + l];
    }
    v.T1[(long)r * v.Ny + j] = s;
}

// Y[i][j] (+)= sum over the owners (e, l) of row i of sum_ii Ex[ii][l] T1[e q + ii][j]
__global__ void __launch_bounds__(256) sep_points_to_rows(VarCoefDev v, const double* __restrict__ Ex, double* Y,
                                                          long ldy, int accumulate) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= v.Ny) return;
    const int Lx = v.px + 1;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int e = v.ownx[4 * i + 2 * a], l = v.ownx[4 * i + 2 * a + 1];
        if (e < 0) continue;
        for (int ii = 0; ii < v.qx; ++ii) s += Ex[ii * Lx + l] * v.T1[(long)(e * v.qx + ii) * v.Ny + j];
    }
    double* y = Y + (long)i * ldy + j;
    *y = accumulate ? *y + s : s;
}

// ---- vector kernels (compact row-major N_x x N_y arrays, FP64) ------------

__device__ inline double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    __syncthreads();
    return s;
}

// part[k * gridDim.x + block] = partial sum of a . b_k, k < nb (at most 4)
__global__ void __launch_bounds__(256) multidot_kernel(const double* __restrict__ a, MultiB bs, long n,
                                                       double* __restrict__ part) {
    __shared__ double red[4];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
        const double av = a[idx];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < bs.nb) s[k] += av * bs.b[k][idx];
    }
    for (int k = 0; k < bs.nb; ++k) {
        const double t = block_sum(s[k], red);
        if (threadIdx.x == 0) part[k * gridDim.x + blockIdx.x] = t;
    }
}

// out[k] = sum of the partials of dot k (one workgroup, fixed order)
__global__ void __launch_bounds__(256) finish_dot_kernel(const double* __restrict__ part, int nparts, int nb,
                                                         double* __restrict__ out) {
    __shared__ double red[4];
    for (int k = 0; k < nb; ++k) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += part[k * nparts + i];
        const double t = block_sum(s, red);
        if (threadIdx.x == 0) out[k] = t;
    }
}

// y = y + sum_k c_k x_k  (nk <= 4)
__global__ void axpys_kernel(double* __restrict__ y, MultiB xs, Coefs c, long n) {
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
        double v = y[idx];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < xs.nb) v += c.c[k] * xs.b[k][idx];
        y[idx] = v;
    }
}

// y = x + beta y
__global__ void xpby_kernel(double* __restrict__ y, const double* __restrict__ x, double beta, long n) {
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x)
        y[idx] = x[idx] + beta * y[idx];
}

// strided 2D copy (rows x cols), FP64
__global__ void copy2d_kernel(const double* __restrict__ x, long ldx, double* __restrict__ y, long ldy, int cols) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j < cols) y[(long)i * ldy + j] = x[(long)i * ldx + j];
}

constexpr int kDotBlocks = 512;

}  // namespace

size_t vc_lds_bytes(int px, int py) {
    const int Lx = px + 1, Ly = py + 1, qx = px + 2, qy = py + 2;
    return sizeof(double) * ((size_t)Lx * Ly + (size_t)qx * Ly + (size_t)qx * qy + (size_t)Ly * qy);
}

hipError_t launch_vc_apply(const VarCoefDev& v, const double* U, long ldu, double* Y, long ldy, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (v.element_terms) {
        const size_t lds = vc_lds_bytes(v.px, v.py);
        if (lds > 160 * 1024) return hipErrorInvalidValue;
        hipLaunchKernelGGL(vc_element_kernel, dim3(v.nx * v.ny), dim3(256), lds, s, v, U, ldu);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(vc_gather_kernel, dim3((v.Ny + 255) / 256, v.Nx), dim3(256), 0, s, v, Y, ldy);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int nqx = v.nx * v.qx, nqy = v.ny * v.qy;
    for (int t = 0; t < v.nsep; ++t) {
        hipLaunchKernelGGL(sep_rows_to_points, dim3((v.Ny + 255) / 256, nqx), dim3(256), 0, s, v, v.sEx[t], U, ldu);
        hipLaunchKernelGGL(sep_cols_to_points, dim3((nqy + 255) / 256, nqx), dim3(256), 0, s, v, v.sEy[t], v.sC[t]);
        hipLaunchKernelGGL(sep_points_to_cols, dim3((v.Ny + 255) / 256, nqx), dim3(256), 0, s, v, v.sEy[t]);
        hipLaunchKernelGGL(sep_points_to_rows, dim3((v.Ny + 255) / 256, v.Nx), dim3(256), 0, s, v, v.sEx[t], Y, ldy,
                           (v.element_terms || t > 0) ? 1 : 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

int dot_parts() { return kDotBlocks; }

hipError_t launch_multidot(const double* a, const MultiB& bs, long n, double* part, double* out, hipStream_t s) {
    if (bs.nb < 1 || bs.nb > 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(multidot_kernel, dim3(kDotBlocks), dim3(256), 0, s, a, bs, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finish_dot_kernel, dim3(1), dim3(256), 0, s, part, kDotBlocks, bs.nb, out);
    return hipGetLastError();
}

hipError_t launch_axpys(double* y, const MultiB& xs, const Coefs& c, long n, hipStream_t s) {
    if (xs.nb < 1 || xs.nb > 4) return hipErrorInvalidValue;
    const long blocks = std::min<long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(axpys_kernel, dim3((unsigned)blocks), dim3(256), 0, s, y, xs, c, n);
    return hipGetLastError();
}

hipError_t launch_xpby(double* y, const double* x, double beta, long n, hipStream_t s) {
    const long blocks = std::min<long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(xpby_kernel, dim3((unsigned)blocks), dim3(256), 0, s, y, x, beta, n);
    return hipGetLastError();
}

hipError_t launch_copy2d(const double* x, long ldx, double* y, long ldy, int rows, int cols, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy2d_kernel, dim3((cols + 255) / 256, rows), dim3(256), 0, s, x, ldx, y, ldy, cols);
    return hipGetLastError();
}

}  // namespace hpadi
