// Per-element dense passes of the grid transforms (Sec. 6).
//
// Every map between grid values, piecewise Legendre coefficients and the hat+bubble basis
// acts element by element along one axis with one small dense matrix shared by all
// elements (the reference-element transform, or the evaluation of the local basis or of its
// derivative at the reference points).  One pass applies such a matrix along x (a row pass:
// every column of the array is an independent line) or along y (a column pass: every row
// is one).  A lane owns one line of one element and keeps a chunk of up to RB outputs in
// registers; the matrix entries are the same for every lane of the workgroup and come
// through the scalar cache, so the inner loop is one vector load and RB FMAs per input.
// Row passes read and write whole rows (coalesced); column passes have the lanes of a wave
// on consecutive elements of a row, which makes Legendre- and Q-ordered accesses contiguous
// and leaves the element-major value accesses strided by the points per element (their
// cache lines are used over consecutive inputs).  FP64 throughout.
//
// The paper composes a DCT with a fast Chebyshev-Legendre transform; at the degrees used
// here (p <= 128) the dense per-element product costs 2 (p+1) flops per output, about what
// the memory traffic of the pass costs, so the fast transform would not be faster.

#include <hip/hip_runtime.h>

#include "transforms.h"

namespace hpadi {

namespace {

__device__ __forceinline__ int local_index(const AxisMap& a, int e, int l) {
    if (a.layout == AX_VALUES) return e * a.m + l;
    if (a.layout == AX_LEGENDRE) return l * a.n + e;
    if (l >= 2) return a.nh + (l - 2) * a.n + e;
    const int v = e + l;  // vertex of the local hat
    if (a.bc == 0) return (v >= 1 && v <= a.n - 1) ? v - 1 : -1;
    return v;
}

// Block b of a launch of 8 k nchunks workgroups along x: the nchunks chunks of one tile
// run on one XCD (workgroups are dealt to the 8 XCDs round robin), so a tile's input is
// read from HBM once and reused from that XCD's L2.
__device__ __forceinline__ void tile_and_chunk(int nchunks, int& tile, int& chunk) {
    const int b = blockIdx.x;
    const int slot = b >> 3;
    chunk = slot % nchunks;
    tile = (slot / nchunks) * 8 + (b & 7);
}

template <int RB, bool BURG>
__global__ void __launch_bounds__(256) elem_rows_kernel(ElemPass a, int ntiles) {
    int tile, chunk;
    tile_and_chunk(a.nchunks, tile, chunk);
    if (tile >= ntiles) return;
    const int e = blockIdx.y;
    const int c = tile * 256 + threadIdx.x;
    const bool act = c < a.lines;
    const double* __restrict__ in = a.in;
    const double* __restrict__ tab = a.tab + (long)chunk * a.L * RB;
    const double* __restrict__ tab2 = BURG ? a.tab2 + (long)chunk * a.L * RB : nullptr;
    double acc[RB], acc2[BURG ? RB : 1];
#pragma unroll
    for (int k = 0; k < RB; ++k) acc[k] = 0.0;
    if (BURG) {
#pragma unroll
        for (int k = 0; k < RB; ++k) acc2[k] = 0.0;
    }
    for (int l = 0; l < a.L; ++l) {
        const int r = local_index(a.ain, e, l);
        double x = 0.0;
        if (r >= 0 && act) x = in[(long)r * a.ldin + c];
        const double* t = tab + l * RB;
#pragma unroll
        for (int k = 0; k < RB; ++k) acc[k] = fma(t[k], x, acc[k]);
        if (BURG) {
            const double* t2 = tab2 + l * RB;
#pragma unroll
            for (int k = 0; k < RB; ++k) acc2[k] = fma(t2[k], x, acc2[k]);
        }
    }
    if (!act) return;
    const double s = a.scale ? a.scale[e] : 1.0;
    const double s2 = BURG ? a.scale2[e] : 0.0;
#pragma unroll
    for (int k = 0; k < RB; ++k) {
        const int i = chunk * RB + k;
        if (i < a.M) {
            double v = acc[k] * s;
            if (BURG) v = v - a.dt * (acc2[k] * s2) * v;
            a.out[(long)local_index(a.aout, e, i) * a.ldout + c] = v;
        }
    }
}

template <int RB>
__global__ void __launch_bounds__(256) elem_cols_kernel(ElemPass a, int ntiles) {
    int tile, chunk;
    tile_and_chunk(a.nchunks, tile, chunk);
    if (tile >= ntiles) return;
    const int n = a.ain.n;
    const long item = (long)tile * 256 + threadIdx.x;
    const long r = item / n;
    const int e = (int)(item - r * n);
    const bool act = r < a.lines;
    const double* __restrict__ row = a.in + (act ? r : 0) * a.ldin;
    const double* __restrict__ tab = a.tab + (long)chunk * a.L * RB;
    double acc[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) acc[k] = 0.0;
    for (int l = 0; l < a.L; ++l) {
        const int idx = local_index(a.ain, e, l);
        const double x = (idx >= 0 && act) ? row[idx] : 0.0;
        const double* t = tab + l * RB;
#pragma unroll
        for (int k = 0; k < RB; ++k) acc[k] = fma(t[k], x, acc[k]);
    }
    if (!act) return;
    const double s = a.scale ? a.scale[e] : 1.0;
    double* orow = a.out + r * a.ldout;
#pragma unroll
    for (int k = 0; k < RB; ++k) {
        const int i = chunk * RB + k;
        if (i < a.M) orow[local_index(a.aout, e, i)] = acc[k] * s;
    }
}

template <int RB>
hipError_t rows_rb(const ElemPass& a, hipStream_t s) {
    const int ntiles = (a.lines + 255) / 256;
    const dim3 grid((unsigned)((ntiles + 7) / 8 * 8 * a.nchunks), (unsigned)a.ain.n);
    if (a.tab2)
        hipLaunchKernelGGL((elem_rows_kernel<RB, true>), grid, dim3(256), 0, s, a, ntiles);
    else
        hipLaunchKernelGGL((elem_rows_kernel<RB, false>), grid, dim3(256), 0, s, a, ntiles);
    return hipGetLastError();
}

template <int RB>
hipError_t cols_rb(const ElemPass& a, hipStream_t s) {
    const long items = (long)a.lines * a.ain.n;
    const int ntiles = (int)((items + 255) / 256);
    const dim3 grid((unsigned)((ntiles + 7) / 8 * 8 * a.nchunks));
    hipLaunchKernelGGL((elem_cols_kernel<RB>), grid, dim3(256), 0, s, a, ntiles);
    return hipGetLastError();
}

}  // namespace

int elem_chunk(int M) { return M <= 8 ? 8 : (M <= 16 ? 16 : 33); }

hipError_t launch_elem_rows(const ElemPass& a, hipStream_t s) {
    if (a.lines <= 0 || a.ain.n <= 0) return hipSuccess;
    switch (a.rb) {
        case 8: return rows_rb<8>(a, s);
        case 16: return rows_rb<16>(a, s);
        case 33: return rows_rb<33>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_elem_cols(const ElemPass& a, hipStream_t s) {
    if (a.lines <= 0 || a.ain.n <= 0) return hipSuccess;
    if (a.tab2) return hipErrorInvalidValue;
    switch (a.rb) {
        case 8: return cols_rb<8>(a, s);
        case 16: return cols_rb<16>(a, s);
        case 33: return cols_rb<33>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hpadi
