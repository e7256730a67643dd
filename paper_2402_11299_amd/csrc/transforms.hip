// Per-element dense passes of the grid transforms (Sec. 6).
//
// Every map between grid values, piecewise Legendre coefficients and the hat+bubble basis
// acts element by element along one axis with one small dense matrix shared by all
// elements (the reference-element transform, or the evaluation of the local basis or of its
// derivative at the reference points).  One pass applies such a matrix along x (a row pass:
// every column of the array is an independent line) or along y (a column pass: every row
// is one).  Per workgroup and element this is a small dense product, out (M x 64 lines) =
// Mat (M x L) . in (L x 64 lines), run on the matrix cores in FP64
// (v_mfma_f64_16x16x4f64): the inputs of 64 lines are staged in LDS with coalesced loads,
// wave w owns the output rows 16 w .. 16 w + 15 and streams its fragments of Mat from a
// precomputed fragment-ordered table (L2-resident), four 16 x 16 accumulator tiles cover
// the 64 lines.  On MI355X the FP64 matrix rate equals the FP64 vector rate; the matrix
// cores are used because they take both operands from registers, where a vector FMA
// kernel would need one table entry per FMA broadcast through the scalar cache.
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
    const int v = e + l;  // vertex of the local hat; bc is the hat mask (bit 0 vertex 0, bit 1 vertex n)
    const int first = (a.bc & 1) ? 0 : 1, last = (a.bc & 2) ? a.n : a.n - 1;
    return (v >= first && v <= last) ? v - first : -1;
}


typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kLines = 64;     // lines per workgroup (32-line tiles, twice the resident workgroups,
                               // measured slower: 0.240 against 0.209 ms per 2D transform at 4160^2)
constexpr int kCT = kLines / 16;  // 16-line accumulator tiles per wave
constexpr int kStride = kLines + 1;  // LDS row stride (doubles): odd, so that walking a tile column
                               // (consecutive l of one line) spreads over the banks
constexpr int kBatch = 24;     // loads in flight per thread while staging (one batch covers a tile)
constexpr int kMaxKsteps = 60; // L <= 240

// Column passes: the 64 items of a workgroup are R rows x E consecutive elements.
__device__ __forceinline__ int col_tile_E(int n) { return n < kLines ? n : kLines; }

// Accumulator layout of v_mfma_f64_16x16x4f64 (checked on the device): register r of lane
// holds row (lane / 16) + 4 r, column lane % 16; operand A is read at (lane % 16, lane / 16)
// and B at (lane / 16, lane % 16).
template <int KS, bool ROWS, bool BURG>
__global__ void __launch_bounds__(1024) elem_pass_kernel(ElemPass a) {
    extern __shared__ double tile[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nt = blockDim.x;
    const int L = a.L, S = a.ksteps, Lpad = 4 * S;
    const double* __restrict__ in = a.in;
    int e = 0, c0 = 0, r0 = 0, e0 = 0, En = 0, E = 1, rows = 0;
    if (ROWS) {
        e = blockIdx.y;
        c0 = blockIdx.x * kLines;
    } else {
        E = col_tile_E(a.ain.n);
        const int R = kLines / E;
        e0 = blockIdx.y * E;
        En = min(E, a.ain.n - e0);
        r0 = blockIdx.x * R;
        rows = min(R, a.lines - r0);
    }
    // ---- stage the inputs: tile[l][line], rows L..Lpad-1 zero
    int total;
    if (ROWS) total = L * kLines;
    else total = rows * En * L;
    for (int base = threadIdx.x; base < total; base += nt * kBatch) {
        double v[kBatch];
        int dst[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int idx = base + b * nt;
            v[b] = 0.0;
            dst[b] = -1;
            if (idx < total) {
                long src = -1;
                if (ROWS) {
                    const int l = idx / kLines, j = idx % kLines;
                    const int r = local_index(a.ain, e, l);
                    dst[b] = l * kStride + j;
                    if (r >= 0 && c0 + j < a.lines) src = (long)r * a.ldin + c0 + j;
                } else if (a.ain.layout == AX_VALUES) {
                    // a row's segment of En elements is contiguous: walk it in address order
                    const int seg = En * L;
                    const int rl = idx / seg, rem = idx - rl * seg;
                    const int el = rem / L, l = rem - el * L;
                    dst[b] = l * kStride + rl * E + el;
                    src = (long)(r0 + rl) * a.ldin + (long)(e0 + el) * L + l;
                } else {
                    // degree- or basis-major: consecutive elements are contiguous for a fixed l
                    const int el = idx % En, t = idx / En;
                    const int l = t % L, rl = t / L;
                    const int gi = local_index(a.ain, e0 + el, l);
                    dst[b] = l * kStride + rl * E + el;
                    if (gi >= 0) src = (long)(r0 + rl) * a.ldin + gi;
                }
                if (src >= 0) v[b] = in[src];
            }
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
            if (dst[b] >= 0) tile[dst[b]] = v[b];
    }
    // the padded rows L..Lpad-1 meet zero table entries and must hold finite values (lines
    // past a tile's items only feed their own, unstored, output columns)
    for (int idx = threadIdx.x; idx < (Lpad - L) * kLines; idx += nt)
        tile[(L + idx / kLines) * kStride + idx % kLines] = 0.0;
    __syncthreads();
    // ---- rows 16 w .. 16 w + 15 of the outputs for the 64 lines
    const int kr = lane >> 4, jc = lane & 15;
    // this wave's operand fragments of the matrix: in registers for the whole product when
    // KS > 0 (the loop is unrolled), else streamed from the L2-resident table
    const double* __restrict__ tf = a.tab + (long)w * S * 64 + lane;
    const double* __restrict__ tf2 = BURG ? a.tab2 + (long)w * S * 64 + lane : nullptr;
    double4_t acc[kCT], acc2[BURG ? kCT : 1];
#pragma unroll
    for (int ct = 0; ct < kCT; ++ct) {
        acc[ct] = double4_t{0.0, 0.0, 0.0, 0.0};
        if (BURG) acc2[ct] = double4_t{0.0, 0.0, 0.0, 0.0};
    }
    if (KS > 0) {
        double af[KS > 0 ? KS : 1];
#pragma unroll
        for (int s = 0; s < KS; ++s) af[s] = s < S ? tf[s * 64] : 0.0;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (s < S) {  // uniform
                const double* brow = tile + (4 * s + kr) * kStride + jc;
#pragma unroll
                for (int ct = 0; ct < kCT; ++ct)
                    acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s], brow[16 * ct], acc[ct], 0, 0, 0);
            }
        }
    } else {
        for (int s = 0; s < S; ++s) {
            const double av = tf[s * 64];
            const double av2 = BURG ? tf2[s * 64] : 0.0;
            const double* brow = tile + (4 * s + kr) * kStride + jc;
#pragma unroll
            for (int ct = 0; ct < kCT; ++ct) {
                const double bv = brow[16 * ct];
                acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[ct], 0, 0, 0);
                if (BURG) acc2[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av2, bv, acc2[ct], 0, 0, 0);
            }
        }
    }
    // ---- tail rows 16 nwaves .. M - 1 (at most 4, when M = 16 nwaves + tail): vector FMAs
    // in the first kCT waves, wave w for lines 16 w .. 16 w + 15, each 16-lane group of
    // it a quarter of the inputs, the quarters summed by cross-lane adds.  This keeps one
    // wave per SIMD where a padded wave would add a fifth for a single output row.
    const int T = a.tail, i0t = 16 * a.nwaves;
    double tv[4] = {0.0, 0.0, 0.0, 0.0}, tv2[4] = {0.0, 0.0, 0.0, 0.0};
    if (T > 0 && w < kCT) {
        const int line = 16 * w + jc;
        for (int l = kr; l < L; l += 4) {
            const double x = tile[l * kStride + line];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t < T) {
                    tv[t] = fma(a.ttab[t * L + l], x, tv[t]);
                    if (BURG) tv2[t] = fma(a.ttab2[t * L + l], x, tv2[t]);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            tv[t] += __shfl_xor(tv[t], 16, 64);
            tv[t] += __shfl_xor(tv[t], 32, 64);
            if (BURG) {
                tv2[t] += __shfl_xor(tv2[t], 16, 64);
                tv2[t] += __shfl_xor(tv2[t], 32, 64);
            }
        }
    }
    const bool tail_lane = T > 0 && w < kCT && kr == 0;  // stores the tail rows of line 16 w + jc
    // ---- results: output row i = 16 w + kr + 4 r, line 16 ct + jc
    if (ROWS) {
        const double sc = a.scale ? a.scale[e] : 1.0;
        const double s2 = BURG ? a.scale2[e] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + kr + 4 * r;
            if (i >= a.M) continue;
            double* orow = a.out + (long)local_index(a.aout, e, i) * a.ldout + c0;
#pragma unroll
            for (int ct = 0; ct < kCT; ++ct) {
                const int j = 16 * ct + jc;
                if (c0 + j >= a.lines) continue;
                double v = acc[ct][r] * sc;
                if (BURG) v = v - a.dt * (acc2[ct][r] * s2) * v;
                orow[j] = v;
            }
        }
        if (tail_lane && c0 + 16 * w + jc < a.lines) {
            for (int t = 0; t < T; ++t) {
                double v = tv[t] * sc;
                if (BURG) v = v - a.dt * (tv2[t] * s2) * v;
                a.out[(long)local_index(a.aout, e, i0t + t) * a.ldout + c0 + 16 * w + jc] = v;
            }
        }
        return;
    }
    if (a.aout.layout != AX_VALUES) {
#pragma unroll
        for (int ct = 0; ct < kCT; ++ct) {
            const int j = 16 * ct + jc;
            const int rl = j / E, el = j - rl * E;
            if (rl >= rows || el >= En) continue;
            const double sc = a.scale ? a.scale[e0 + el] : 1.0;
            double* orow = a.out + (long)(r0 + rl) * a.ldout;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * w + kr + 4 * r;
                if (i < a.M) orow[local_index(a.aout, e0 + el, i)] = acc[ct][r] * sc;
            }
        }
        if (tail_lane) {
            const int j = 16 * w + jc;
            const int rl = j / E, el = j - rl * E;
            if (rl < rows && el < En) {
                const double sc = a.scale ? a.scale[e0 + el] : 1.0;
                double* orow = a.out + (long)(r0 + rl) * a.ldout;
                for (int t = 0; t < T; ++t) orow[local_index(a.aout, e0 + el, i0t + t)] = tv[t] * sc;
            }
        }
        return;
    }
    // element-major outputs: through the tile, then stored in address order
    __syncthreads();  // every wave has read its inputs
#pragma unroll
    for (int ct = 0; ct < kCT; ++ct) {
        const int j = 16 * ct + jc;
        const int rl = j / E, el = j - rl * E;
        const double sc = (a.scale && rl < rows && el < En) ? a.scale[e0 + el] : 1.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + kr + 4 * r;
            if (i < a.M) tile[i * kStride + j] = acc[ct][r] * sc;
        }
    }
    if (tail_lane) {
        const int j = 16 * w + jc;
        const int rl = j / E, el = j - rl * E;
        const double sc = (a.scale && rl < rows && el < En) ? a.scale[e0 + el] : 1.0;
        for (int t = 0; t < T; ++t) tile[(i0t + t) * kStride + j] = tv[t] * sc;
    }
    __syncthreads();
    const int M = a.M, seg = En * M;
    for (int idx = threadIdx.x; idx < rows * seg; idx += nt) {
        const int rl = idx / seg, rem = idx - rl * seg;
        const int el = rem / M, i = rem - el * M;
        a.out[(long)(r0 + rl) * a.ldout + (long)(e0 + el) * M + i] = tile[i * kStride + rl * E + el];
    }
}

// LDS of a pass: the staged inputs (4 ksteps rows), or the M output rows when a column pass
// stores element-major values through the tile.
size_t pass_lds(const ElemPass& a, bool rows_pass) {
    int rows = 4 * a.ksteps;
    if (!rows_pass && a.aout.layout == AX_VALUES && a.M > rows) rows = a.M;
    return (size_t)rows * kStride * sizeof(double);
}

template <int KS, bool ROWS>
hipError_t launch_ks(const ElemPass& a, hipStream_t s) {
    const int n = a.ain.n;
    dim3 grid;
    if (ROWS) {
        grid = dim3((unsigned)((a.lines + kLines - 1) / kLines), (unsigned)n);
    } else {
        const int E = n < kLines ? n : kLines, R = kLines / E;
        grid = dim3((unsigned)((a.lines + R - 1) / R), (unsigned)((n + E - 1) / E));
    }
    const dim3 block((unsigned)(64 * a.nwaves));
    if (ROWS && a.tab2)  // two products: fragments streamed (registers would spill)
        hipLaunchKernelGGL((elem_pass_kernel<0, true, true>), grid, block, pass_lds(a, ROWS), s, a);
    else if (ROWS)
        hipLaunchKernelGGL((elem_pass_kernel<KS, true, false>), grid, block, pass_lds(a, ROWS), s, a);
    else
        hipLaunchKernelGGL((elem_pass_kernel<KS, false, false>), grid, block, pass_lds(a, ROWS), s, a);
    return hipGetLastError();
}

template <bool ROWS>
hipError_t launch_pass(const ElemPass& a, hipStream_t s) {
    if (a.lines <= 0 || a.ain.n <= 0) return hipSuccess;
    const bool tail_ok = a.tail == 0 || (a.tail <= 4 && a.nwaves >= 4 && a.ttab && (!a.tab2 || a.ttab2));
    if ((!ROWS && a.tab2) || a.nwaves < 1 || 16 * a.nwaves + a.tail < a.M || a.nwaves > 16 || !tail_ok ||
        a.ksteps < 1 || 4 * a.ksteps < a.L || a.ksteps > kMaxKsteps || pass_lds(a, ROWS) > 160 * 1024 ||
        a.ain.n != a.aout.n)
        return hipErrorInvalidValue;
    // the k-steps of the product, rounded up to a compiled count (fragments in registers),
    // or streamed beyond 33
    if (a.ksteps <= 4) return launch_ks<4, ROWS>(a, s);
    if (a.ksteps <= 9) return launch_ks<9, ROWS>(a, s);
    if (a.ksteps <= 17) return launch_ks<17, ROWS>(a, s);
    if (a.ksteps <= 33) return launch_ks<33, ROWS>(a, s);
    return launch_ks<0, ROWS>(a, s);
}

}  // namespace

int elem_max_outputs() { return 240; }

hipError_t launch_elem_rows(const ElemPass& a, hipStream_t s) { return launch_pass<true>(a, s); }

hipError_t launch_elem_cols(const ElemPass& a, hipStream_t s) { return launch_pass<false>(a, s); }

}  // namespace hpadi
