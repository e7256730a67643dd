// Uniform-mesh fast path of the mass-balanced half-sweeps: launch wrappers for one
// problem per launch (the body is in sweep_uni_body.h; grouped launches of many
// problems are in sweep_group.hip).

#include <hip/hip_runtime.h>

#include "internal.h"
#include "sweep_common.h"
#include "sweep_uni_body.h"

namespace hpadi {

using namespace sweep_detail;

namespace {

template <typename TIN, typename TOUT, int CL, int MODE, bool COL, int LW>
__global__ void __launch_bounds__(sweep_max_threads(CL)) sweep_uni_kernel(DimDev d, SweepArgs a) {
    sweep_uni_body<TIN, TOUT, CL, MODE, COL, LW>(d, a, blockIdx.x, gridDim.x, true);
}

template <typename TIN, typename TOUT, int CL, int MODE, bool COL, int LW>
hipError_t launch_u(const DimDev& d, const SweepArgs& a, hipStream_t s) {
    constexpr int CW = 64 / LW;
    const int threads = 64 * ((2 * d.n + CW - 1) / CW);
    if (threads > sweep_max_threads(CL) || d.nh > 65) return hipErrorInvalidValue;
    const int blocks = (a.hpad_lines + a.nlines - a.nh_lines + LW - 1) / LW;
    // LDS: per line A, B (hats) and H1, H2 (chain heads), then the two hat factors
    const int hs = d.nh + 1;
    size_t words = (size_t)LW * (2 * hs + 4 * d.n) + 2 * (3 * hs + 4 * d.n);
    if (MODE == SWEEP_FINAL && words < (size_t)threads * 2) words = (size_t)threads * 2;
    hipLaunchKernelGGL((sweep_uni_kernel<TIN, TOUT, CL, MODE, COL, LW>), dim3(blocks), dim3(threads),
                       words * sizeof(double), s, d, a);
    return hipGetLastError();
}

template <typename TIN, typename TOUT, int CL, int MODE>
hipError_t by_dir(const DimDev& d, const SweepArgs& a, bool col, hipStream_t s) {
    // one line per workgroup for the ADI half-sweeps only (the transforms keep 8)
    if constexpr (MODE == SWEEP_FULL || MODE == SWEEP_SOLVE) {
        if (a.lpb == 1)
            return col ? launch_u<TIN, TOUT, CL, MODE, true, 1>(d, a, s) : launch_u<TIN, TOUT, CL, MODE, false, 1>(d, a, s);
    }
    if (a.lpb == 4) return col ? launch_u<TIN, TOUT, CL, MODE, true, 4>(d, a, s) : launch_u<TIN, TOUT, CL, MODE, false, 4>(d, a, s);
    if (a.lpb == 16)
        return col ? launch_u<TIN, TOUT, CL, MODE, true, 16>(d, a, s) : launch_u<TIN, TOUT, CL, MODE, false, 16>(d, a, s);
    return col ? launch_u<TIN, TOUT, CL, MODE, true, 8>(d, a, s) : launch_u<TIN, TOUT, CL, MODE, false, 8>(d, a, s);
}

template <typename TIN, typename TOUT, int MODE>
hipError_t by_cl(const DimDev& d, const SweepArgs& a, bool col, hipStream_t s) {
    switch (d.p / 2) {
        case 4: return by_dir<TIN, TOUT, 4, MODE>(d, a, col, s);
        case 8: return by_dir<TIN, TOUT, 8, MODE>(d, a, col, s);
        case 16: return by_dir<TIN, TOUT, 16, MODE>(d, a, col, s);
        case 32: return by_dir<TIN, TOUT, 32, MODE>(d, a, col, s);
        case 64: return by_dir<TIN, TOUT, 64, MODE>(d, a, col, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t sweep_uni_threads(const DimDev& d, int lw) { return 64 * ((2 * d.n + 64 / lw - 1) / (64 / lw)); }

size_t sweep_uni_lds_bytes(const DimDev& d, int lw, int threads, int mode) {
    const int hs = d.nh + 1;
    size_t words = (size_t)lw * (2 * hs + 4 * d.n) + 2 * (3 * hs + 4 * d.n);
    if (mode == SWEEP_FINAL && words < (size_t)threads * 2) words = (size_t)threads * 2;
    return words * sizeof(double);
}

int sweep_uni_max_threads(int cl) { return sweep_max_threads(cl); }

bool sweep_uni_available(const DimDev& d, int lines_per_block) {
    const int cw = 64 / lines_per_block;
    const int cl = d.p / 2;
    return d.n % cw == 0 && (cl == 4 || cl == 8 || cl == 16 || cl == 32 || cl == 64) && d.nh <= 65;
}

hipError_t launch_sweep_uni(const DimDev& d, const SweepArgs& a, int mode, int tin, int tout, bool column,
                            hipStream_t s) {
    switch (mode) {
        case SWEEP_FULL:
            if (tin == 4 && tout == 4) return by_cl<float, float, SWEEP_FULL>(d, a, column, s);
            if (tin == 8 && tout == 8) return by_cl<double, double, SWEEP_FULL>(d, a, column, s);
            break;
        case SWEEP_SOLVE:
            if (tin == 4 && tout == 4) return by_cl<float, float, SWEEP_SOLVE>(d, a, column, s);
            if (tin == 8 && tout == 8) return by_cl<double, double, SWEEP_SOLVE>(d, a, column, s);
            break;
        case SWEEP_TRANSFORM:
            if (tin == 8 && tout == 8) return by_cl<double, double, SWEEP_TRANSFORM>(d, a, column, s);
            if (tin == 8 && tout == 4) return by_cl<double, float, SWEEP_TRANSFORM>(d, a, column, s);
            break;
        case SWEEP_FINAL:
            if (tin == 4 && tout == 8) return by_cl<float, double, SWEEP_FINAL>(d, a, column, s);
            if (tin == 8 && tout == 8) return by_cl<double, double, SWEEP_FINAL>(d, a, column, s);
            break;
        default:
            break;
    }
    return hipErrorInvalidValue;
}

}  // namespace hpadi
