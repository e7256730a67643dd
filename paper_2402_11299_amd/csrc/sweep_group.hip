// Grouped launches of the uniform-mesh half-sweep: one launch runs the same kind of
// half-sweep for many independent problems (a batch), each workgroup finding its
// problem in a device task table by binary search over the first workgroup of each
// task.  The per-problem work is the body in sweep_uni_body.h.

#include <hip/hip_runtime.h>

#include "internal.h"
#include "sweep_common.h"
#include "sweep_uni_body.h"

namespace hpadi {

using namespace sweep_detail;

namespace {

// Many problems in one launch: task k owns workgroups [block0_k, block0_k + nblk_k).
template <typename TIN, typename TOUT, int CL, int MODE, bool COL, int LW>
__global__ void __launch_bounds__(sweep_max_threads(CL)) sweep_uni_grouped_kernel(const GroupTask* __restrict__ t,
                                                                                   int nt) {
    const int b = blockIdx.x;
    int lo = 0, hi = nt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    sweep_uni_body<TIN, TOUT, CL, MODE, COL, LW>(t[lo].d, t[lo].a, b - t[lo].block0, t[lo].nblk, false);
}

template <typename TIN, typename TOUT, int CL, int MODE, bool COL, int LW>
hipError_t launch_g(const GroupLaunch& g, hipStream_t s) {
    hipLaunchKernelGGL((sweep_uni_grouped_kernel<TIN, TOUT, CL, MODE, COL, LW>), dim3(g.nblocks), dim3(g.threads),
                       g.lds_bytes, s, g.tasks, g.ntasks);
    return hipGetLastError();
}

template <typename TIN, typename TOUT, int MODE>
hipError_t group_by_cl(const GroupLaunch& g, hipStream_t s) {
#define HPADI_G(CLV)                                                                                          \
    if (g.cl == CLV) {                                                                                        \
        if (g.lw == 4) return g.column ? launch_g<TIN, TOUT, CLV, MODE, true, 4>(g, s)                        \
                                       : launch_g<TIN, TOUT, CLV, MODE, false, 4>(g, s);                      \
        if (g.lw == 8) return g.column ? launch_g<TIN, TOUT, CLV, MODE, true, 8>(g, s)                        \
                                       : launch_g<TIN, TOUT, CLV, MODE, false, 8>(g, s);                      \
        if (g.lw == 16) return g.column ? launch_g<TIN, TOUT, CLV, MODE, true, 16>(g, s)                      \
                                        : launch_g<TIN, TOUT, CLV, MODE, false, 16>(g, s);                    \
        return hipErrorInvalidValue;                                                                          \
    }
    HPADI_G(4)
    HPADI_G(8)
    HPADI_G(16)
    HPADI_G(32)
    HPADI_G(64)
#undef HPADI_G
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_sweep_uni_grouped(const GroupLaunch& g, hipStream_t s) {
    if (g.ntasks <= 0 || g.nblocks <= 0) return hipSuccess;
    switch (g.mode) {
        case SWEEP_FULL:
            if (g.tin == 4 && g.tout == 4) return group_by_cl<float, float, SWEEP_FULL>(g, s);
            if (g.tin == 8 && g.tout == 8) return group_by_cl<double, double, SWEEP_FULL>(g, s);
            break;
        case SWEEP_SOLVE:
            if (g.tin == 4 && g.tout == 4) return group_by_cl<float, float, SWEEP_SOLVE>(g, s);
            if (g.tin == 8 && g.tout == 8) return group_by_cl<double, double, SWEEP_SOLVE>(g, s);
            break;
        case SWEEP_TRANSFORM:
            if (g.tin == 8 && g.tout == 8) return group_by_cl<double, double, SWEEP_TRANSFORM>(g, s);
            if (g.tin == 8 && g.tout == 4) return group_by_cl<double, float, SWEEP_TRANSFORM>(g, s);
            break;
        case SWEEP_FINAL:
            if (g.tin == 4 && g.tout == 8) return group_by_cl<float, double, SWEEP_FINAL>(g, s);
            if (g.tin == 8 && g.tout == 8) return group_by_cl<double, double, SWEEP_FINAL>(g, s);
            break;
        default:
            break;
    }
    return hipErrorInvalidValue;
}

}  // namespace hpadi
