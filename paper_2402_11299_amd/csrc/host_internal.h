// Host-side state shared by the host sources of hpadi: 1D operators and plans.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "hpadi.h"
#include "internal.h"

// 1D operator (Sec. 2.2-2.3, App. A): mesh, degree and boundary condition.
// Boundary conditions per end (Sec. 3.3): Dirichlet drops the end's hat; Neumann keeps it;
// Robin keeps it and adds alpha to its stiffness diagonal.
struct hpadi_op1d_s {
    int n, p, bc, nh, N, Nleg;      // bc: hat mask (bit 0 vertex 0, bit 1 vertex n)
    int kind[2] = {HPADI_DIRICHLET, HPADI_DIRICHLET};
    double alpha[2] = {0.0, 0.0};   // Robin coefficients (0 unless Robin)
    std::vector<double> x, delta;

    int first_hat_vertex() const { return (bc & 1) ? 0 : 1; }
    bool vertex_is_hat(int v) const { return v >= first_hat_vertex() && v <= ((bc & 2) ? n : n - 1); }
    int hat_of_vertex(int v) const { return v - first_hat_vertex(); }
    int vertex_of_hat(int h) const { return h + first_hat_vertex(); }
    int bubble(int m, int e) const { return nh + m * n + e; }
    // alpha of the end at vertex v (0 for interior vertices and non-Robin ends)
    double robin(int v) const { return (v == 0 ? alpha[0] : 0.0) + (v == n ? alpha[1] : 0.0); }
    // K has a null space (the constants) only with Neumann conditions at both ends
    bool k_singular() const { return bc == 3 && alpha[0] == 0.0 && alpha[1] == 0.0; }
};

// One axis of a plan: the operator and its device-side description.
struct DimHost {
    hpadi_op1d_s op;
    hpadi::DimDev dev{};
    double* buf = nullptr;  // device: delta, invdelta, mdiag, tab64
    float* tab32 = nullptr;
    int hpad = 0;           // hats padded to a multiple of 8 (internal layout)
    int Npad = 0;           // internal length: hpad + (p-1) n
    bool uniform = false;   // all elements of equal width and n % 4 == 0 (per-degree coefficient fast path)
};

// One shift family of Alg. 2: the J shift pairs for a tolerance and the reverse
// Cholesky factors of the shifted 1D operators (plus the mass matrices) on the device.
struct ShiftFamily {
    int J = 0;
    double eps = 0.0;             // tolerance the shifts were built for
    std::vector<double> P, Q;
    bool shared = false;          // x and y use one factor family
    double* facx64 = nullptr;     // J+1 records: K_x + (w/2 - q_j) M_x, then M_x
    double* facy64 = nullptr;     // J+1 records: K_y + (w/2 + p_j) M_y, then M_y
    double* coefx = nullptr;      // uniform meshes: (J+1) (p_x-1) 8 per-degree coefficient records
    double* coefy = nullptr;
    double* ptabx = nullptr;      // uniform meshes: J folded per-pass tables (p_x records of 16 doubles)
    double* ptaby = nullptr;
    int* status = nullptr;
};

struct hpadi_plan_s {
    DimHost dx, dy;
    double omega2 = 0.0, tol = 0.0;
    // A_x = kx K_x + sx M_x, A_y = ky K_y + sy M_y (kx = ky = 1, sx = sy = omega2 / 2 for the
    // screened Poisson problem): Alg. 2 with A = A_x, D = M_x, C = M_y, B = -A_y
    double kx = 1.0, sx = 0.0, ky = 1.0, sy = 0.0;
    int precision = HPADI_FP64;
    hpadi_options opt{};
    double interval[4] = {0, 0, 0, 0};
    // fam[0]: the family of an FP64 plan, or of the FP32 rounds of a mixed plan;
    // fam[iref]: the family of the first FP64 refinement round of a mixed plan; further
    // (looser) families are built on first use for later rounds (ladder_family)
    static constexpr int kMaxFam = 8;
    ShiftFamily fam[kMaxFam];
    int nfam = 1;
    int iref = 0;
    int lpb_col = 8, lpb_row = 8; // lines per workgroup of the column / row half-sweeps
    hipStream_t stream = nullptr;
    hpadi::FactorLayout flx{}, fly{};
    const ShiftFamily& first() const { return fam[0]; }
    const ShiftFamily& refine() const { return fam[iref]; }
    // work arrays in the internal panel layout
    hpadi::Layout lint{};
    size_t nint = 0;              // elements per internal array
    void* Wk = nullptr;           // balanced iterate (TS)
    void* Gt = nullptr;           // balanced right-hand side G~ (TS)
    double* T64 = nullptr;        // transform temporary (FP64, internal layout)
    // FP64 row-major work (mixed refinement, apply)
    long ldw = 0;
    double* T12 = nullptr;        // row products U M_y, U A_y as interleaved pairs
    double* R64 = nullptr;
    double* H = nullptr;          // load temporary (Nleg_x x N_y)
    long ldh = 0;
    double* acc = nullptr;        // device accumulators
    double* part = nullptr;       // per-block partial sums of the residual's norms
    double* acc_host = nullptr;   // pinned host copy
    // measurement
    std::vector<hipEvent_t> phase_ev;  // per-round events of a mixed solve (stats t_ms)
    bool timing = false;
    struct Rec { hipEvent_t a, b; int kind; double bytes; };
    std::vector<Rec> recs;        // event pool; the first nrec are in use
    size_t nrec = 0;
};

namespace hpadi {
// out[2 i + k] = accs[i][k], k = 0, 1 (gathers the plans' norm accumulators of a batch)
hipError_t launch_gather_acc(const double* const* accs, int count, double* out, hipStream_t s);
// accs[i][0] = accs[i][1] = 0 for i < count (the norm accumulators of a batch's plans)
hipError_t launch_zero_accs(double* const* accs, int count, hipStream_t s);
}  // namespace hpadi

namespace hpadi_host {

template <typename T>
hipError_t dmalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) return hipSuccess;
    return hipMalloc((void**)p, count * sizeof(T));
}

}  // namespace hpadi_host
