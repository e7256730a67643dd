// Internal declarations shared by the host code and the HIP kernels of hpadi.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace hpadi {

// Device view of one 1D discretisation (Sec. 2.2: mesh, degree, boundary condition).
struct DimDev {
    int n, p, nh, N, Nleg, bc;  // bc: hat mask, bit 0 vertex 0 carries a hat, bit 1 vertex n
                                // (0 Dirichlet at both ends, 3 Neumann or Robin at both)
    double rob0, rob1;          // Robin coefficients of the ends (0 unless Robin): alpha v(x) u(x)
                                // at that end adds alpha to the stiffness diagonal of its hat
    const double* delta;        // element widths, n
    const double* invdelta;     // 1 / delta, n
    const double* mdiag;        // diagonal of M (length N), weights of the error estimate
    const double* tab64;        // per-degree constants, 3 * tabstride (see below)
    const float* tab32;         // FP32 copy
    int tabstride;              // >= p + 4
};
// Per-degree constant tables (m = 0 .. p-2 used), reference-element values of
// the bubble blocks of K and M (App. A via eq. app:1):
//   tab[0*ts + m] = 4 / (2m+3)                       K bubble diagonal * delta
//   tab[1*ts + m] = 2 / ((2m+1)(2m+3)(2m+5))          M bubble diagonal / delta
//   tab[2*ts + m] = -1 / ((2m+3)(2m+5)(2m+7))         M between degrees m, m+2, / delta

// Offsets of one structured factor record (units: elements of the factor type).
struct FactorLayout {
    int nb;         // (p-1) n bubble entries
    int off_invd;   // 1/diag of L at bubble (m, e): index m n + e
    int off_link;   // L[(m,e),(m-2,e)]: index m n + e (0 for m < 2)
    int off_cpl;    // coupling to hats: index 4e + 2 pi + side
    int off_invd0;  // hat factor 1/diag, n_h
    int off_link0;  // hat factor L0[h, h-1], n_h
    int off_d;      // diagonal of L at bubble (m, e) (= 1 / invd), (p-1) n
    int off_d0;     // diagonal of the hat factor L0, n_h
    int size;       // used length
    int stride;     // distance between consecutive records (multiple of 64)
};

inline FactorLayout make_factor_layout(int n, int p, int nh) {
    FactorLayout L;
    L.nb = (p - 1) * n;
    L.off_invd = 0;
    L.off_link = L.nb;
    L.off_cpl = 2 * L.nb;
    L.off_invd0 = 2 * L.nb + 4 * n;
    L.off_link0 = L.off_invd0 + nh;
    L.off_d = L.off_link0 + nh;
    L.off_d0 = L.off_d + L.nb;
    L.size = L.off_d0 + nh;
    L.stride = (L.size + 63) / 64 * 64;
    return L;
}

// Launch helpers implemented in kernels.hip (all asynchronous on `s`).
// Factorise nf matrices kappa[f] K + sigma[f] M of one dimension (Alg. 1).
hipError_t launch_factor(const DimDev& d, int nf, const double* kappa_dev, const double* sigma_dev,
                         double* fac64, float* fac32, int stride, int* status_dev, hipStream_t s);

// Entry (i, j) of an Nx x Ny array: row-major (ptr[i*ld + j]) or the internal
// panel layout of width w (panel j/w at offset (j/w)*ld, row i at w i within it),
// with row/column indices past the hats shifted by offr/offc (alignment padding).
struct Layout {
    long ld;
    int panel;       // 0 row-major; else the panel width (4 or 8 columns)
    int nhr, nhc;    // hats along x (rows) and y (columns)
    int offr, offc;  // padding shift of indices >= nhr / >= nhc
};

// Half-sweeps in mass-balanced coordinates (sweep.hip).
enum SweepMode { SWEEP_FULL = 0, SWEEP_SOLVE = 1, SWEEP_TRANSFORM = 2, SWEEP_FINAL = 3 };
struct SweepArgs {
    const void* in; Layout lin;     // y (FULL, SOLVE), right-hand side (TRANSFORM), w (FINAL)
    const void* g; Layout lg;       // balanced right-hand side G~ (FULL)
    void* out; Layout lout;
    const double* facS;             // factor of the shifted operator (FULL, SOLVE)
    const double* facM;             // factor of this direction's mass matrix
    const double* coef;             // uniform meshes: per-degree coefficient records (8 doubles per m), or NULL
    const double* ptab;             // uniform meshes: folded per-pass records (16 doubles per m), or NULL
    FactorLayout fl;
    double kappa, tau;              // FULL: product kappa K + tau M
    int nlines;                     // lines of the problem
    int nh_lines, hpad_lines;       // hats along the line index, and their padded count
    int accumulate;                 // FINAL: U += u (1) or U = u (0)
    int lpb;                        // lines per workgroup: the panel width of the internal layout (4 or 8)
    int idx32;                      // every array addressed by this sweep has < 2^31 entries
    int xcd_group;                  // row passes: workgroups sharing 128-byte lines (1 = none)
    double* norm_acc;               // SOLVE (column pass): adds |Lm w|^2 over the lines, or NULL
};
hipError_t launch_sweep(const DimDev& d, const SweepArgs& a, int mode, int tin, int tout, bool column,
                        hipStream_t s);
// Per-degree coefficient records for a uniform mesh, for nf shifted factors (records f * stride of
// facS) each paired with the mass factor facM: out[(f p + m) * 8 + k] =
//   S.invd, S.link, M.d, M.link, M.invd (at degree m, element 0), 4/((2m+3) delta),
//   2 delta/((2m+1)(2m+3)(2m+5)), -delta/((2m+3)(2m+5)(2m+7)),
// for m = 0..p-2, and a zero record at m = p-1 (a phantom degree that pads a chain
// one short of the compile-time chain length).
hipError_t launch_coef_tables(const DimDev& d, int nf, const double* facS, int stride, const double* facM,
                              FactorLayout fl, double* out, hipStream_t s);
// Folded per-pass records for the uniform-mesh kernel: for pass f (shifted factor f of
// facS, product tau[f]), out[(f p + m) * 16 + k], m = 0..p-1 (m = p-1 a zero record):
//   0 b1 = M.d(m) S.invd(m)        1 b2 = M.link(m+2) S.invd(m)    2 b3 = -S.link(m+2) S.invd(m)
//   3 c1 = S.invd(m)               4 c2 = -S.link(m) S.invd(m)
//   5 a1 = M.invd(m) (kappa K_mm + tau M_mm)   6 a2 = M.invd(m) tau M_{m-2,m}
//   7 a3 = M.invd(m) tau M_{m,m+2}             8 a4 = -M.invd(m) M.link(m+2)
//   9 f1 = M.invd(m)               10 f2 = -M.link(m) M.invd(m)   11 t2 = -M.link(m+2) M.invd(m)
//   12 M.invd(m) tau delta (head term), 13 M_mm (diagonal of M), 14..15 unused.
hipError_t launch_pass_tables(const DimDev& d, int nf, const double* facS, int stride, const double* facM,
                              FactorLayout fl, const double* tau_dev, double kappa, double* out, hipStream_t s);
int sweep_threads(int n, int lines_per_block);
// Uniform-mesh fast path (sweep_uni.hip): usable when the mesh is uniform (coef != NULL),
// n is a multiple of the chains per wavefront and p/2 is one of 4, 8, 16, 32, 64.
bool sweep_uni_available(const DimDev& d, int lines_per_block);
// Grouped launches of the uniform-mesh kernel: one launch runs the same half-sweep kind
// (mode, types, direction, chain length, lines per workgroup) for many problems.
struct GroupTask {
    DimDev d;
    SweepArgs a;
    int block0;   // first workgroup of this task
    int nblk;     // its workgroups
};
struct GroupLaunch {
    const GroupTask* tasks;  // device table, sorted by block0
    int ntasks, nblocks, threads;
    size_t lds_bytes;
    int mode, tin, tout, cl, lw;
    bool column;
};
size_t sweep_uni_threads(const DimDev& d, int lw);
size_t sweep_uni_lds_bytes(const DimDev& d, int lw, int threads, int mode);
int sweep_uni_max_threads(int cl);
hipError_t launch_sweep_uni_grouped(const GroupLaunch& g, hipStream_t s);
hipError_t launch_sweep_uni(const DimDev& d, const SweepArgs& a, int mode, int tin, int tout, bool column,
                            hipStream_t s);

// Banded operator along lines, elementwise: out = (kappa K + tau M) x per line
// (and optionally a second output with (kappa2, tau2)).  FP64.
struct OpApply {
    const double* in; long in_sl, in_sp;
    double* out1; long o1_sl, o1_sp; double k1, t1;
    double* out2; long o2_sl, o2_sp; double k2, t2;   // out2 may be NULL
    int nlines;
};
hipError_t launch_op_apply(const DimDev& d, const OpApply& a, bool column, hipStream_t s);

// r = G - (A_x T1 + M_x T2) along columns (x direction), FP64 in; writes r as FP64
// (r64, may be NULL) and/or FP32 (r32, may be NULL); accumulates sum w r^2, sum w G^2.
struct Residual {
    const double* G; long g_ld;
    const double* T1; const double* T2; long t_ld;  // T2 NULL: T1 holds (T1, T2) pairs, t_ld pairs
                                                    // per row
    double* r64; long r64_ld;
    float* r32; long r32_ld;
    double ax_k, ax_t;   // A_x = ax_k K + ax_t M
    double alpha, beta;  // r = alpha G + beta (A_x T1 + M_x T2)
    int ncols;
    double* norm_acc;    // [sum w r^2, sum w G^2, <U, M_x T1>] or NULL
    const double* wcol;  // diag of M^y (weights along columns)
    const double* U; long u_ld;  // with T1 = U M_y: <U, M_x U M_y>, the squared norm of U in
                                 // the ADI lemma's norm, into norm_acc[2] (U may be NULL)
    double* partials;            // residual_partials(dx, ncols) doubles for the per-block sums
                                 // (summed by a second small kernel), or NULL: atomics
};
hipError_t launch_residual(const DimDev& dx, const Residual& a, hipStream_t s);
long residual_partials(const DimDev& dx, int ncols);

// G = scale T_x F T_y^T, two elementwise gather passes (Sec. 3.2).
hipError_t launch_load(const DimDev& dx, const DimDev& dy, const double* F, long ldf, double* H,
                       long ldh, double* G, long ldg, hipStream_t s, double scale = 1.0);
// The same for the columns j0 <= j < j0 + ncols of G only; H then holds ncols columns.
hipError_t launch_load_cols(const DimDev& dx, const DimDev& dy, const double* F, long ldf, double* H,
                            long ldh, double* G, long ldg, int j0, int ncols, hipStream_t s,
                            double scale = 1.0);

// Fixed device scratch of the allocation-free load (16 MiB per device, kept until the
// process ends), and the device address of the current device's copy.
constexpr long kLoadScratchWords = 2L * 1024 * 1024;
hipError_t load_scratch(double** out);

// Convert / copy helpers.
hipError_t launch_convert_f64_f32(const double* src, long ld_src, float* dst, long ld_dst, int rows,
                                  int cols, double* norm_acc, const double* wr, const double* wc,
                                  hipStream_t s);
hipError_t launch_zero_f64(double* dst, long ld, int rows, int cols, hipStream_t s);

}  // namespace hpadi
