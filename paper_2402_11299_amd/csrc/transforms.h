// Per-element dense passes between grid values, piecewise Legendre coefficients and the
// hat+bubble basis (Sec. 6: the transforms F_p, F_p^{-1} and the conversions R, D).
#pragma once

#include <hip/hip_runtime.h>

namespace hpadi {

// Index layouts of one axis of a 2D array.
enum AxisLayout {
    AX_VALUES = 0,    // grid values, element-major: e m + k (m points per element)
    AX_LEGENDRE = 1,  // piecewise Legendre coefficients, degree-major: k n + e
    AX_Q = 2          // hat+bubble basis: local 0 = hat of vertex e, 1 = hat of vertex e + 1,
                      // 2 + j = bubble W_j of element e (absent Dirichlet boundary hats read 0)
};

struct AxisMap {
    int layout;
    int n;    // elements
    int m;    // entries per element (AX_VALUES)
    int nh;   // hats (AX_Q)
    int bc;   // hat mask (AX_Q): bit 0 vertex 0 carries a hat, bit 1 vertex n
};

// out[line, o(e, i)] = s_e sum_l Mat[i][l] in[line, g(e, l)] along one axis of a
// row-major array, for every element e and output i < M.  The matrix is stored as the A
// operands of v_mfma_f64_16x16x4f64: tab[((w S + s) 64 + lane)] = Mat[16 w + lane % 16]
// [4 s + lane / 16] (zero outside M x L), w < ceil(M / 16), s < ksteps = ceil(L / 4).
// A workgroup of nwaves waves stages the inputs of 64 lines in LDS (max(4 ksteps, 16 nwaves)
// rows of 65 doubles, under 160 KiB).  With tab2 set (Burgers epilogue, row passes only) a
// second matrix scaled per element by scale2[e] gives w = tab2 . in, and the pass stores
// v - dt w v.
struct ElemPass {
    const double* in; long ldin;
    double* out; long ldout;
    AxisMap ain, aout;
    int L, M;              // inputs and outputs per element
    int nwaves, ksteps;    // matrix-core waves (16 output rows each) and ceil(L / 4)
    int tail;              // output rows 16 nwaves .. M - 1 done by vector FMAs (0, or <= 4 with
                           // nwaves >= 4)
    const double* ttab;    // those rows of the matrix, row-major (tail x L)
    const double* ttab2;   // the same of the second matrix (tab2 set)
    const double* tab;
    const double* tab2;    // or NULL
    const double* scale;   // per-element factor of tab (NULL = 1)
    const double* scale2;  // per-element factor of tab2
    double dt;
    int lines;             // independent lines: columns (row pass) or rows (column pass)
};

// The largest M and L a pass takes (the LDS tile bounds them).
int elem_max_outputs();
// Row pass: the transformed axis is x (array rows); lines are columns.
hipError_t launch_elem_rows(const ElemPass& a, hipStream_t s);
// Column pass: the transformed axis is y (array columns); lines are rows.  No tab2.
hipError_t launch_elem_cols(const ElemPass& a, hipStream_t s);

}  // namespace hpadi
