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
    int bc;   // 0 Dirichlet, 1 Neumann (AX_Q)
};

// out[line, o(e, i)] = s_e sum_l Mat[i][l] in[line, g(e, l)] along one axis of a
// row-major array, for every element e and output i < M.  The matrix is stored in
// chunks of RB outputs, transposed within a chunk: tab[(c L + l) RB + k] = Mat[c RB + k][l]
// (rows past M zero).  With tab2 set (Burgers epilogue, row passes only) a second matrix
// scaled per element by scale2[e] gives w = tab2 . in, and the pass stores v - dt w v.
struct ElemPass {
    const double* in; long ldin;
    double* out; long ldout;
    AxisMap ain, aout;
    int L, M;              // inputs and outputs per element
    int rb, nchunks;       // chunk size (the kernel's RB) and count
    const double* tab;
    const double* tab2;    // or NULL
    const double* scale;   // per-element factor of tab (NULL = 1)
    const double* scale2;  // per-element factor of tab2
    double dt;
    int lines;             // independent lines: columns (row pass) or rows (column pass)
};

// Chunk size of the passes for M outputs per element (8, 16 or 33).
int elem_chunk(int M);
// Row pass: the transformed axis is x (array rows); lines are columns.
hipError_t launch_elem_rows(const ElemPass& a, hipStream_t s);
// Column pass: the transformed axis is y (array columns); lines are rows.  No tab2.
hipError_t launch_elem_cols(const ElemPass& a, hipStream_t s);

}  // namespace hpadi
