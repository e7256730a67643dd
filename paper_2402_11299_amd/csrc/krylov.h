// Declarations shared by the variable-coefficient kernels (varcoef.hip) and the
// host code of the Krylov solvers (krylov.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace hpadi {

// Device view of the variable-coefficient operator -div(a grad u) on one mesh pair.
struct VarCoefDev {
    int nx, px, qx, Nx;
    int ny, py, qy, Ny;
    const int* l2gx; const int* l2gy;        // [n (p+1)] global index of local function, -1 if absent
    const int* ownx; const int* owny;        // [4 N]: (element, local) x 2 owners of each global index, -1 = none
    const double* delx; const double* dely;  // element widths
    const double* wx; const double* wy;      // reference Gauss weights [q]
    const double* Evx; const double* Edx;    // [q (p+1)] local values / reference derivatives at the points
    const double* Evy; const double* Edy;
    const double* a; long lda;               // coefficient on the (n_x q_x) x (n_y q_y) grid
    double* Ye;                              // element results [n_x n_y (p_x+1)(p_y+1)]
    // Separable terms (any degree): Y (+)= sum_t E_t^x^T [C_t . (E_t^x U E_t^y^T)] E_t^y with
    // E the local value or reference-derivative tables above and C_t the weights of the
    // term on the Gauss grid (coefficient, Gauss weights and Jacobian factors folded in,
    // compact (n_x q_x) x (n_y q_y)).  element_terms = 0: the gradient terms are among
    // them (a = 1); 1: the element kernel computes the gradient terms.
    int nsep;
    int element_terms;
    const double* sEx[3]; const double* sEy[3]; const double* sC[3];
    double* T1;                              // (n_x q_x) x N_y work
    double* T2;                              // (n_x q_x) x (n_y q_y) work
};
size_t vc_lds_bytes(int px, int py);
hipError_t launch_vc_apply(const VarCoefDev& v, const double* U, long ldu, double* Y, long ldy, hipStream_t s);

struct MultiB { const double* b[4]; int nb; };
struct Coefs { double c[4]; };
int dot_parts();
// out[k] = a . b_k for k < nb (two-stage, fixed summation order); part: 4 * dot_parts() doubles
hipError_t launch_multidot(const double* a, const MultiB& bs, long n, double* part, double* out, hipStream_t s);
hipError_t launch_axpys(double* y, const MultiB& xs, const Coefs& c, long n, hipStream_t s);  // y += sum c_k x_k
hipError_t launch_xpby(double* y, const double* x, double beta, long n, hipStream_t s);      // y = x + beta y
hipError_t launch_copy2d(const double* x, long ldx, double* y, long ldy, int rows, int cols, hipStream_t s);

}  // namespace hpadi
