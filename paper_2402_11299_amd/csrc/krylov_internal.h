// Host-side state of the variable-coefficient operator, shared by the Krylov
// solvers (krylov.cpp) and the learned correction (net.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <vector>

#include "host_internal.h"
#include "hpadi.h"
#include "krylov.h"
#include "net.h"

struct hpadi_varcoef_s {
    hpadi::VarCoefDev dev{};
    hipStream_t stream = nullptr;
    int Nx = 0, Ny = 0;
    std::vector<void*> allocs;
    // Krylov work (allocated on first use): r, z, the directions d_i and q_i = A d_i
    double* r = nullptr;
    double* z = nullptr;
    double* zs = nullptr;         // learned correction c of z
    double* Az = nullptr;         // A z and A c for the energy-optimal combination
    double* Ac = nullptr;
    std::vector<double*> d, q;
    double* part = nullptr;
    double* dots = nullptr;
    double* dots_host = nullptr;
    // operators (for the coefficient-image maps of the learned correction)
    hpadi_op1d_s opx, opy;
    std::vector<double> a_host;   // coefficient on the Gauss grid (compact, host copy)
    // slot image (built on first use): H = n_x p_x + 1, W = n_y p_y + 1
    int H = 0, W = 0;
    int* sx = nullptr;
    int* sy = nullptr;
    float* loga = nullptr;
    float* wx = nullptr;
    float* wy = nullptr;
    float* img = nullptr;         // [H W 3] network input
    float* img_out = nullptr;     // [H W] network output
    float* img_zn = nullptr;      // [H W] target images (training pairs)
    float* img_t = nullptr;
    float* img_w = nullptr;
    ~hpadi_varcoef_s() {
        if (stream) (void)hipStreamSynchronize(stream);
        for (void* p : allocs) (void)hipFree(p);
        for (double* p : d) (void)hipFree(p);
        for (double* p : q) (void)hipFree(p);
        (void)hipFree(r);
        (void)hipFree(z);
        (void)hipFree(zs);
        (void)hipFree(Az);
        (void)hipFree(Ac);
        (void)hipFree(part);
        (void)hipFree(dots);
        if (dots_host) (void)hipHostFree(dots_host);
        for (void* p : {(void*)sx, (void*)sy, (void*)loga, (void*)wx, (void*)wy, (void*)img, (void*)img_out,
                        (void*)img_zn, (void*)img_t, (void*)img_w})
            (void)hipFree(p);
    }
};

namespace hpadi_host {

// Slot image of the coefficient arrays (element-major: per element its left-vertex hat
// then W_0 .. W_{p-2}; one trailing slot for the last vertex), log a at the slots and
// the diagonal-mass weights of the slots.  Built once per operator.
int ensure_slots(hpadi_varcoef_s* V);

// Per-iteration observer of the Krylov loop: (k, r, z, x) device pointers to compact
// N_x x N_y arrays after the preconditioner (and correction) of iteration k.
typedef std::function<int(int, const double*, const double*, const double*)> KrylovObserver;

int fcg_core(hpadi_varcoef_s* V, hpadi_plan precond, hpadi_net net, const double* b, int ldb, double* x, int ldx,
             double tol, int maxit, int truncation, double* res_hist, int hist_len, hpadi_krylov_stats* stats,
             const KrylovObserver& observe);

// Learned correction of the preconditioned residual at Krylov iteration iter (only at
// multiples of the net's period): c = s_z NN([z/s_z, (z/s_z)/a, log a]) on the slot image
// (s_z = root-mean-square value of z).  Damping 0: z <- z + (beta/alpha) c with (alpha, beta)
// minimising the energy error f(v) = v.Av - 2 v.r of alpha z + beta c (the error equation is
// A e = r, and f(v) = ||v - e||_A^2 - e.r); *applied = false when the combination is
// degenerate or not finite, z is then left as it was.  Damping omega > 0: z <- z + omega c.
int net_correct(hpadi_net net, hpadi_varcoef_s* V, const double* r, double* z, int iter, bool* applied);

}  // namespace hpadi_host
