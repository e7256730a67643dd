// Host side of the variable-coefficient operator and of the ADI-preconditioned
// Krylov solvers (Sec. 7: CG preconditioned by the constant-coefficient ADI
// solve at a loose tolerance).  Declared in include/hpadi.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <new>
#include <vector>

#include "host_internal.h"
#include "hpadi.h"
#include "krylov.h"
#include "krylov_internal.h"

using hpadi_host::dmalloc;

static_assert(sizeof(hpadi_krylov_stats) == 64 && offsetof(hpadi_krylov_stats, fallback_iters) == 40,
              "hpadi_krylov_stats layout");

namespace {

constexpr double kPi = 3.14159265358979323846;

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_q from the
// Chebyshev-like initial guesses cos(pi (i - 1/4) / (q + 1/2)) (Golub-Welsch's
// eigenvalue route gives the same rule); weights 2 / ((1 - t^2) P_q'(t)^2).
void gauss_legendre(int q, std::vector<double>& t, std::vector<double>& w) {
    t.assign(q, 0.0);
    w.assign(q, 0.0);
    for (int i = 0; i < (q + 1) / 2; ++i) {
        double x = std::cos(kPi * (i + 0.75) / (q + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= q; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double pq = q == 0 ? 1.0 : (q == 1 ? x : p1);
            const double pqm1 = q == 1 ? 1.0 : p0;
            dp = q * (x * pq - pqm1) / (x * x - 1.0);
            const double dx = pq / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) {
                // one more evaluation of the derivative at the converged node
                p0 = 1.0;
                p1 = x;
                for (int k = 2; k <= q; ++k) {
                    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = q * (x * (q == 1 ? x : p1) - (q == 1 ? 1.0 : p0)) / (x * x - 1.0);
                break;
            }
        }
        // nodes ascending: t[i] = -x (x descending from near 1), mirrored at q-1-i
        t[i] = -x;
        t[q - 1 - i] = x;
        const double wi = 2.0 / ((1.0 - x * x) * dp * dp);
        w[i] = wi;
        w[q - 1 - i] = wi;
    }
}

// Values and reference derivatives at t of the local functions
// [left hat, right hat, W_0 .. W_{p-2}], W_k = (P_k - P_{k+2}) / (2k + 3), W_k' = -P_{k+1}.
void local_tables(int p, const std::vector<double>& t, std::vector<double>& V, std::vector<double>& D) {
    const int q = (int)t.size(), L = p + 1;
    V.assign((size_t)q * L, 0.0);
    D.assign((size_t)q * L, 0.0);
    std::vector<double> P(p + 2);
    for (int i = 0; i < q; ++i) {
        const double x = t[i];
        P[0] = 1.0;
        if (p + 1 >= 1) P[1] = x;
        for (int k = 2; k <= p + 1; ++k) P[k] = ((2.0 * k - 1.0) * x * P[k - 1] - (k - 1.0) * P[k - 2]) / k;
        V[i * L + 0] = (1.0 - x) / 2.0;
        V[i * L + 1] = (1.0 + x) / 2.0;
        D[i * L + 0] = -0.5;
        D[i * L + 1] = 0.5;
        for (int k = 0; k + 2 <= p; ++k) {
            V[i * L + 2 + k] = (P[k] - P[k + 2]) / (2.0 * k + 3.0);
            D[i * L + 2 + k] = -P[k + 1];
        }
    }
}

struct VcAxis {
    int n, p, q, N;
    std::vector<int> l2g, own;
    std::vector<double> delta, t, w, V, D;
};

void make_axis(const hpadi_op1d_s& o, VcAxis& A) {
    A.n = o.n;
    A.p = o.p;
    A.q = o.p + 2;
    A.N = o.N;
    A.delta = o.delta;
    gauss_legendre(A.q, A.t, A.w);
    local_tables(o.p, A.t, A.V, A.D);
    const int L = o.p + 1;
    A.l2g.assign((size_t)o.n * L, -1);
    A.own.assign((size_t)4 * o.N, -1);
    auto add_owner = [&](int g, int e, int l) {
        int* ow = &A.own[4 * (size_t)g];
        const int slot = ow[0] < 0 ? 0 : 1;
        ow[2 * slot] = e;
        ow[2 * slot + 1] = l;
    };
    for (int e = 0; e < o.n; ++e) {
        if (o.vertex_is_hat(e)) A.l2g[e * L + 0] = o.hat_of_vertex(e);
        if (o.vertex_is_hat(e + 1)) A.l2g[e * L + 1] = o.hat_of_vertex(e + 1);
        for (int m = 0; m + 2 <= o.p; ++m) A.l2g[e * L + 2 + m] = o.bubble(m, e);
        for (int l = 0; l < L; ++l)
            if (A.l2g[e * L + l] >= 0) add_owner(A.l2g[e * L + l], e, l);
    }
}

}  // namespace

namespace {

template <typename T>
int upload(hpadi_varcoef_s* V, const std::vector<T>& h, const T** out) {
    T* p = nullptr;
    if (dmalloc(&p, h.size()) != hipSuccess) return HPADI_ENOMEM;
    V->allocs.push_back(p);
    if (!h.empty() && hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return HPADI_EHIP;
    *out = p;
    return HPADI_OK;
}

int ensure_work(hpadi_varcoef_s* V, int m) {
    const size_t n = (size_t)V->Nx * V->Ny;
    if (!V->r) {
        if (dmalloc(&V->r, n) != hipSuccess || dmalloc(&V->z, n) != hipSuccess || dmalloc(&V->zs, n) != hipSuccess ||
            dmalloc(&V->Az, n) != hipSuccess || dmalloc(&V->Ac, n) != hipSuccess ||
            dmalloc(&V->part, 4 * (size_t)hpadi::dot_parts()) != hipSuccess || dmalloc(&V->dots, 8) != hipSuccess)
            return HPADI_ENOMEM;
        if (hipHostMalloc((void**)&V->dots_host, 8 * sizeof(double)) != hipSuccess) return HPADI_ENOMEM;
    }
    const int need = std::max(m, 1) + 1;
    while ((int)V->d.size() < need) {
        double *dd = nullptr, *qq = nullptr;
        if (dmalloc(&dd, n) != hipSuccess || dmalloc(&qq, n) != hipSuccess) {
            (void)hipFree(dd);
            return HPADI_ENOMEM;
        }
        V->d.push_back(dd);
        V->q.push_back(qq);
    }
    return HPADI_OK;
}

// out[k] = a . b_k on the device, copied to V->dots_host (synchronises the stream)
int dots(hpadi_varcoef_s* V, const double* a, std::initializer_list<const double*> bs, double* res) {
    hpadi::MultiB mb{};
    mb.nb = 0;
    for (const double* b : bs) mb.b[mb.nb++] = b;
    const long n = (long)V->Nx * V->Ny;
    if (hpadi::launch_multidot(a, mb, n, V->part, V->dots, V->stream) != hipSuccess) return HPADI_EHIP;
    if (hipMemcpyAsync(V->dots_host, V->dots, mb.nb * sizeof(double), hipMemcpyDeviceToHost, V->stream) != hipSuccess ||
        hipStreamSynchronize(V->stream) != hipSuccess)
        return HPADI_EHIP;
    for (int k = 0; k < mb.nb; ++k) res[k] = V->dots_host[k];
    return HPADI_OK;
}

int axpy(hpadi_varcoef_s* V, double* y, double c, const double* x) {
    hpadi::MultiB mb{};
    mb.nb = 1;
    mb.b[0] = x;
    hpadi::Coefs cc{};
    cc.c[0] = c;
    return hpadi::launch_axpys(y, mb, cc, (long)V->Nx * V->Ny, V->stream) == hipSuccess ? HPADI_OK : HPADI_EHIP;
}

}  // namespace

extern "C" {

int hpadi_varcoef_grid(hpadi_op1d op, double* x, double* w, int len) {
    if (!op) return HPADI_EINVAL;
    const int q = op->p + 2;
    if (len < op->n * q) return HPADI_EINVAL;
    std::vector<double> t, wt;
    gauss_legendre(q, t, wt);
    for (int e = 0; e < op->n; ++e)
        for (int i = 0; i < q; ++i) {
            const double d = op->delta[e];
            if (x) x[e * q + i] = op->x[e] + (t[i] + 1.0) * d / 2.0;
            if (w) w[e * q + i] = wt[i] * d / 2.0;
        }
    return HPADI_OK;
}

int hpadi_varcoef_create(hpadi_op1d x, hpadi_op1d y, const double* a_dev, int lda, void* hip_stream,
                         hpadi_varcoef* out) {
    if (!a_dev) return HPADI_EINVAL;
    return hpadi_varcoef_create_ex(x, y, a_dev, lda, nullptr, 0, hip_stream, out);
}

int hpadi_varcoef_create_ex(hpadi_op1d x, hpadi_op1d y, const double* a_dev, int lda, const double* c_dev, int ldc,
                            void* hip_stream, hpadi_varcoef* out) {
    if (!x || !y || !out) return HPADI_EINVAL;
    *out = nullptr;
    // the Gauss-point form has no boundary term: Robin ends are not supported here
    if (x->alpha[0] != 0.0 || x->alpha[1] != 0.0 || y->alpha[0] != 0.0 || y->alpha[1] != 0.0) return HPADI_EINVAL;
    const int qx = x->p + 2, qy = y->p + 2;
    const long rows = (long)x->n * qx, cols = (long)y->n * qy;
    if ((a_dev && lda < cols) || (c_dev && ldc < cols)) return HPADI_EINVAL;
    if (a_dev && hpadi::vc_lds_bytes(x->p, y->p) > 160 * 1024) return HPADI_EINVAL;
    hpadi_varcoef_s* V = new (std::nothrow) hpadi_varcoef_s();
    if (!V) return HPADI_ENOMEM;
    V->stream = (hipStream_t)hip_stream;
    V->Nx = x->N;
    V->Ny = y->N;
    VcAxis ax, ay;
    make_axis(*x, ax);
    make_axis(*y, ay);
    hpadi::VarCoefDev& d = V->dev;
    d.nx = x->n; d.px = x->p; d.qx = qx; d.Nx = x->N;
    d.ny = y->n; d.py = y->p; d.qy = qy; d.Ny = y->N;
    int rc = HPADI_OK;
    if ((rc = upload(V, ax.l2g, &d.l2gx)) || (rc = upload(V, ay.l2g, &d.l2gy)) || (rc = upload(V, ax.own, &d.ownx)) ||
        (rc = upload(V, ay.own, &d.owny)) || (rc = upload(V, ax.delta, &d.delx)) || (rc = upload(V, ay.delta, &d.dely)) ||
        (rc = upload(V, ax.w, &d.wx)) || (rc = upload(V, ay.w, &d.wy)) || (rc = upload(V, ax.V, &d.Evx)) ||
        (rc = upload(V, ax.D, &d.Edx)) || (rc = upload(V, ay.V, &d.Evy)) || (rc = upload(V, ay.D, &d.Edy))) {
        delete V;
        return rc;
    }
    V->opx = *x;
    V->opy = *y;
    V->a_host.assign((size_t)rows * cols, 1.0);
    // reference weight x Jacobian factor of a term on the Gauss grid
    auto weights = [&](const std::vector<double>* coef, auto&& factor) {
        std::vector<double> C((size_t)rows * cols);
        for (long r = 0; r < rows; ++r)
            for (long c = 0; c < cols; ++c) {
                const int ex = (int)(r / qx), i = (int)(r % qx), ey = (int)(c / qy), j = (int)(c % qy);
                const double f = factor(ax.delta[ex], ay.delta[ey]);
                C[(size_t)r * cols + c] = (coef ? (*coef)[(size_t)r * cols + c] : 1.0) * ax.w[i] * ay.w[j] * f;
            }
        return C;
    };
    auto sep_term = [&](const std::vector<double>& C, const double* Ex, const double* Ey) -> int {
        const double* dC = nullptr;
        int r2 = upload(V, C, &dC);
        if (r2 != HPADI_OK) return r2;
        d.sEx[d.nsep] = Ex;
        d.sEy[d.nsep] = Ey;
        d.sC[d.nsep] = dC;
        d.nsep++;
        return HPADI_OK;
    };
    d.nsep = 0;
    if (a_dev) {
        // the gradient terms by the element kernel: own compact copy of a and the element scratch
        double* a = nullptr;
        double* ye = nullptr;
        if (dmalloc(&a, (size_t)rows * cols) != hipSuccess ||
            dmalloc(&ye, (size_t)x->n * y->n * (x->p + 1) * (y->p + 1)) != hipSuccess) {
            (void)hipFree(a);
            delete V;
            return HPADI_ENOMEM;
        }
        V->allocs.push_back(a);
        V->allocs.push_back(ye);
        if (hpadi::launch_copy2d(a_dev, lda, a, cols, (int)rows, (int)cols, V->stream) != hipSuccess ||
            hipStreamSynchronize(V->stream) != hipSuccess) {
            delete V;
            return HPADI_EHIP;
        }
        d.a = a;
        d.lda = cols;
        d.Ye = ye;
        d.element_terms = 1;
        if (hipMemcpy(V->a_host.data(), a, V->a_host.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
            delete V;
            return HPADI_EHIP;
        }
    } else {
        // a = 1: the gradient terms as separable passes (d/dx u d/dx v: derivative table on
        // x, values on y, Jacobian factor delta_y / delta_x; the y pair likewise)
        d.element_terms = 0;
        if ((rc = sep_term(weights(nullptr, [](double dx, double dy) { return dy / dx; }), d.Edx, d.Evy)) ||
            (rc = sep_term(weights(nullptr, [](double dx, double dy) { return dx / dy; }), d.Evx, d.Edy))) {
            delete V;
            return rc;
        }
    }
    if (c_dev) {
        // potential: values on both axes, Jacobian delta_x delta_y / 4
        std::vector<double> ch((size_t)rows * cols);
        if (hipMemcpy2D(ch.data(), cols * sizeof(double), c_dev, (size_t)ldc * sizeof(double), cols * sizeof(double),
                        rows, hipMemcpyDeviceToHost) != hipSuccess) {
            delete V;
            return HPADI_EHIP;
        }
        if ((rc = sep_term(weights(&ch, [](double dx, double dy) { return dx * dy / 4.0; }), d.Evx, d.Evy))) {
            delete V;
            return rc;
        }
    }
    if (d.nsep > 0) {
        double *t1 = nullptr, *t2 = nullptr;
        if (dmalloc(&t1, (size_t)rows * y->N) != hipSuccess || dmalloc(&t2, (size_t)rows * cols) != hipSuccess) {
            (void)hipFree(t1);
            delete V;
            return HPADI_ENOMEM;
        }
        V->allocs.push_back(t1);
        V->allocs.push_back(t2);
        d.T1 = t1;
        d.T2 = t2;
    }
    *out = V;
    return HPADI_OK;
}

int hpadi_varcoef_apply(hpadi_varcoef V, const double* U, int ldu, double* Y, int ldy) {
    if (!V || !U || !Y || ldu < V->Ny || ldy < V->Ny) return HPADI_EINVAL;
    return hpadi::launch_vc_apply(V->dev, U, ldu, Y, ldy, V->stream) == hipSuccess ? HPADI_OK : HPADI_EHIP;
}

void hpadi_varcoef_destroy(hpadi_varcoef V) { delete V; }

int hpadi_fcg_solve(hpadi_varcoef V, hpadi_plan precond, hpadi_net net, const double* b, int ldb, double* x, int ldx,
                    double tol, int maxit, int truncation, double* res_hist, int hist_len, hpadi_krylov_stats* stats) {
    return hpadi_host::fcg_core(V, precond, net, b, ldb, x, ldx, tol, maxit, truncation, res_hist, hist_len, stats,
                                hpadi_host::KrylovObserver());
}

}  // extern "C"

namespace hpadi_host {

int fcg_core(hpadi_varcoef_s* V, hpadi_plan precond, hpadi_net net, const double* b, int ldb, double* x, int ldx,
             double tol, int maxit, int truncation, double* res_hist, int hist_len, hpadi_krylov_stats* stats,
             const KrylovObserver& observe) {
    if (!V || !b || !x || ldb < V->Ny || ldx < V->Ny || !(tol > 0.0) || maxit < 0 || truncation < 0 ||
        truncation > 4)
        return HPADI_EINVAL;
    if (precond && (precond->dx.op.N != V->Nx || precond->dy.op.N != V->Ny)) return HPADI_EINVAL;
    if (net && ensure_slots(V) != HPADI_OK) return HPADI_ENOMEM;
    const auto t0 = std::chrono::steady_clock::now();
    int rc = ensure_work(V, truncation);
    if (rc != HPADI_OK) return rc;
    hipStream_t s = V->stream;
    const int Nx = V->Nx, Ny = V->Ny;
    const long n = (long)Nx * Ny;
    hpadi_krylov_stats st{};
    // compact copy of b lives in q[last] for the true residual; x starts at 0
    double* bc = V->q.back();
    double* xc = V->d.back();
    if (hpadi::launch_copy2d(b, ldb, bc, Ny, Nx, Ny, s) != hipSuccess ||
        hipMemsetAsync(xc, 0, n * sizeof(double), s) != hipSuccess ||
        hipMemcpyAsync(V->r, bc, n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return HPADI_EHIP;
    double bb;
    if ((rc = dots(V, bc, {bc}, &bb)) != HPADI_OK) return rc;
    const double bn = std::sqrt(bb);
    if (res_hist && hist_len > 0) res_hist[0] = 1.0;
    auto precondition = [&]() -> int {
        // z = P r (ADI solve of the constant-coefficient operator), or z = r
        if (!precond)
            return hipMemcpyAsync(V->z, V->r, n * sizeof(double), hipMemcpyDeviceToDevice, s) == hipSuccess
                       ? HPADI_OK
                       : HPADI_EHIP;
        if (precond->stream != s && hipStreamSynchronize(s) != hipSuccess) return HPADI_EHIP;
        hpadi_stats ps{};
        int r2 = hpadi_solve(precond, V->r, Ny, V->z, Ny, &ps);
        if (r2 != HPADI_OK && r2 != HPADI_ENOCONV) return r2;
        if (precond->stream != s && hipStreamSynchronize(precond->stream) != hipSuccess) return HPADI_EHIP;
        st.precond_calls++;
        return HPADI_OK;
    };
    const int ring = std::max(truncation, 1);
    std::vector<double> dq_hist(ring + 1, 0.0);
    int k = 0;
    bool converged = bn == 0.0;
    double rel = converged ? 0.0 : 1.0;
    // Iterations k0 .. kmax - 1 from the current x and r with truncation m (0 = PCG) and
    // the network nn (or none).  A corrected run gives up (returns with *give_up) on a
    // non-finite or non-positive curvature, on divergence (the residual 100 times its
    // best) and after kmax iterations; a plain run ends ENOTSPD on a non-positive one.
    auto iterate = [&](int m, hpadi_net nn, int kmax, bool* give_up) -> int {
        *give_up = false;
        double rz_old = 0.0, best = rel, mark = rel;
        const int k0 = k;
        int k_mark = k;  // iteration of the last halving of the residual
        while (!converged && k < kmax) {
            int r2;
            if ((r2 = precondition()) != HPADI_OK) return r2;
            if (nn) {
                bool applied = false;
                if ((r2 = net_correct(nn, V, V->r, V->z, k, &applied)) != HPADI_OK) return r2;
                if (applied) st.corrections++;
            }
            if (observe && (r2 = observe(k, V->r, V->z, xc)) != HPADI_OK) return r2;
            const int kk = k - k0;  // directions of this run only
            double* dk = V->d[kk % ring];
            double* qk = V->q[kk % ring];
            if (m == 0) {
                // PCG: d = z + beta d, beta = (r.z) / (r_old.z_old)
                double rz;
                if ((r2 = dots(V, V->r, {V->z}, &rz)) != HPADI_OK) return r2;
                const double beta = kk == 0 ? 0.0 : rz / rz_old;
                rz_old = rz;
                if (hpadi::launch_xpby(dk, V->z, beta, n, s) != hipSuccess) return HPADI_EHIP;
            } else {
                // FCG(m): d = z - sum_{i in window} (z.q_i / d_i.q_i) d_i
                const int nw = std::min(kk, m);
                double c[4] = {0, 0, 0, 0};
                if (nw > 0) {
                    hpadi::MultiB mb{};
                    mb.nb = nw;
                    for (int i2 = 0; i2 < nw; ++i2) mb.b[i2] = V->q[(kk - 1 - i2) % ring];
                    if (hpadi::launch_multidot(V->z, mb, n, V->part, V->dots, s) != hipSuccess ||
                        hipMemcpyAsync(V->dots_host, V->dots, nw * sizeof(double), hipMemcpyDeviceToHost, s) !=
                            hipSuccess ||
                        hipStreamSynchronize(s) != hipSuccess)
                        return HPADI_EHIP;
                    for (int i2 = 0; i2 < nw; ++i2) c[i2] = -V->dots_host[i2] / dq_hist[(kk - 1 - i2) % ring];
                }
                // the oldest direction of the ring is overwritten by d_k: form d_k in z first
                if (nw > 0) {
                    hpadi::MultiB xs{};
                    hpadi::Coefs cc{};
                    xs.nb = nw;
                    for (int i2 = 0; i2 < nw; ++i2) {
                        xs.b[i2] = V->d[(kk - 1 - i2) % ring];
                        cc.c[i2] = c[i2];
                    }
                    if (hpadi::launch_axpys(V->z, xs, cc, n, s) != hipSuccess) return HPADI_EHIP;
                }
                if (hipMemcpyAsync(dk, V->z, n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
                    return HPADI_EHIP;
            }
            // q = A d; alpha = d.r / d.q
            if (hpadi::launch_vc_apply(V->dev, dk, Ny, qk, Ny, s) != hipSuccess) return HPADI_EHIP;
            double dd[2];
            if ((r2 = dots(V, dk, {qk, V->r}, dd)) != HPADI_OK) return r2;
            const double dq = dd[0];
            if (!(dq > 0.0) || !std::isfinite(dq)) {
                if (nn) {
                    *give_up = true;
                    return HPADI_OK;
                }
                return HPADI_ENOTSPD;
            }
            dq_hist[kk % ring] = dq;
            const double alpha = (m == 0 ? rz_old : dd[1]) / dq;
            if ((r2 = axpy(V, xc, alpha, dk)) != HPADI_OK || (r2 = axpy(V, V->r, -alpha, qk)) != HPADI_OK) return r2;
            ++k;
            double rr;
            if ((r2 = dots(V, V->r, {V->r}, &rr)) != HPADI_OK) return r2;
            rel = std::sqrt(std::max(rr, 0.0)) / bn;
            if (res_hist && k < hist_len) res_hist[k] = rel;
            if (!std::isfinite(rel) || (nn && rel > 100.0 * best)) {
                if (nn) *give_up = true;
                return HPADI_OK;
            }
            best = std::min(best, rel);
            if (rel <= 0.5 * mark) {
                mark = rel;
                k_mark = k;
            } else if (nn && k - k_mark >= 10) {
                // stagnation: ten iterations without halving the residual
                *give_up = true;
                return HPADI_OK;
            }
            if (rel <= tol) converged = true;
        }
        if (nn && !converged) *give_up = true;
        return HPADI_OK;
    };
    bool give_up = false;
    // with a network: at most half the iterations, then plain ADI-PCG from the last finite
    // iterate (from x = 0 if none) for the rest
    rc = iterate(truncation, net, net ? std::max(1, maxit / 2) : maxit, &give_up);
    if (rc == HPADI_OK && net && give_up && !converged) {
        // r = b - A x; restart from 0 when x or that residual is not finite
        if (hpadi::launch_vc_apply(V->dev, xc, Ny, V->z, Ny, s) != hipSuccess) return HPADI_EHIP;
        if (hipMemcpyAsync(V->r, bc, n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess ||
            axpy(V, V->r, -1.0, V->z) != HPADI_OK)
            return HPADI_EHIP;
        double rr;
        if ((rc = dots(V, V->r, {V->r}, &rr)) != HPADI_OK) return rc;
        rel = std::sqrt(std::max(rr, 0.0)) / bn;
        if (!std::isfinite(rel) || rel > 1.0) {
            if (hipMemsetAsync(xc, 0, n * sizeof(double), s) != hipSuccess ||
                hipMemcpyAsync(V->r, bc, n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
                return HPADI_EHIP;
            rel = 1.0;
        }
        const int k_switch = k;
        rc = iterate(0, nullptr, maxit, &give_up);
        st.fallback_iters = k - k_switch;
    }
    if (rc != HPADI_OK && rc != HPADI_ENOTSPD) return rc;
    // true residual b - A x, and x to the caller's layout
    double* tr = V->z;
    if (hpadi::launch_vc_apply(V->dev, xc, Ny, tr, Ny, s) != hipSuccess) return HPADI_EHIP;
    if (axpy(V, tr, -1.0, bc) != HPADI_OK) return HPADI_EHIP;
    double trr = 0.0;
    if (dots(V, tr, {tr}, &trr) != HPADI_OK) return HPADI_EHIP;
    if (hpadi::launch_copy2d(xc, Ny, x, ldx, Nx, Ny, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return HPADI_EHIP;
    st.iters = k;
    st.rel_res = rel;
    st.true_rel_res = bn > 0 ? std::sqrt(std::max(trr, 0.0)) / bn : 0.0;
    st.status = rc != HPADI_OK ? rc : (converged ? HPADI_OK : HPADI_ENOCONV);
    st.t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return st.status;
}


int ensure_slots(hpadi_varcoef_s* V) {
    if (V->sx) return HPADI_OK;
    const hpadi_op1d_s* ops[2] = {&V->opx, &V->opy};
    std::vector<int> slot[2];
    std::vector<int> gidx[2];      // Gauss index (e q + i) of each slot
    std::vector<float> wts[2];
    for (int a = 0; a < 2; ++a) {
        const hpadi_op1d_s& o = *ops[a];
        const int S = o.n * o.p + 1, q = o.p + 2;
        std::vector<double> t, w;
        gauss_legendre(q, t, w);
        slot[a].assign(S, -1);
        gidx[a].assign(S, 0);
        wts[a].assign(2 * S, 0.0f);  // [mass diagonal | stiffness diagonal] of the slot functions
        for (int s = 0; s < S; ++s) {
            const int e = std::min(s / o.p, o.n - 1);
            const int j = s - e * o.p;  // 0 = left vertex, p = right vertex (last slot), else bubble j-1
            double xi;
            if (j == 0 || j == o.p) {
                const int v = e + (j == o.p ? 1 : 0);
                if (o.vertex_is_hat(v)) {
                    slot[a][s] = o.hat_of_vertex(v);
                    const double dl = v > 0 ? o.delta[v - 1] : 0.0, dr = v < o.n ? o.delta[v] : 0.0;
                    wts[a][s] = (float)((dl + dr) / 3.0);
                    wts[a][S + s] = (float)((v > 0 ? 1.0 / dl : 0.0) + (v < o.n ? 1.0 / dr : 0.0));
                }
                xi = j == 0 ? -1.0 : 1.0;
            } else {
                const int m = j - 1;
                slot[a][s] = o.bubble(m, e);
                wts[a][s] = (float)(2.0 * o.delta[e] / ((2.0 * m + 1) * (2.0 * m + 3) * (2.0 * m + 5)));
                wts[a][S + s] = (float)(4.0 / ((2.0 * m + 3) * o.delta[e]));
                xi = -1.0 + 2.0 * j / o.p;
            }
            int best = 0;
            for (int i = 1; i < q; ++i)
                if (std::fabs(t[i] - xi) < std::fabs(t[best] - xi)) best = i;
            gidx[a][s] = e * q + best;
        }
    }
    const int H = (int)slot[0].size(), W = (int)slot[1].size();
    const long lda = (long)V->opy.n * (V->opy.p + 2);
    std::vector<float> la((size_t)H * W);
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j)
            la[(size_t)i * W + j] = (float)std::log(std::max(V->a_host[(size_t)gidx[0][i] * lda + gidx[1][j]], 1e-300));
    auto up = [](const void* h, size_t bytes, void** d) -> bool {
        return hipMalloc(d, bytes) == hipSuccess && hipMemcpy(*d, h, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    const size_t hw = (size_t)H * W;
    if (!up(slot[0].data(), H * sizeof(int), (void**)&V->sx) || !up(slot[1].data(), W * sizeof(int), (void**)&V->sy) ||
        !up(la.data(), hw * sizeof(float), (void**)&V->loga) || !up(wts[0].data(), 2 * H * sizeof(float), (void**)&V->wx) ||
        !up(wts[1].data(), 2 * W * sizeof(float), (void**)&V->wy) || dmalloc(&V->img, 3 * hw) != hipSuccess ||
        dmalloc(&V->img_out, hw) != hipSuccess || dmalloc(&V->img_zn, hw) != hipSuccess ||
        dmalloc(&V->img_t, hw) != hipSuccess || dmalloc(&V->img_w, hw) != hipSuccess)
        return HPADI_ENOMEM;
    V->H = H;
    V->W = W;
    return HPADI_OK;
}

}  // namespace hpadi_host

