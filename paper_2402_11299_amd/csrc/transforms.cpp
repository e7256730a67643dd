// Host side of the grid transforms and of the Burgers time-stepper (Sec. 6).
// Declared in include/hpadi.h.
//
// Reference-element tables, computed once per axis in long double:
//   forward  (values at the m = p + 1 Chebyshev points of the first kind -> Legendre
//            coefficients of degrees 0..p): the DCT that gives the Chebyshev coefficients
//            of the interpolant (discrete orthogonality of T_0..T_p at those points),
//            followed by the Chebyshev -> Legendre connection matrix;
//   inverse  P_k at the points;
//   eval     the local hat+bubble functions at the points, and their t-derivatives
//            (d/dx = 2/delta_e d/dt is applied per element on the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "host_internal.h"
#include "hpadi.h"
#include "transforms.h"

using hpadi_host::dmalloc;

namespace {

using real = long double;
const real kPiL = 3.141592653589793238462643383279502884L;

// t_k = sin(pi (m - 2k - 1) / (2m)), k = 0..m-1 (descending): the roots of T_m, whose
// angles are theta_k = (2k + 1) pi / (2m).
real cheb_angle(int m, int k) { return (2 * k + 1) * kPiL / (2 * m); }
real cheb_point(int m, int k) { return std::sin(kPiL * (m - 2 * k - 1) / (2 * m)); }

// P_0(t) .. P_q(t) by the three-term recurrence (k+1) P_{k+1} = (2k+1) t P_k - k P_{k-1}.
void legendre_values(int q, real t, real* P) {
    P[0] = 1;
    if (q >= 1) P[1] = t;
    for (int k = 1; k < q; ++k) P[k + 1] = ((2 * k + 1) * t * P[k] - k * P[k - 1]) / (k + 1);
}

// Column j of the result holds the Legendre coefficients of T_j, j = 0..p:
// T_{j+1} = 2 x T_j - T_{j-1}, with multiplication by x in the Legendre basis,
// x P_k = ((k + 1) P_{k+1} + k P_{k-1}) / (2k + 1).  Row-major (p+1) x (p+1).
std::vector<real> cheb_to_legendre(int p) {
    const int m = p + 1;
    std::vector<real> C((size_t)m * m, 0);
    std::vector<real> prev(m + 1, 0), cur(m + 1, 0), next(m + 1, 0);
    cur[0] = 1;  // T_0
    for (int j = 0; j < m; ++j) {
        for (int k = 0; k < m; ++k) C[(size_t)k * m + j] = cur[k];
        // next = 2 x cur - prev (T_1 = x T_0)
        for (int k = 0; k <= m; ++k) {
            real xk = 0;
            if (k >= 1) xk += cur[k - 1] * k / (2 * k - 1);
            if (k + 1 <= m) xk += cur[k + 1] * (k + 1) / (2 * k + 3);
            next[k] = (j == 0 ? 1 : 2) * xk - (j == 0 ? 0 : prev[k]);
        }
        prev.swap(cur);
        cur.swap(next);
    }
    return C;
}

// Forward transform, row-major (p+1) x (p+1): Leg[k] = sum_i F[k][i] v(t_i).
std::vector<double> forward_matrix(int p) {
    const int m = p + 1;
    const std::vector<real> C = cheb_to_legendre(p);
    std::vector<real> D((size_t)m * m);  // Chebyshev coefficient j from value i
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) D[(size_t)j * m + i] = (j == 0 ? 1 : 2) * std::cos(j * cheb_angle(m, i)) / m;
    std::vector<double> F((size_t)m * m);
    for (int k = 0; k < m; ++k)
        for (int i = 0; i < m; ++i) {
            real s = 0;
            for (int j = k; j < m; ++j) s += C[(size_t)k * m + j] * D[(size_t)j * m + i];
            F[(size_t)k * m + i] = (double)s;
        }
    return F;
}

// Inverse transform: I[i][k] = P_k(t_i).
std::vector<double> inverse_matrix(int p) {
    const int m = p + 1;
    std::vector<double> I((size_t)m * m);
    std::vector<real> P(m + 1);
    for (int i = 0; i < m; ++i) {
        legendre_values(p, cheb_point(m, i), P.data());
        for (int k = 0; k < m; ++k) I[(size_t)i * m + k] = (double)P[k];
    }
    return I;
}

// Local basis at the points, m x (p+1): columns 0, 1 the hats of the left and right
// vertices, (1 - t)/2 and (1 + t)/2; column 2 + j the bubble W_j = (P_j - P_{j+2}) / (2j + 3)
// (Sec. 2.2).  deriv: d/dt, i.e. -1/2, 1/2 and -P_{j+1}.
std::vector<double> local_basis_matrix(int p, bool deriv) {
    const int m = p + 1;
    std::vector<double> E((size_t)m * m);
    std::vector<real> P(m + 2);
    for (int i = 0; i < m; ++i) {
        const real t = cheb_point(m, i);
        legendre_values(p + 1, t, P.data());
        double* row = E.data() + (size_t)i * m;
        row[0] = (double)(deriv ? real(-0.5) : (1 - t) / 2);
        row[1] = (double)(deriv ? real(0.5) : (1 + t) / 2);
        for (int j = 0; j + 2 <= p; ++j)
            row[2 + j] = (double)(deriv ? -P[j + 1] : (P[j] - P[j + 2]) / (2 * j + 3));
    }
    return E;
}

// The matrix (M x L, row-major) as matrix-core operand fragments for the device passes:
// out[((w S + s) 64 + lane)] = mat[16 w + lane % 16][4 s + lane / 16], zero outside.
std::vector<double> fragments(const std::vector<double>& mat, int M, int L) {
    const int W = (M + 15) / 16, S = (L + 3) / 4;
    std::vector<double> out((size_t)W * S * 64, 0.0);
    for (int w = 0; w < W; ++w)
        for (int s = 0; s < S; ++s)
            for (int lane = 0; lane < 64; ++lane) {
                const int i = 16 * w + lane % 16, l = 4 * s + lane / 16;
                if (i < M && l < L) out[((size_t)w * S + s) * 64 + lane] = mat[(size_t)i * L + l];
            }
    return out;
}

struct TrAxis {
    int n = 0, p = 0, m = 0, nh = 0, N = 0, bc = 0;
    double* fwd = nullptr;   // device tables in the fragment layout
    double* inv = nullptr;
    double* ev = nullptr;
    double* dv = nullptr;
    double* fwd_r = nullptr; // the same matrices row-major (tail rows of the passes)
    double* inv_r = nullptr;
    double* ev_r = nullptr;
    double* dv_r = nullptr;
    double* two_over_delta = nullptr;  // 2 / delta_e
};

hpadi::AxisMap axis_map(const TrAxis& a, int layout) { return hpadi::AxisMap{layout, a.n, a.m, a.nh, a.bc}; }

}  // namespace

struct hpadi_transform_s {
    TrAxis ax[2];
    hipStream_t stream = nullptr;
    double* S = nullptr;  // intermediate, max(Nleg_x, N_x) x lds
    long lds = 0;
    std::vector<void*> allocs;

    ~hpadi_transform_s() {
        for (void* p : allocs) (void)hipFree(p);
    }
    int upload(const std::vector<double>& h, double** d) {
        if (dmalloc(d, h.size()) != hipSuccess) return HPADI_ENOMEM;
        allocs.push_back(*d);
        return hipMemcpy(*d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess ? HPADI_OK
                                                                                                       : HPADI_EHIP;
    }
    int make_axis(const hpadi_op1d_s& op, TrAxis& a) {
        a.n = op.n; a.p = op.p; a.m = op.p + 1; a.nh = op.nh; a.N = op.N; a.bc = op.bc;
        std::vector<double> tod(op.n);
        for (int e = 0; e < op.n; ++e) tod[e] = 2.0 / op.delta[e];
        int rc;
        const std::vector<double> F = forward_matrix(a.p), I = inverse_matrix(a.p);
        const std::vector<double> E = local_basis_matrix(a.p, false), D = local_basis_matrix(a.p, true);
        if ((rc = upload(fragments(F, a.m, a.m), &a.fwd)) || (rc = upload(fragments(I, a.m, a.m), &a.inv)) ||
            (rc = upload(fragments(E, a.m, a.m), &a.ev)) || (rc = upload(fragments(D, a.m, a.m), &a.dv)) ||
            (rc = upload(F, &a.fwd_r)) || (rc = upload(I, &a.inv_r)) || (rc = upload(E, &a.ev_r)) ||
            (rc = upload(D, &a.dv_r)) ||
            (rc = upload(tod, &a.two_over_delta)))
            return rc;
        return HPADI_OK;
    }
};

namespace {

// A pass along x (rows) of the transform's x axis, or along y (columns) of its y axis.
// tab_r: the same matrix row-major (its tail rows).
hpadi::ElemPass make_pass(const TrAxis& a, int lin, int lout, const double* tab, const double* tab_r,
                          const double* in, long ldin, double* out, long ldout, int lines) {
    hpadi::ElemPass e{};
    e.in = in; e.ldin = ldin; e.out = out; e.ldout = ldout;
    e.ain = axis_map(a, lin);
    e.aout = axis_map(a, lout);
    e.L = a.m;  // m points, p + 1 degrees, p + 1 local basis functions
    e.M = a.m;
    // m = 16 k + r with k >= 4 and r <= 4 (m = 65, 129: r = 1): k matrix-core waves and r
    // tail rows by vector FMAs; otherwise ceil(m / 16) waves
    const int k = a.m / 16, r = a.m % 16;
    const bool tail = k >= 4 && r > 0 && r <= 4;
    e.nwaves = tail ? k : (a.m + 15) / 16;
    e.tail = tail ? r : 0;
    e.ttab = tail ? tab_r + (size_t)16 * k * a.m : nullptr;
    e.ksteps = (a.m + 3) / 4;
    e.tab = tab;
    e.lines = lines;
    return e;
}

int hip_status(hipError_t e) { return e == hipSuccess ? HPADI_OK : HPADI_EHIP; }

int forward(hpadi_transform_s* T, const double* V, long ldv, double* F, long ldf) {
    const TrAxis &X = T->ax[0], &Y = T->ax[1];
    const int nlx = X.n * X.m, nly = Y.n * Y.m;
    hipError_t e = hpadi::launch_elem_rows(
        make_pass(X, hpadi::AX_VALUES, hpadi::AX_LEGENDRE, X.fwd, X.fwd_r, V, ldv, T->S, T->lds, nly), T->stream);
    if (e == hipSuccess)
        e = hpadi::launch_elem_cols(
            make_pass(Y, hpadi::AX_VALUES, hpadi::AX_LEGENDRE, Y.fwd, Y.fwd_r, T->S, T->lds, F, ldf, nlx), T->stream);
    return hip_status(e);
}

int inverse(hpadi_transform_s* T, const double* F, long ldf, double* V, long ldv) {
    const TrAxis &X = T->ax[0], &Y = T->ax[1];
    const int nlx = X.n * X.m, nly = Y.n * Y.m;
    hipError_t e = hpadi::launch_elem_rows(
        make_pass(X, hpadi::AX_LEGENDRE, hpadi::AX_VALUES, X.inv, X.inv_r, F, ldf, T->S, T->lds, nly), T->stream);
    if (e == hipSuccess)
        e = hpadi::launch_elem_cols(
            make_pass(Y, hpadi::AX_LEGENDRE, hpadi::AX_VALUES, Y.inv, Y.inv_r, T->S, T->lds, V, ldv, nlx), T->stream);
    return hip_status(e);
}

// Y-pass of the evaluation: S = U E_y^T (values along y), N_x rows.
hipError_t eval_cols(hpadi_transform_s* T, const double* U, long ldu) {
    const TrAxis &X = T->ax[0], &Y = T->ax[1];
    return hpadi::launch_elem_cols(make_pass(Y, hpadi::AX_Q, hpadi::AX_VALUES, Y.ev, Y.ev_r, U, ldu, T->S, T->lds, X.N),
                                   T->stream);
}

}  // namespace

int hpadi_grid(hpadi_op1d op, double* x, int len) {
    if (!op || !x || len < op->n * (op->p + 1)) return HPADI_EINVAL;
    const int m = op->p + 1;
    for (int e = 0; e < op->n; ++e)
        for (int k = 0; k < m; ++k)
            x[e * m + k] = (double)(op->x[e] + (1 + cheb_point(m, k)) * (real)op->delta[e] / 2);
    return HPADI_OK;
}

int hpadi_transform_export(int p, int which, double* buf, int len) {
    if (p < 1 || p > 1024 || !buf || len < (p + 1) * (p + 1) || which < 0 || which > 3) return HPADI_EINVAL;
    const std::vector<double> M = which == 0   ? forward_matrix(p)
                                  : which == 1 ? inverse_matrix(p)
                                               : local_basis_matrix(p, which == 3);
    std::memcpy(buf, M.data(), M.size() * sizeof(double));
    return HPADI_OK;
}

int hpadi_transform_create(hpadi_op1d x, hpadi_op1d y, void* hip_stream, hpadi_transform* out) {
    if (!out) return HPADI_EINVAL;
    *out = nullptr;
    if (!x || !y || x->p + 1 > hpadi::elem_max_outputs() || y->p + 1 > hpadi::elem_max_outputs()) return HPADI_EINVAL;
    hpadi_transform_s* T = new (std::nothrow) hpadi_transform_s();
    if (!T) return HPADI_ENOMEM;
    T->stream = (hipStream_t)hip_stream;
    int rc;
    if ((rc = T->make_axis(*x, T->ax[0])) || (rc = T->make_axis(*y, T->ax[1]))) {
        delete T;
        return rc;
    }
    const long rows = std::max<long>(x->Nleg, x->N);
    T->lds = ((long)y->Nleg + 63) / 64 * 64;
    if (dmalloc(&T->S, (size_t)rows * T->lds) != hipSuccess) {
        delete T;
        return HPADI_ENOMEM;
    }
    T->allocs.push_back(T->S);
    *out = T;
    return HPADI_OK;
}

int hpadi_values_to_legendre(hpadi_transform T, const double* V, int ldv, double* F, int ldf) {
    if (!T || !V || !F || ldv < T->ax[1].n * T->ax[1].m || ldf < T->ax[1].n * T->ax[1].m) return HPADI_EINVAL;
    return forward(T, V, ldv, F, ldf);
}

int hpadi_legendre_to_values(hpadi_transform T, const double* F, int ldf, double* V, int ldv) {
    if (!T || !V || !F || ldv < T->ax[1].n * T->ax[1].m || ldf < T->ax[1].n * T->ax[1].m) return HPADI_EINVAL;
    return inverse(T, F, ldf, V, ldv);
}

int hpadi_q_to_values(hpadi_transform T, int deriv_x, const double* U, int ldu, double* V, int ldv) {
    if (!T || !U || !V || (deriv_x != 0 && deriv_x != 1)) return HPADI_EINVAL;
    const TrAxis &X = T->ax[0], &Y = T->ax[1];
    if (ldu < Y.N || ldv < Y.n * Y.m) return HPADI_EINVAL;
    hipError_t e = eval_cols(T, U, ldu);
    if (e != hipSuccess) return HPADI_EHIP;
    hpadi::ElemPass r = make_pass(X, hpadi::AX_Q, hpadi::AX_VALUES, deriv_x ? X.dv : X.ev, deriv_x ? X.dv_r : X.ev_r, T->S, T->lds, V, ldv,
                                  Y.n * Y.m);
    if (deriv_x) r.scale = X.two_over_delta;
    return hip_status(hpadi::launch_elem_rows(r, T->stream));
}

void hpadi_transform_destroy(hpadi_transform T) { delete T; }

// ---- Burgers ------------------------------------------------------------

struct hpadi_burgers_s {
    hpadi_plan plan = nullptr;
    hpadi_transform tr = nullptr;
    double omega2 = 0.0, dt = 0.0;
    double* G = nullptr;  // N_x x ldn
    double* U = nullptr;
    double* W = nullptr;  // Nleg_x x tr->lds: grid values of the step; the load's intermediate before
    long ldn = 0;

    ~hpadi_burgers_s() {
        (void)hipFree(G);
        (void)hipFree(U);
        (void)hipFree(W);
        hpadi_transform_destroy(tr);
        hpadi_plan_destroy(plan);
    }
};

int hpadi_burgers_create(hpadi_op1d x, hpadi_op1d y, double eps, double dt, double tol, int precision,
                         const hpadi_options* opts, void* hip_stream, hpadi_burgers* out) {
    if (!out) return HPADI_EINVAL;
    *out = nullptr;
    if (!x || !y || !(eps > 0.0) || !(dt > 0.0) || !std::isfinite(eps * dt)) return HPADI_EINVAL;
    const double omega2 = 1.0 / (dt * eps);
    if (!std::isfinite(omega2)) return HPADI_EINVAL;
    hpadi_burgers_s* B = new (std::nothrow) hpadi_burgers_s();
    if (!B) return HPADI_ENOMEM;
    B->omega2 = omega2;
    B->dt = dt;
    int rc = hpadi_plan_create_ex(x, y, omega2, tol, precision, nullptr, hip_stream, opts, &B->plan);
    if (rc == HPADI_OK) rc = hpadi_transform_create(x, y, hip_stream, &B->tr);
    if (rc != HPADI_OK) {
        delete B;
        return rc;
    }
    B->ldn = ((long)y->N + 63) / 64 * 64;
    if (dmalloc(&B->G, (size_t)x->N * B->ldn) != hipSuccess || dmalloc(&B->U, (size_t)x->N * B->ldn) != hipSuccess ||
        dmalloc(&B->W, (size_t)x->Nleg * B->tr->lds) != hipSuccess) {
        delete B;
        return HPADI_ENOMEM;
    }
    *out = B;
    return HPADI_OK;
}

int hpadi_burgers_step(hpadi_burgers B, double* F, int ldf, int nsteps, hpadi_stats* stats) {
    if (!B || !F || nsteps < 0) return HPADI_EINVAL;
    hpadi_plan P = B->plan;
    hpadi_transform_s* T = B->tr;
    const TrAxis &X = T->ax[0], &Y = T->ax[1];
    const int nly = Y.n * Y.m;
    if (ldf < nly) return HPADI_EINVAL;
    hpadi_stats st{};
    int status = HPADI_OK;
    for (int s = 0; s < nsteps; ++s) {
        // implicit Euler for the linear part: (K (x) M + M (x) K + omega^2 M (x) M) U = omega^2 T_x F T_y^T,
        // omega^2 = 1 / (dt eps)
        if (hpadi::launch_load(P->dx.dev, P->dy.dev, F, ldf, B->W, T->lds, B->G, B->ldn, T->stream, B->omega2) !=
            hipSuccess)
            return HPADI_EHIP;
        int rc = hpadi_solve(P, B->G, (int)B->ldn, B->U, (int)B->ldn, &st);
        if (rc != HPADI_OK && rc != HPADI_ENOCONV) return rc;
        if (rc == HPADI_ENOCONV) status = rc;
        // values of u and u_x at the grid and the explicit Euler step of the nonlinear part,
        // w = u - dt u u_x, fused into the x pass of the evaluation
        if (eval_cols(T, B->U, B->ldn) != hipSuccess) return HPADI_EHIP;
        hpadi::ElemPass r = make_pass(X, hpadi::AX_Q, hpadi::AX_VALUES, X.ev, X.ev_r, T->S, T->lds, B->W, T->lds, nly);
        r.tab2 = X.dv;
        if (r.tail) r.ttab2 = X.dv_r + (size_t)16 * r.nwaves * X.m;
        r.scale2 = X.two_over_delta;
        r.dt = B->dt;
        if (hpadi::launch_elem_rows(r, T->stream) != hipSuccess) return HPADI_EHIP;
        // back to Legendre coefficients
        int rf = forward(T, B->W, T->lds, F, ldf);
        if (rf != HPADI_OK) return rf;
        if (status != HPADI_OK) break;
    }
    if (stats) *stats = st;
    return status;
}

void hpadi_burgers_destroy(hpadi_burgers B) { delete B; }
