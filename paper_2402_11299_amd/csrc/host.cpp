// Host side of hpadi: 1D operators, spectral interval, ADI shifts, plans and
// the C ABI declared in include/hpadi.h.
#include "hpadi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

#include "internal.h"
#include "host_internal.h"

// The Python binding mirrors these structs with ctypes; their layout is part of the ABI.
static_assert(sizeof(hpadi_options) == 48 && offsetof(hpadi_options, row_lines_per_block) == 40, "hpadi_options layout");
static_assert(sizeof(hpadi_stats) == 96 && offsetof(hpadi_stats, J_refine) == 68, "hpadi_stats layout");

using hpadi::DimDev;
using hpadi::FactorLayout;

// ===========================================================================
// 1D operators (Sec. 2.2-2.3, App. A).
// ===========================================================================

namespace {

constexpr double kPi = 3.14159265358979323846;
// The hat block of a line is solved by one wavefront (64 lanes, the last also taking a
// 65th hat), so plans take at most 65 hats per axis: n <= 64 (Dirichlet), n <= 64
// (Neumann, n + 1 hats).
constexpr int kMaxHats = 65;

// Bubble blocks on the reference element, scaled by delta (App. A, eq. app:1):
double k_bub(int m) { return 4.0 / (2.0 * m + 3.0); }                                      // K (m,m) * delta
double m_bub(int m) { return 2.0 / ((2.0 * m + 1) * (2.0 * m + 3) * (2.0 * m + 5)); }       // M (m,m) / delta
double m_off(int m) { return -1.0 / ((2.0 * m + 3) * (2.0 * m + 5) * (2.0 * m + 7)); }      // M (m,m+2) / delta

// Sparse row representation of kappa K + sigma M for one basis (host, FP64).
struct SparseOp {
    int N;
    std::vector<int> ptr, col;
    std::vector<double> val;
};

SparseOp build_op(const hpadi_op1d_s& o, double kap, double sig) {
    std::vector<std::vector<std::pair<int, double>>> rows(o.N);
    auto add = [&](int i, int j, double v) {
        if (v == 0.0) return;
        rows[i].push_back({j, v});
    };
    // Robin ends (Sec. 3.3): alpha v(x) u(x) at the end adds alpha to its hat's diagonal
    for (int v : {0, o.n})
        if (o.vertex_is_hat(v)) add(o.hat_of_vertex(v), o.hat_of_vertex(v), kap * o.robin(v));
    // hat-hat
    for (int e = 0; e < o.n; ++e) {
        const double d = o.delta[e];
        const int vl = e, vr = e + 1;
        const bool hl = o.vertex_is_hat(vl), hr = o.vertex_is_hat(vr);
        const double kdg = kap / d + sig * d / 3.0, kof = -kap / d + sig * d / 6.0;
        if (hl) add(o.hat_of_vertex(vl), o.hat_of_vertex(vl), kdg);
        if (hr) add(o.hat_of_vertex(vr), o.hat_of_vertex(vr), kdg);
        if (hl && hr) {
            add(o.hat_of_vertex(vl), o.hat_of_vertex(vr), kof);
            add(o.hat_of_vertex(vr), o.hat_of_vertex(vl), kof);
        }
        // hat - W_0, W_1 (mass only)
        if (o.p >= 2) {
            const int b0 = o.bubble(0, e);
            if (hl) { add(o.hat_of_vertex(vl), b0, sig * d / 6.0); add(b0, o.hat_of_vertex(vl), sig * d / 6.0); }
            if (hr) { add(o.hat_of_vertex(vr), b0, sig * d / 6.0); add(b0, o.hat_of_vertex(vr), sig * d / 6.0); }
        }
        if (o.p >= 3) {
            const int b1 = o.bubble(1, e);
            if (hl) { add(o.hat_of_vertex(vl), b1, -sig * d / 30.0); add(b1, o.hat_of_vertex(vl), -sig * d / 30.0); }
            if (hr) { add(o.hat_of_vertex(vr), b1, sig * d / 30.0); add(b1, o.hat_of_vertex(vr), sig * d / 30.0); }
        }
        for (int m = 0; m + 2 <= o.p; ++m) {
            const int b = o.bubble(m, e);
            add(b, b, kap * k_bub(m) / d + sig * m_bub(m) * d);
            if (m + 2 <= o.p - 2) {
                const int b2 = o.bubble(m + 2, e);
                add(b, b2, sig * m_off(m) * d);
                add(b2, b, sig * m_off(m) * d);
            }
        }
    }
    SparseOp S;
    S.N = o.N;
    S.ptr.assign(o.N + 1, 0);
    for (int i = 0; i < o.N; ++i) {
        std::sort(rows[i].begin(), rows[i].end());
        // merge duplicates (hat diagonals receive two element contributions)
        std::vector<std::pair<int, double>> mr;
        for (auto& kv : rows[i]) {
            if (!mr.empty() && mr.back().first == kv.first) mr.back().second += kv.second;
            else mr.push_back(kv);
        }
        rows[i] = mr;
        S.ptr[i + 1] = S.ptr[i] + (int)mr.size();
    }
    for (int i = 0; i < o.N; ++i)
        for (auto& kv : rows[i]) {
            S.col.push_back(kv.first);
            S.val.push_back(kv.second);
        }
    return S;
}

void spmv(const SparseOp& S, const double* x, double* y) {
    for (int i = 0; i < S.N; ++i) {
        double acc = 0.0;
        for (int k = S.ptr[i]; k < S.ptr[i + 1]; ++k) acc += S.val[k] * x[S.col[k]];
        y[i] = acc;
    }
}

double entry(const SparseOp& S, int i, int j) {
    for (int k = S.ptr[i]; k < S.ptr[i + 1]; ++k)
        if (S.col[k] == j) return S.val[k];
    return 0.0;
}

// Host reverse Cholesky of an arrowhead kappa K + sigma M (Alg. 1 steps, FP64),
// in the same structured record as the device factor.  Used by the Lanczos
// interval estimate (for M^{-1}).
struct HostFactor {
    FactorLayout fl;
    std::vector<double> f;
};

bool host_factor(const hpadi_op1d_s& o, const SparseOp& S, HostFactor& H) {
    H.fl = hpadi::make_factor_layout(o.n, o.p, o.nh);
    H.f.assign(H.fl.size, 0.0);
    double* F = H.f.data();
    const int n = o.n, p = o.p;
    for (int e = 0; e < n; ++e)
        for (int pi = 0; pi < 2; ++pi) {
            const int len = pi ? (p - 1) / 2 : p / 2;
            double dup = 0.0, dhead = 1.0;
            for (int s = len - 1; s >= 0; --s) {
                const int m = pi + 2 * s;
                const int b = o.bubble(m, e);
                double a = entry(S, b, b);
                if (s + 1 < len) {
                    const double l = entry(S, b, o.bubble(m + 2, e)) / dup;
                    F[H.fl.off_link + (m + 2) * n + e] = l;
                    a -= l * l;
                }
                if (!(a > 0.0)) return false;
                const double dd = std::sqrt(a);
                F[H.fl.off_invd + m * n + e] = 1.0 / dd;
                dup = dd;
                if (s == 0) dhead = dd;
            }
            if (len > 0) {
                const int b = o.bubble(pi, e);
                if (o.vertex_is_hat(e)) F[H.fl.off_cpl + 4 * e + 2 * pi] = entry(S, o.hat_of_vertex(e), b) / dhead;
                if (o.vertex_is_hat(e + 1))
                    F[H.fl.off_cpl + 4 * e + 2 * pi + 1] = entry(S, o.hat_of_vertex(e + 1), b) / dhead;
            }
        }
    const double* C = F + H.fl.off_cpl;
    double dup = 0.0;
    for (int h = o.nh - 1; h >= 0; --h) {
        const int v = o.vertex_of_hat(h);
        double a = entry(S, h, h);
        if (v >= 1) { const int e = v - 1; a -= C[4 * e + 1] * C[4 * e + 1] + C[4 * e + 3] * C[4 * e + 3]; }
        if (v <= n - 1) { const int e = v; a -= C[4 * e] * C[4 * e] + C[4 * e + 2] * C[4 * e + 2]; }
        if (h + 1 < o.nh) {
            const int e = v;
            double b = entry(S, h, h + 1) - (C[4 * e] * C[4 * e + 1] + C[4 * e + 2] * C[4 * e + 3]);
            const double l = b / dup;
            F[H.fl.off_link0 + h + 1] = l;
            a -= l * l;
        }
        if (!(a > 0.0)) return false;
        const double dd = std::sqrt(a);
        F[H.fl.off_invd0 + h] = 1.0 / dd;
        dup = dd;
    }
    return true;
}

// x = S^{-1} b with the structured factor (corollary of Sec. 4), in place.
void host_solve(const hpadi_op1d_s& o, const HostFactor& H, double* x) {
    const double* F = H.f.data();
    const FactorLayout& fl = H.fl;
    const int n = o.n, p = o.p, nh = o.nh;
    std::vector<double> hat(nh);
    for (int h = 0; h < nh; ++h) hat[h] = x[h];
    for (int e = 0; e < n; ++e)
        for (int pi = 0; pi < 2; ++pi) {
            const int len = pi ? (p - 1) / 2 : p / 2;
            for (int s = len - 1; s >= 0; --s) {
                const int m = pi + 2 * s;
                double v = x[o.bubble(m, e)];
                if (s + 1 < len) v -= F[fl.off_link + (m + 2) * n + e] * x[o.bubble(m + 2, e)];
                x[o.bubble(m, e)] = v * F[fl.off_invd + m * n + e];
            }
            if (len > 0) {
                const double y0 = x[o.bubble(pi, e)];
                if (o.vertex_is_hat(e)) hat[o.hat_of_vertex(e)] -= F[fl.off_cpl + 4 * e + 2 * pi] * y0;
                if (o.vertex_is_hat(e + 1)) hat[o.hat_of_vertex(e + 1)] -= F[fl.off_cpl + 4 * e + 2 * pi + 1] * y0;
            }
        }
    double z = 0.0;
    for (int h = nh - 1; h >= 0; --h) {
        double v = hat[h];
        if (h + 1 < nh) v -= F[fl.off_link0 + h + 1] * z;
        z = v * F[fl.off_invd0 + h];
        hat[h] = z;
    }
    double xv = 0.0;
    for (int h = 0; h < nh; ++h) {
        double v = hat[h];
        if (h > 0) v -= F[fl.off_link0 + h] * xv;
        xv = v * F[fl.off_invd0 + h];
        hat[h] = xv;
        x[h] = xv;
    }
    for (int e = 0; e < n; ++e)
        for (int pi = 0; pi < 2; ++pi) {
            const int len = pi ? (p - 1) / 2 : p / 2;
            double prev = 0.0;
            for (int s = 0; s < len; ++s) {
                const int m = pi + 2 * s;
                double v = x[o.bubble(m, e)];
                if (s == 0) {
                    if (o.vertex_is_hat(e)) v -= F[fl.off_cpl + 4 * e + 2 * pi] * hat[o.hat_of_vertex(e)];
                    if (o.vertex_is_hat(e + 1)) v -= F[fl.off_cpl + 4 * e + 2 * pi + 1] * hat[o.hat_of_vertex(e + 1)];
                } else {
                    v -= F[fl.off_link + m * n + e] * prev;
                }
                prev = v * F[fl.off_invd + m * n + e];
                x[o.bubble(m, e)] = prev;
            }
        }
}

// Largest eigenvalue of the symmetric tridiagonal (alpha, beta) by bisection
// on the Sturm count.
double tridiag_max_eig(const std::vector<double>& al, const std::vector<double>& be) {
    const int k = (int)al.size();
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(be[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(be[i]) : 0.0);
        lo = std::min(lo, al[i] - r);
        hi = std::max(hi, al[i] + r);
    }
    auto count_above = [&](double x) {  // number of eigenvalues > x
        int c = 0;
        double q = 1.0;
        for (int i = 0; i < k; ++i) {
            const double b2 = i > 0 ? be[i - 1] * be[i - 1] : 0.0;
            q = (al[i] - x) - (i > 0 ? b2 / q : 0.0);
            if (q == 0.0) q = 1e-300;
            if (q > 0) ++c;
        }
        return c;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::fabs(hi); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count_above(mid) >= 1) lo = mid;
        else hi = mid;
    }
    return hi;
}

// Largest generalised eigenvalue of (A, M) by Lanczos in the M inner product.
bool lanczos_lmax(const hpadi_op1d_s& o, const SparseOp& A, const SparseOp& M, const HostFactor& Mf,
                  double* lmax) {
    const int N = o.N;
    std::vector<double> q(N), qprev(N, 0.0), w(N), Mq(N);
    // deterministic start vector with components of every frequency
    uint64_t st = 0x9E3779B97F4A7C15ull;
    for (int i = 0; i < N; ++i) {
        st ^= st << 13; st ^= st >> 7; st ^= st << 17;
        q[i] = ((st >> 11) * (1.0 / 9007199254740992.0)) - 0.5;
    }
    spmv(M, q.data(), Mq.data());
    double nrm = 0.0;
    for (int i = 0; i < N; ++i) nrm += q[i] * Mq[i];
    nrm = std::sqrt(nrm);
    for (int i = 0; i < N; ++i) q[i] /= nrm;
    std::vector<double> al, be;
    double beta = 0.0, last = 0.0;
    int stable = 0;
    const int kmax = std::min(600, std::max(N, 1));
    for (int k = 0; k < kmax; ++k) {
        spmv(A, q.data(), w.data());
        double alpha = 0.0;
        for (int i = 0; i < N; ++i) alpha += q[i] * w[i];
        host_solve(o, Mf, w.data());  // w = M^{-1} A q
        for (int i = 0; i < N; ++i) w[i] -= alpha * q[i] + beta * qprev[i];
        spmv(M, w.data(), Mq.data());
        double b2 = 0.0;
        for (int i = 0; i < N; ++i) b2 += w[i] * Mq[i];
        al.push_back(alpha);
        // the Ritz value is checked every 4th step (each check is a bisection over the
        // tridiagonal matrix built so far); converged after 3 checks in a row move it by at
        // most 1e-11 relative
        if (k % 4 == 3 || !(b2 > 0.0) || k + 1 == kmax) {
            const double th = tridiag_max_eig(al, be);
            if (k > 3 && std::fabs(th - last) <= 1e-11 * std::fabs(th)) {
                if (++stable >= 3) { last = th; break; }
            } else {
                stable = 0;
            }
            last = th;
        }
        if (!(b2 > 0.0)) break;
        beta = std::sqrt(b2);
        be.push_back(beta);
        qprev = q;
        for (int i = 0; i < N; ++i) q[i] = w[i] / beta;
    }
    *lmax = last;
    return std::isfinite(last) && last > 0.0;
}

// ---------------------------------------------------------------------------
// Elliptic functions and Zolotarev shifts (Alg. 2, with the cited construction).
// ---------------------------------------------------------------------------
double agm(double a, double b) {
    for (int i = 0; i < 200; ++i) {
        const double an = 0.5 * (a + b), bn = std::sqrt(a * b);
        if (std::fabs(an - bn) <= 4e-16 * an) return 0.5 * (an + bn);
        a = an;
        b = bn;
    }
    return 0.5 * (a + b);
}
double K_of_kp(double kp) { return kPi / (2.0 * agm(1.0, kp)); }
double k_of_kp(double kp) { return std::sqrt((1.0 - kp) * (1.0 + kp)); }

// dn(u, k) on [0, K]: a lattice sum of hyperbolic secants with period 2K for
// small k' (geometric convergence at ratio exp(-pi K / K')); Landen descent of
// the amplitude with reflection about K/2 otherwise.
double jacobi_dn(double u, double kp) {
    const double K = K_of_kp(kp);
    if (kp <= 0.2) {
        const double Kp = K_of_kp(k_of_kp(kp));
        const double c = kPi / (2.0 * Kp);
        double s = 0.0;
        for (int m = -8; m <= 8; ++m) {
            const double x = c * (u - 2.0 * m * K);
            if (std::fabs(x) < 700.0) s += 1.0 / std::cosh(x);
        }
        return c * s;
    }
    bool refl = false;
    if (u > 0.5 * K) {
        u = K - u;
        refl = true;
    }
    double a[64], c[64];
    double aa = 1.0, bb = kp, cc = k_of_kp(kp);
    int N = 0;
    a[0] = aa;
    c[0] = cc;
    while (std::fabs(cc) > 1e-17 * aa && N < 60) {
        const double an = 0.5 * (aa + bb), bn = std::sqrt(aa * bb), cn = 0.5 * (aa - bb);
        aa = an; bb = bn; cc = cn;
        ++N;
        a[N] = aa;
        c[N] = cc;
    }
    double phi = std::ldexp(a[N] * u, N), phi1 = phi;
    for (int i = N; i >= 1; --i) {
        phi1 = phi;
        phi = 0.5 * (phi + std::asin(c[i] / a[i] * std::sin(phi)));
    }
    const double dn = (N == 0) ? 1.0 : std::cos(phi) / std::cos(phi1 - phi);
    return refl ? kp / dn : dn;
}

int compute_shifts(const double iv[4], double tol, int J_in, int* Jout, std::vector<double>& P,
                   std::vector<double>& Q) {
    const double a = iv[0], b = iv[1], c = iv[2], d = iv[3];
    if (!(a < b && c < d) || !(d < a || b < c) || !std::isfinite(a + b + c + d)) return HPADI_EINTERVAL;
    if (!(tol > 0.0 && tol < 1.0)) return HPADI_EINVAL;
    const double gamma = std::fabs(c - a) * std::fabs(d - b) / (std::fabs(c - b) * std::fabs(d - a));
    int J = J_in > 0 ? J_in : (int)std::ceil(std::log(16.0 * gamma) * std::log(4.0 / tol) / (kPi * kPi));
    if (J < 1) J = 1;
    const double alpha = -1.0 + 2.0 * gamma + 2.0 * std::sqrt(gamma * gamma - gamma);
    const double kp = 1.0 / alpha;
    const double K = K_of_kp(kp);
    const bool sym = (c == -b && d == -a);
    P.resize(J);
    Q.resize(J);
    for (int j = 1; j <= J; ++j) {
        const double dn = jacobi_dn((2.0 * j - 1.0) * K / (2.0 * J), kp);
        if (sym) {  // T(z) = -b / z maps -alpha, -1, 1, alpha to a, b, -b, -a
            P[j - 1] = a / dn;
            Q[j - 1] = -a / dn;
        } else {  // T = psi^{-1}(phi(z)), phi(z) = cr(z; -alpha, -1, 1), psi(w) = cr(w; a, b, c)
            auto T = [&](double z) {
                const double ph = -2.0 * (z + alpha) / ((z - 1.0) * (alpha - 1.0));
                return (a * (b - c) - ph * c * (b - a)) / ((b - c) - ph * (b - a));
            };
            P[j - 1] = T(-alpha * dn);
            Q[j - 1] = T(alpha * dn);
        }
    }
    *Jout = J;
    return HPADI_OK;
}

// Smallest eigenvalue of -u'' = lambda u on [x_0, x_n] with the operator's end conditions
// (a Galerkin eigenvalue is never below it).  With u = sin(k x + phi_l), an end condition
// alpha u + du/dn = 0 fixes its phase by tan(phi) = k / alpha (Dirichlet 0, Neumann pi/2),
// and k l + phi_l + phi_r = pi closes the interval; both phases grow with k, so the
// smallest root on (0, pi / l] is found by bisection.
double continuous_lowest(const hpadi_op1d_s& o) {
    const double ell = o.x[o.n] - o.x[0];
    auto phase = [&](int end, double k) {
        return o.kind[end] == HPADI_DIRICHLET ? 0.0 : std::atan2(k, o.alpha[end]);
    };
    auto f = [&](double k) { return k * ell + phase(0, k) + phase(1, k) - kPi; };
    if (f(0.0) >= 0.0) return 0.0;  // Neumann at both ends
    double lo = 0.0, hi = kPi / ell;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (f(mid) < 0.0) lo = mid;
        else hi = mid;
    }
    return lo * lo;
}

// [lo, hi] containing the generalised eigenvalues of (kap K + sig M, M).
int interval_of(const hpadi_op1d_s& o, double kap, double sig, double out[2]) {
    if (!(kap > 0.0) || !std::isfinite(kap) || !std::isfinite(sig)) return HPADI_EINVAL;
    if (sig < 0.0 || (o.k_singular() && !(sig > 0.0))) return HPADI_ESINGULAR;
    const double lo = kap * continuous_lowest(o) + sig;
    if (!(lo > 0.0)) return HPADI_ESINGULAR;
    if (o.N == 0) return HPADI_EINVAL;
    const double dmin = *std::min_element(o.delta.begin(), o.delta.end());
    const double dmax = *std::max_element(o.delta.begin(), o.delta.end());
    if (o.n >= 16 && dmax - dmin <= 1e-12 * dmax && o.alpha[0] == 0.0 && o.alpha[1] == 0.0) {
        // Upper end from the elements: x^T K x = sum_e x_e^T K_e x_e and likewise for M, so the
        // largest eigenvalue of (K, M) is at most the largest element-level one (a Dirichlet
        // constraint only lowers it).  An element of width delta has the pair (K_1/delta,
        // delta M_1) of the unit element, eigenvalues lambda(K_1, M_1)/delta^2: one Lanczos run
        // of size p + 1.  On uniform meshes of 16 or more elements it is within 0.7% of the
        // assembled eigenvalue (0.004% at n = p = 64); coarser or graded meshes, where the
        // boundary elements make it looser (up to 30% measured), take the assembled Lanczos.
        hpadi_op1d_s u;
        u.n = 1;
        u.p = o.p;
        u.bc = 3;
        u.kind[0] = u.kind[1] = HPADI_NEUMANN;
        u.x = {0.0, 1.0};
        u.delta = {1.0};
        u.nh = 2;
        u.N = u.nh + (o.p - 1);
        u.Nleg = o.p + 1;
        SparseOp K1 = build_op(u, 1.0, 0.0);
        SparseOp M1 = build_op(u, 0.0, 1.0);
        HostFactor M1f;
        if (!host_factor(u, M1, M1f)) return HPADI_ENOTSPD;
        double lk = 0.0;
        if (!lanczos_lmax(u, K1, M1, M1f, &lk)) return HPADI_EINVAL;
        out[0] = lo;
        out[1] = std::max((kap * lk / (dmin * dmin) + sig) * (1.0 + 1e-6), lo * 1.0000001);
        return HPADI_OK;
    }
    SparseOp A = build_op(o, kap, sig);
    SparseOp M = build_op(o, 0.0, 1.0);
    HostFactor Mf;
    if (!host_factor(o, M, Mf)) return HPADI_ENOTSPD;
    double lmax = 0.0;
    if (!lanczos_lmax(o, A, M, Mf, &lmax)) return HPADI_EINVAL;
    out[0] = lo;
    out[1] = std::max(lmax * 1.01, lo * 1.0000001);
    return HPADI_OK;
}

}  // namespace

// ===========================================================================
// Plan.
// ===========================================================================

namespace {

using hpadi_host::dmalloc;

int make_dim(DimHost& D, const hpadi_op1d_s& o) {
    D.op = o;
    const int n = o.n, p = o.p, N = o.N;
    const int ts = p + 4;
    std::vector<double> h(2 * n + N + 3 * ts, 0.0);
    for (int e = 0; e < n; ++e) {
        h[e] = o.delta[e];
        h[n + e] = 1.0 / o.delta[e];
    }
    SparseOp M = build_op(o, 0.0, 1.0);
    for (int i = 0; i < N; ++i) h[2 * n + i] = entry(M, i, i);
    double* tab = h.data() + 2 * n + N;
    for (int m = 0; m < ts; ++m) {
        tab[m] = k_bub(m);
        tab[ts + m] = m_bub(m);
        tab[2 * ts + m] = m_off(m);
    }
    if (dmalloc(&D.buf, h.size()) != hipSuccess) return HPADI_ENOMEM;
    if (hipMemcpy(D.buf, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return HPADI_EHIP;
    std::vector<float> t32(3 * ts);
    for (int i = 0; i < 3 * ts; ++i) t32[i] = (float)tab[i];
    if (dmalloc(&D.tab32, t32.size()) != hipSuccess) return HPADI_ENOMEM;
    if (hipMemcpy(D.tab32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return HPADI_EHIP;
    D.dev.n = n;
    D.dev.p = p;
    D.dev.nh = o.nh;
    D.dev.N = N;
    D.dev.Nleg = o.Nleg;
    D.dev.bc = o.bc;
    D.dev.rob0 = (o.bc & 1) ? o.alpha[0] : 0.0;
    D.dev.rob1 = (o.bc & 2) ? o.alpha[1] : 0.0;
    D.dev.delta = D.buf;
    D.dev.invdelta = D.buf + n;
    D.dev.mdiag = D.buf + 2 * n;
    D.dev.tab64 = D.buf + 2 * n + N;
    D.dev.tab32 = D.tab32;
    D.dev.tabstride = ts;
    D.hpad = (o.nh + 7) / 8 * 8;
    D.Npad = D.hpad + (p - 1) * n;
    D.uniform = n % 4 == 0;
    for (int e = 1; e < n && D.uniform; ++e) D.uniform = o.delta[e] == o.delta[0];
    return HPADI_OK;
}

void free_dim(DimHost& D) {
    if (D.buf) hipFree(D.buf);
    if (D.tab32) hipFree(D.tab32);
    D.buf = nullptr;
    D.tab32 = nullptr;
}

bool same_op(const hpadi_op1d_s& a, const hpadi_op1d_s& b) {
    return a.n == b.n && a.p == b.p && a.bc == b.bc && a.x == b.x && a.alpha[0] == b.alpha[0] &&
           a.alpha[1] == b.alpha[1];
}

int factor_family(DimHost& D, const std::vector<double>& kap, const std::vector<double>& sig, FactorLayout& fl,
                  double** f64, int* status, hipStream_t s) {
    const int nf = (int)kap.size();
    fl = hpadi::make_factor_layout(D.op.n, D.op.p, D.op.nh);
    if (dmalloc(f64, (size_t)nf * fl.stride) != hipSuccess) return HPADI_ENOMEM;
    if (hipMemsetAsync(*f64, 0, (size_t)nf * fl.stride * sizeof(double), s) != hipSuccess) return HPADI_EHIP;
    double* ks = nullptr;
    if (dmalloc(&ks, 2 * nf) != hipSuccess) return HPADI_ENOMEM;
    std::vector<double> h(kap);
    h.insert(h.end(), sig.begin(), sig.end());
    int rc = HPADI_OK;
    if (hipMemcpyAsync(ks, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(status, 0, nf * sizeof(int), s) != hipSuccess ||
        hpadi::launch_factor(D.dev, nf, ks, ks + nf, *f64, nullptr, fl.stride, status, s) != hipSuccess) {
        rc = HPADI_EHIP;
    }
    std::vector<int> st(nf, 0);
    if (rc == HPADI_OK && (hipMemcpyAsync(st.data(), status, nf * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
                           hipStreamSynchronize(s) != hipSuccess))
        rc = HPADI_EHIP;
    hipFree(ks);
    if (rc != HPADI_OK) return rc;
    for (int v : st)
        if (v) return HPADI_ENOTSPD;
    return HPADI_OK;
}

void family_free(ShiftFamily& F) {
    if (F.facy64 != F.facx64 && F.facx64) hipFree(F.facx64);
    if (F.facy64) hipFree(F.facy64);
    if (F.coefy != F.coefx && F.coefx) hipFree(F.coefx);
    if (F.coefy) hipFree(F.coefy);
    if (F.ptabx) hipFree(F.ptabx);
    if (F.ptaby) hipFree(F.ptaby);
    if (F.status) hipFree(F.status);
    F = ShiftFamily{};
}

void plan_free(hpadi_plan_s* P) {
    if (!P) return;
    for (ShiftFamily& F : P->fam) family_free(F);
    for (void* q : {P->Wk, P->Gt, (void*)P->T64, (void*)P->T12, (void*)P->R64,
                    (void*)P->H, (void*)P->acc, (void*)P->part})
        if (q) hipFree(q);
    if (P->acc_host) hipHostFree(P->acc_host);
    for (auto& r : P->recs) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (hipEvent_t e : P->phase_ev) hipEventDestroy(e);
    free_dim(P->dx);
    free_dim(P->dy);
    delete P;
}

hpadi::Layout user_layout(const hpadi_plan_s* P, long ld) {
    hpadi::Layout L{};
    L.ld = ld;
    L.panel = 0;
    L.nhr = P->dx.op.nh;
    L.nhc = P->dy.op.nh;
    return L;
}

// Workgroups that share cache lines of a panel layout get an XCD-aware order (the
// workgroups sharing each line run on one XCD in consecutive dispatch slots): a row pass
// whose workgroup rows are narrower than a 128-byte line (lines per workgroup x panel
// width x element size < 128), a column pass whose workgroup covers fewer lines than a
// panel holds (the workgroups of one panel share every sector).
hpadi::SweepArgs with_xcd_group(hpadi::SweepArgs a, bool column, int tin) {
    const int w = a.lpb * a.lin.panel * tin;
    if (column) a.xcd_group = (a.lin.panel > 0 && a.lpb > 0 && a.lpb < a.lin.panel) ? a.lin.panel / a.lpb : 1;
    else a.xcd_group = (a.lin.panel > 0 && w > 0 && w < 128) ? 128 / w : 1;
    return a;
}

// Launch a half-sweep, bracketed by timing events when measurement is enabled.
// kind: 0 full column sweep, 1 full row sweep, 2 the others (transforms, the last
// column solve, the final solve), plus 3 when the sweep stores FP64; bytes:
// algorithmic HBM bytes.
int timed_sweep(hpadi_plan_s* P, bool column, const hpadi::SweepArgs& a, int mode, int tin, int tout, int kind,
                double bytes) {
    hpadi_plan_s::Rec* r = nullptr;
    if (P->timing && P->nrec < 65536) {
        if (P->nrec == P->recs.size()) {
            hpadi_plan_s::Rec nr{};
            if (hipEventCreate(&nr.a) != hipSuccess || hipEventCreate(&nr.b) != hipSuccess) return HPADI_EHIP;
            P->recs.push_back(nr);
        }
        r = &P->recs[P->nrec++];
        // FP64 storage (either side of the sweep 8-byte) goes to kinds 3..5
        r->kind = kind + ((tin == 8 && tout == 8) || (mode != hpadi::SWEEP_TRANSFORM && mode != hpadi::SWEEP_FINAL && tin == 8) ? 3 : 0);
        r->bytes = bytes;
        if (hipEventRecord(r->a, P->stream) != hipSuccess) return HPADI_EHIP;
    }
    const DimDev& d = column ? P->dx.dev : P->dy.dev;
    if (hpadi::launch_sweep(d, with_xcd_group(a, column, tin), mode, tin, tout, column, P->stream) != hipSuccess)
        return HPADI_EHIP;
    if (r && hipEventRecord(r->b, P->stream) != hipSuccess) return HPADI_EHIP;
    return HPADI_OK;
}

// Arguments common to every sweep along one direction; j selects the shifted factor of
// family F (j = J: the mass factor alone, for the transforms and the final solve).
hpadi::SweepArgs sweep_args(const hpadi_plan_s* P, const ShiftFamily& F, bool column, int j) {
    hpadi::SweepArgs a{};
    const DimHost& D = column ? P->dx : P->dy;
    const DimHost& O = column ? P->dy : P->dx;
    const FactorLayout& fl = column ? P->flx : P->fly;
    const double* fac = column ? F.facx64 : F.facy64;
    const double* coef = column ? F.coefx : F.coefy;
    a.nlines = O.op.N;
    a.nh_lines = O.op.nh;
    a.hpad_lines = O.hpad;
    a.fl = fl;
    a.facS = fac + (size_t)j * fl.stride;
    a.facM = fac + (size_t)F.J * fl.stride;
    a.coef = coef ? coef + (size_t)j * D.op.p * 8 : nullptr;
    const double* ptab = column ? F.ptabx : F.ptaby;
    a.ptab = ptab ? ptab + (size_t)(j < F.J ? j : 0) * D.op.p * 16 : nullptr;
    a.lpb = column ? P->lpb_col : P->lpb_row;
    // byte offsets of 8-byte entries must fit the 32-bit offsets of the uniform kernel
    a.idx32 = P->nint < (size_t(1) << 29) ? 1 : 0;
    return a;
}

// Arguments of the transform passes (row: R -> T64, reading the caller's row-major R
// along its rows; column: T64 -> G~ in ts bytes).
hpadi::SweepArgs transform_row_args(const hpadi_plan_s* P, const double* R, long ldr) {
    hpadi::SweepArgs r = sweep_args(P, P->first(), false, P->first().J);
    r.in = R;
    r.lin = user_layout(P, ldr);
    if ((double)ldr * P->dx.op.N >= 536870912.0) r.idx32 = 0;
    r.out = P->T64;
    r.lout = P->lint;
    return r;
}
hpadi::SweepArgs transform_col_args(const hpadi_plan_s* P) {
    hpadi::SweepArgs c = sweep_args(P, P->first(), true, P->first().J);
    c.in = P->T64;
    c.lin = P->lint;
    c.out = P->Gt;
    c.lout = P->lint;
    return c;
}
// Arguments of the ADI half-sweeps of iteration j (row: shift q_j; column: p_{j+1}).
hpadi::SweepArgs adi_row_args(const hpadi_plan_s* P, const ShiftFamily& F, int j) {
    hpadi::SweepArgs r = sweep_args(P, F, false, j);
    r.in = j == 0 ? P->Gt : P->Wk;
    r.lin = P->lint;
    r.g = P->Gt;
    r.lg = P->lint;
    r.out = P->Wk;
    r.lout = P->lint;
    r.kappa = P->ky;
    r.tau = P->sy + F.Q[j];
    return r;
}
hpadi::SweepArgs adi_col_args(const hpadi_plan_s* P, const ShiftFamily& F, int j) {
    hpadi::SweepArgs c = sweep_args(P, F, true, j);
    c.in = P->Wk;
    c.lin = P->lint;
    c.g = P->Gt;
    c.lg = P->lint;
    c.out = P->Wk;
    c.lout = P->lint;
    c.kappa = P->kx;
    c.tau = j + 1 == F.J ? 0.0 : P->sx - F.P[j + 1];
    return c;
}
// Arguments of the final mass solve U (+)= L^{-1} w.
hpadi::SweepArgs final_args(const hpadi_plan_s* P, double* U, long ldu, bool accumulate) {
    hpadi::SweepArgs f = sweep_args(P, P->first(), false, P->first().J);
    f.in = P->Wk;
    f.lin = P->lint;
    f.out = U;
    f.lout = user_layout(P, ldu);
    if ((double)ldu * P->dx.op.N >= 536870912.0) f.idx32 = 0;
    f.accumulate = accumulate ? 1 : 0;
    return f;
}

// G~ = V^{-T} R L^{-1} (mass factors M^x = V^T V, M^y = L^T L): the two sides commute, so
// the row transform goes first and reads R along its contiguous rows.
int transform_rhs(hpadi_plan_s* P, const double* R, long ldr, int ts) {
    const double dofs = (double)P->dx.op.N * P->dy.op.N;
    int rc = timed_sweep(P, false, transform_row_args(P, R, ldr), hpadi::SWEEP_TRANSFORM, 8, 8, 2, dofs * 16.0);
    if (rc != HPADI_OK) return rc;
    return timed_sweep(P, true, transform_col_args(P), hpadi::SWEEP_TRANSFORM, 8, ts, 2, dofs * (8.0 + ts));
}

// Arguments of the last column pass of family F (the solve that ends the ADI loop);
// norms: add the squared norm of the round's correction in the ADI lemma's norm,
// ||V delta L^T||_F^2, to P->acc[0].
hpadi::SweepArgs last_col_args(const hpadi_plan_s* P, const ShiftFamily& F, bool norms) {
    hpadi::SweepArgs c = adi_col_args(P, F, F.J - 1);
    c.norm_acc = norms ? P->acc : nullptr;
    return c;
}

// Alg. 2 solve loop in balanced coordinates with the shifts of family F, from G~ (in
// P->Gt) to U (user layout): U = u or U += u (accumulate); norms as in last_col_args.
int run_adi(hpadi_plan_s* P, const ShiftFamily& F, int ts, double* U, long ldu, bool accumulate, bool norms) {
    const double dofs = (double)P->dx.op.N * P->dy.op.N;
    for (int j = 0; j < F.J; ++j) {
        int rc = timed_sweep(P, false, adi_row_args(P, F, j), hpadi::SWEEP_FULL, ts, ts, 1, dofs * 3.0 * ts);
        if (rc != HPADI_OK) return rc;
        const bool last = j + 1 == F.J;
        rc = timed_sweep(P, true, last ? last_col_args(P, F, norms) : adi_col_args(P, F, j),
                         last ? hpadi::SWEEP_SOLVE : hpadi::SWEEP_FULL, ts, ts, last ? 2 : 0,
                         dofs * (last ? 2.0 : 3.0) * ts);
        if (rc != HPADI_OK) return rc;
    }
    return timed_sweep(P, false, final_args(P, U, ldu, accumulate), hpadi::SWEEP_FINAL, ts, 8, 2,
                       dofs * (ts + (accumulate ? 16.0 : 8.0)));
}

// Error bound of the ADI lemma (Sec. 5.1) after a refinement round whose shift family
// has tolerance eps: with e the error before the round and delta its correction,
// ||e - delta|| <= eps ||e|| gives ||U* - U_new|| <= f ||delta||, f = eps / (1 - eps);
// and ||U*|| >= ||U_new|| - f ||delta|| >= | ||U_old|| - ||delta|| | - f ||delta||.
// d2 = ||delta||^2, u2 = ||U_old||^2, both in the lemma's norm ||V X L^T||_F.  Returns
// the bound on ||U* - U_new|| / ||U*|| (infinity when the denominator is not positive).
// The lemma holds in exact arithmetic; once the correction is rounding noise the bound
// can fall below what FP64 certifies, so it is never reported below 16 unit roundoffs.
constexpr double kRoundingFloor = 16.0 * 1.1102230246251565e-16;
double lemma_bound(double eps, double d2, double u2) {
    const double nd = std::sqrt(std::max(d2, 0.0)), nu = std::sqrt(std::max(u2, 0.0));
    if (!std::isfinite(nd) || !std::isfinite(nu)) return std::numeric_limits<double>::infinity();
    if (nd == 0.0) return kRoundingFloor;
    const double f = eps / (1.0 - eps);
    const double lo = std::fabs(nu - nd) - f * nd;
    return lo > 0.0 ? std::max(f * nd / lo, kRoundingFloor) : std::numeric_limits<double>::infinity();
}

// T1 = U M_y, T2 = U A_y (row operators, FP64), interleaved as (T1, T2) pairs in P->T12
// (the residual reads both at every tap: one 16-byte load).
int row_products(hpadi_plan_s* P, const double* U, long ldu) {
    hpadi::OpApply a{};
    a.in = U;
    a.in_sl = ldu;
    a.in_sp = 1;
    a.out1 = P->T12;
    a.o1_sl = 2 * P->ldw;
    a.o1_sp = 2;
    a.k1 = 0.0;
    a.t1 = 1.0;
    a.out2 = P->T12 + 1;
    a.o2_sl = 2 * P->ldw;
    a.o2_sp = 2;
    a.k2 = P->ky;
    a.t2 = P->sy;
    a.nlines = P->dx.op.N;
    return hpadi::launch_op_apply(P->dy.dev, a, false, P->stream) == hipSuccess ? HPADI_OK : HPADI_EHIP;
}

int ensure_fp64_work(hpadi_plan_s* P) {
    const size_t cnt = (size_t)P->dx.op.N * P->ldw;
    if (!P->T12 && dmalloc(&P->T12, 2 * cnt) != hipSuccess) return HPADI_ENOMEM;
    return HPADI_OK;
}

// r = G - A U in FP64 into P->R64; P->acc[2..3] get the diagonal-mass weighted squares
// of r and G, P->acc[4] the squared norm of U in the ADI lemma's norm.
int residual_into_r64(hpadi_plan_s* P, const double* G, long ldg, const double* U, long ldu) {
    hipStream_t s = P->stream;
    int rc = row_products(P, U, ldu);
    if (rc != HPADI_OK) return rc;
    if (hpadi::launch_zero_f64(P->acc + 2, 3, 1, 3, s) != hipSuccess) return HPADI_EHIP;
    hpadi::Residual r{};
    r.G = G;
    r.g_ld = ldg;
    r.T1 = P->T12;
    r.T2 = nullptr;
    r.t_ld = P->ldw;
    r.r64 = P->R64;
    r.r64_ld = P->ldw;
    r.ax_k = P->kx;
    r.ax_t = P->sx;
    r.alpha = 1.0;
    r.beta = -1.0;
    r.ncols = P->dy.op.N;
    r.norm_acc = P->acc + 2;
    r.wcol = P->dy.dev.mdiag;
    r.U = U;
    r.u_ld = ldu;
    r.partials = P->part;
    return hpadi::launch_residual(P->dx.dev, r, s) == hipSuccess ? HPADI_OK : HPADI_EHIP;
}

// A refinement schedule with a fixed number of rounds (nfp32 rounds with FP32 storage,
// then nfp64 FP64 rounds) and no host synchronisation or memset node, so that it can be
// captured into a graph.  P->acc[0] and P->acc[4] hold the squared norms of the last
// round's correction and of U before it (the inputs of lemma_bound)
// and of U for the error bound.  Work arrays must already exist.
int enqueue_fixed_solve(hpadi_plan_s* P, const double* G, long ldg, double* U, long ldu, int nfp32, int nfp64) {
    hipStream_t s = P->stream;
    const int rounds = nfp32 + nfp64;
    for (int k = 1; k <= rounds; ++k) {
        const int ts = k <= nfp32 ? 4 : 8;
        int rc;
        if (k > 1 && (rc = residual_into_r64(P, G, ldg, U, ldu)) != HPADI_OK) return rc;
        // round 1 starts from U = 0
        if (hpadi::launch_zero_f64(P->acc, k == 1 ? 5 : 1, 1, k == 1 ? 5 : 1, s) != hipSuccess) return HPADI_EHIP;
        if ((rc = transform_rhs(P, k == 1 ? G : P->R64, k == 1 ? ldg : P->ldw, ts)) != HPADI_OK) return rc;
        // the first round writes U (no zeroing pass), later rounds add to it; FP32 rounds
        // take the first shift family, FP64 rounds the refinement family
        if ((rc = run_adi(P, k <= nfp32 ? P->first() : P->refine(), ts, U, ldu, k > 1, true)) != HPADI_OK) return rc;
    }
    return HPADI_OK;
}

}  // namespace

namespace {

// One launch of a batch schedule.
struct BatchStep {
    int kind = 0;        // 0 grouped sweep, 1 single sweep, 2 residual of one instance, 4 zero all accumulators
    int phase = 0;       // steps of one phase touch disjoint instances and may run concurrently
    hpadi::GroupLaunch g{};
    size_t task_off = 0;
    int inst = -1;
    hpadi::SweepArgs a{};
    int mode = 0, tin = 8, tout = 8;
    bool column = false;
};

// Appends the half-sweeps of one kind for the listed instances: those the uniform-mesh
// kernel takes are grouped by (chain length, lines per workgroup, n) into one launch each,
// the others are launched one by one.
void add_sweeps(std::vector<BatchStep>& steps, std::vector<hpadi::GroupTask>& table,
                const std::vector<hpadi_plan>& plans, const std::vector<std::pair<int, hpadi::SweepArgs>>& items,
                int mode, int tin, int tout, bool column) {
    // (chain length, lines per workgroup, n) -> item indices: equal n keeps the workgroup
    // size of a launch exact
    std::vector<std::pair<std::array<int, 3>, std::vector<int>>> groups;
    for (size_t k = 0; k < items.size(); ++k) {
        const hpadi_plan_s* P = plans[items[k].first];
        const hpadi::DimDev& d = column ? P->dx.dev : P->dy.dev;
        const hpadi::SweepArgs& a = items[k].second;
        if (a.nlines <= 0) continue;
        const bool uni = a.ptab && a.idx32 && (a.lpb == 4 || a.lpb == 8 || a.lpb == 16) &&
                         hpadi::sweep_uni_available(d, a.lpb) &&
                         (int)hpadi::sweep_uni_threads(d, a.lpb) <= hpadi::sweep_uni_max_threads(d.p / 2);
        if (!uni) {
            BatchStep st;
            st.kind = 1;
            st.inst = items[k].first;
            st.a = a;
            st.mode = mode;
            st.tin = tin;
            st.tout = tout;
            st.column = column;
            steps.push_back(st);
            continue;
        }
        const std::array<int, 3> key{d.p / 2, a.lpb, d.n};
        auto it = std::find_if(groups.begin(), groups.end(), [&](const auto& g) { return g.first == key; });
        if (it == groups.end()) groups.push_back({key, {(int)k}});
        else it->second.push_back((int)k);
    }
    for (auto& grp : groups) {
        BatchStep st;
        st.kind = 0;
        st.task_off = table.size();
        hpadi::GroupLaunch& g = st.g;
        g.mode = mode;
        g.tin = tin;
        g.tout = tout;
        g.cl = grp.first[0];
        g.lw = grp.first[1];
        g.column = column;
        int blocks = 0, threads = 0;
        for (int k : grp.second) {
            const hpadi_plan_s* P = plans[items[k].first];
            const hpadi::DimDev& d = column ? P->dx.dev : P->dy.dev;
            hpadi::GroupTask t{};
            t.d = d;
            t.a = items[k].second;
            t.block0 = blocks;
            t.nblk = (t.a.hpad_lines + t.a.nlines - t.a.nh_lines + g.lw - 1) / g.lw;
            blocks += t.nblk;
            threads = std::max(threads, (int)hpadi::sweep_uni_threads(d, g.lw));
            table.push_back(t);
        }
        size_t lds = 0;
        for (int k : grp.second) {
            const hpadi_plan_s* P = plans[items[k].first];
            lds = std::max(lds, hpadi::sweep_uni_lds_bytes(column ? P->dx.dev : P->dy.dev, g.lw, threads, mode));
        }
        g.ntasks = (int)grp.second.size();
        g.nblocks = blocks;
        g.threads = threads;
        g.lds_bytes = lds;
        steps.push_back(st);
    }
}

}  // namespace

// ===========================================================================
// Batched solves: independent plans replayed as one graph.
// ===========================================================================
struct hpadi_batch_s {
    int count = 0;
    std::vector<hpadi_plan> plans;
    std::vector<const double*> G;
    std::vector<double*> U;
    std::vector<int> ldg, ldu, lw;
    hipStream_t origin = nullptr;
    bool own_origin = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // capture lanes besides the origin stream (default priority): the steps of one phase
    // are spread over them, forked from and joined back into the origin stream
    static constexpr int kLanes = 4;
    hipStream_t side[kLanes - 1] = {};
    hipEvent_t fork = nullptr, join[kLanes - 1] = {};
    hpadi::GroupTask* table = nullptr;   // device task tables of the grouped launches
    int nlaunch = 0;                     // launches in the graph
    double tol = 0.0;
    double** acc_ptrs = nullptr;         // device array of the plans' accumulators
    double* acc_all = nullptr;           // device [count][2]
    double* acc_host = nullptr;          // pinned copy
    ~hpadi_batch_s() {
        if (origin) (void)hipStreamSynchronize(origin);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hpadi_plan p : plans) hpadi_plan_destroy(p);
        if (own_origin) (void)hipStreamDestroy(origin);
        for (hipStream_t q : side)
            if (q) (void)hipStreamDestroy(q);
        for (hipEvent_t e : join)
            if (e) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        (void)hipFree(acc_ptrs);
        (void)hipFree(acc_all);
        (void)hipFree(table);
        if (acc_host) (void)hipHostFree(acc_host);
    }
};

// ===========================================================================
// C ABI.
// ===========================================================================
extern "C" {

const char* hpadi_strerror(int st) {
    switch (st) {
        case HPADI_OK: return "ok";
        case HPADI_EINVAL: return "invalid argument";
        case HPADI_ENOTSPD: return "factorisation met a non-positive pivot";
        case HPADI_ESINGULAR: return "singular problem (Neumann with omega^2 <= 0)";
        case HPADI_EINTERVAL: return "spectral intervals are empty or not disjoint";
        case HPADI_ENOCONV: return "tolerance not reached";
        case HPADI_EHIP: return "HIP runtime error";
        case HPADI_ENOMEM: return "out of memory";
        default: return "unknown status";
    }
}

int hpadi_op1d_create(int n, int p, double a, double b, const double* breaks, int bc, hpadi_op1d* out) {
    if (bc != HPADI_DIRICHLET && bc != HPADI_NEUMANN) {
        if (out) *out = nullptr;
        return HPADI_EINVAL;
    }
    return hpadi_op1d_create_ex(n, p, a, b, breaks, bc, bc, 0.0, 0.0, out);
}

int hpadi_op1d_create_ex(int n, int p, double a, double b, const double* breaks, int bc_left, int bc_right,
                         double alpha_left, double alpha_right, hpadi_op1d* out) {
    if (!out) return HPADI_EINVAL;
    *out = nullptr;
    const int kinds[2] = {bc_left, bc_right};
    const double alphas[2] = {alpha_left, alpha_right};
    for (int i = 0; i < 2; ++i) {
        if (kinds[i] != HPADI_DIRICHLET && kinds[i] != HPADI_NEUMANN && kinds[i] != HPADI_ROBIN) return HPADI_EINVAL;
        if (kinds[i] == HPADI_ROBIN && !(alphas[i] >= 0.0 && std::isfinite(alphas[i]))) return HPADI_EINVAL;
    }
    if (n < 1 || p < 1 || n > 1000000 || p > 129) return HPADI_EINVAL;
    hpadi_op1d_s* o = new (std::nothrow) hpadi_op1d_s;
    if (!o) return HPADI_ENOMEM;
    o->n = n;
    o->p = p;
    o->bc = (kinds[0] != HPADI_DIRICHLET ? 1 : 0) | (kinds[1] != HPADI_DIRICHLET ? 2 : 0);
    for (int i = 0; i < 2; ++i) {
        o->kind[i] = kinds[i];
        o->alpha[i] = kinds[i] == HPADI_ROBIN ? alphas[i] : 0.0;
    }
    o->x.resize(n + 1);
    if (breaks) {
        for (int i = 0; i <= n; ++i) o->x[i] = breaks[i];
    } else {
        if (!(b > a)) { delete o; return HPADI_EINVAL; }
        for (int i = 0; i <= n; ++i) o->x[i] = a + (b - a) * (double)i / (double)n;
        o->x[n] = b;
    }
    o->delta.resize(n);
    for (int e = 0; e < n; ++e) {
        o->delta[e] = o->x[e + 1] - o->x[e];
        if (!(o->delta[e] > 0.0) || !std::isfinite(o->delta[e])) { delete o; return HPADI_EINVAL; }
    }
    o->nh = n - 1 + (o->bc & 1) + ((o->bc >> 1) & 1);
    o->N = o->nh + n * (p - 1);
    o->Nleg = (p + 1) * n;
    if (o->N < 1) { delete o; return HPADI_EINVAL; }
    *out = o;
    return HPADI_OK;
}

int hpadi_op1d_dims(hpadi_op1d op, int* N, int* Nleg) {
    if (!op) return HPADI_EINVAL;
    if (N) *N = op->N;
    if (Nleg) *Nleg = op->Nleg;
    return HPADI_OK;
}

int hpadi_op1d_export(hpadi_op1d op, double* K, double* M, double* T) {
    if (!op) return HPADI_EINVAL;
    const int N = op->N, L = op->Nleg, n = op->n;
    auto dense = [&](const SparseOp& S, double* out) {
        std::memset(out, 0, sizeof(double) * (size_t)N * N);
        for (int i = 0; i < N; ++i)
            for (int k = S.ptr[i]; k < S.ptr[i + 1]; ++k) out[(size_t)i * N + S.col[k]] = S.val[k];
    };
    if (K) dense(build_op(*op, 1.0, 0.0), K);
    if (M) dense(build_op(*op, 0.0, 1.0), M);
    if (T) {
        std::memset(T, 0, sizeof(double) * (size_t)N * L);
        for (int e = 0; e < n; ++e) {
            const double d = op->delta[e];
            if (op->vertex_is_hat(e)) {  // left vertex: (P_0 - P_1)/2 on e
                const int h = op->hat_of_vertex(e);
                T[(size_t)h * L + e] += d / 2.0;
                T[(size_t)h * L + n + e] += -d / 6.0;
            }
            if (op->vertex_is_hat(e + 1)) {  // right vertex: (P_0 + P_1)/2 on e
                const int h = op->hat_of_vertex(e + 1);
                T[(size_t)h * L + e] += d / 2.0;
                T[(size_t)h * L + n + e] += d / 6.0;
            }
            for (int m = 0; m + 2 <= op->p; ++m) {
                const int b = op->bubble(m, e);
                T[(size_t)b * L + m * n + e] = d / ((2.0 * m + 1) * (2.0 * m + 3));
                T[(size_t)b * L + (m + 2) * n + e] = -d / ((2.0 * m + 3) * (2.0 * m + 5));
            }
        }
    }
    return HPADI_OK;
}

void hpadi_op1d_destroy(hpadi_op1d op) { delete op; }

int hpadi_interval(hpadi_op1d op, double omega2, double out[2]) {
    if (!op || !out) return HPADI_EINVAL;
    return interval_of(*op, 1.0, omega2 / 2.0, out);
}

int hpadi_shifts(const double iv[4], double tol, int J_in, int* J, double* p, double* q, int maxJ) {
    if (!iv || !J) return HPADI_EINVAL;
    std::vector<double> P, Q;
    int Jc = 0;
    const int rc = compute_shifts(iv, tol, J_in, &Jc, P, Q);
    if (rc != HPADI_OK) return rc;
    *J = Jc;
    if (p || q) {
        if (Jc > maxJ) return HPADI_EINVAL;
        for (int j = 0; j < Jc; ++j) {
            if (p) p[j] = P[j];
            if (q) q[j] = Q[j];
        }
    }
    return HPADI_OK;
}

// Shifts (Alg. 2) for tolerance eps and the reverse Cholesky factors (Alg. 1) of the
// shifted 1D operators of both axes, plus the uniform-mesh coefficient tables.
int build_family(hpadi_plan_s* P, const hpadi_op1d_s& x, const hpadi_op1d_s& y, double eps, ShiftFamily& F) {
    int rc;
    F.eps = eps;
    if ((rc = compute_shifts(P->interval, eps, 0, &F.J, F.P, F.Q)) != HPADI_OK) return rc;
    const int J = F.J;
    if (dmalloc(&F.status, 2 * J + 2) != hipSuccess) return HPADI_ENOMEM;
    // y family: ky K_y + (sy + p_j) M_y for j = 1..J, then M_y
    std::vector<double> ky(J + 1, P->ky), sy(J + 1);
    for (int j = 0; j < J; ++j) sy[j] = P->sy + F.P[j];
    ky[J] = 0.0;
    sy[J] = 1.0;
    if ((rc = factor_family(P->dy, ky, sy, P->fly, &F.facy64, F.status, P->stream)) != HPADI_OK) return rc;
    // x family: kx K_x + (sx - q_j) M_x, then M_x; shared with y when operators and shifts coincide
    bool shared = same_op(x, y) && P->kx == P->ky && P->sx == P->sy;
    for (int j = 0; j < J && shared; ++j) shared = (-F.Q[j] == F.P[j]);
    F.shared = shared;
    if (shared) {
        F.facx64 = F.facy64;
        P->flx = P->fly;
    } else {
        std::vector<double> kx(J + 1, P->kx), sx(J + 1);
        for (int j = 0; j < J; ++j) sx[j] = P->sx - F.Q[j];
        kx[J] = 0.0;
        sx[J] = 1.0;
        if ((rc = factor_family(P->dx, kx, sx, P->flx, &F.facx64, F.status + J + 1, P->stream)) != HPADI_OK) return rc;
    }
    // per-degree coefficient records for the uniform-mesh fast path
    auto tables = [&](DimHost& D, double* fac, const FactorLayout& fl, double** out) -> int {
        if (!D.uniform || D.op.p < 2) return HPADI_OK;
        if (dmalloc(out, (size_t)(J + 1) * D.op.p * 8) != hipSuccess) return HPADI_ENOMEM;
        return hpadi::launch_coef_tables(D.dev, J + 1, fac, fl.stride, fac + (size_t)J * fl.stride, fl, *out,
                                         P->stream) == hipSuccess ? HPADI_OK : HPADI_EHIP;
    };
    if ((rc = tables(P->dy, F.facy64, P->fly, &F.coefy)) != HPADI_OK) return rc;
    if (shared) F.coefx = F.coefy;
    else if ((rc = tables(P->dx, F.facx64, P->flx, &F.coefx)) != HPADI_OK) return rc;
    // folded per-pass records: row pass j (S_y(w/2 + p_j), product tau = w/2 + q_j) and
    // column pass j (S_x(w/2 - q_j), product tau = w/2 - p_{j+1}; none after the last)
    auto ptables = [&](DimHost& D, double* fac, const FactorLayout& fl, const std::vector<double>& tau,
                       double kappa, double** out) -> int {
        if (!D.uniform || D.op.p < 2) return HPADI_OK;
        if (dmalloc(out, (size_t)J * D.op.p * 16) != hipSuccess) return HPADI_ENOMEM;
        double* td = nullptr;
        if (dmalloc(&td, J) != hipSuccess) return HPADI_ENOMEM;
        int r = HPADI_OK;
        if (hipMemcpyAsync(td, tau.data(), J * sizeof(double), hipMemcpyHostToDevice, P->stream) != hipSuccess ||
            hpadi::launch_pass_tables(D.dev, J, fac, fl.stride, fac + (size_t)J * fl.stride, fl, td, kappa, *out,
                                      P->stream) != hipSuccess ||
            hipStreamSynchronize(P->stream) != hipSuccess)
            r = HPADI_EHIP;
        hipFree(td);
        return r;
    };
    std::vector<double> tr(J), tc(J);
    for (int j = 0; j < J; ++j) {
        tr[j] = P->sy + F.Q[j];
        tc[j] = j + 1 < J ? P->sx - F.P[j + 1] : 0.0;
    }
    if ((rc = ptables(P->dy, F.facy64, P->fly, tr, P->ky, &F.ptaby)) != HPADI_OK) return rc;
    return ptables(P->dx, F.facx64, P->flx, tc, P->kx, &F.ptabx);
}

// The shift family for an FP64 refinement round that follows one whose error bound was
// `bound`: the round multiplies the error by at most eps / (1 - eps) (ADI lemma), so the
// loosest family of the ladder 0.1, 0.03, 0.01, ... with eps <= 0.8 tol / bound suffices,
// and costs fewer shifts than the first refinement family.  Ladder families are built
// (factorised on the plan's stream) on first use.  *out = the family to use.
int ladder_family(hpadi_plan_s* P, double bound, const ShiftFamily** out) {
    *out = &P->refine();
    const double want = 0.8 * P->tol / bound;
    if (!(bound > 0.0) || !(want > P->refine().eps)) return HPADI_OK;
    static const double rungs[] = {0.1, 0.03, 0.01, 3e-3, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5};
    double eps = 0.0;
    for (double r : rungs)
        if (r <= want) {
            eps = r;
            break;
        }
    if (!(eps > P->refine().eps)) return HPADI_OK;
    for (int i = 1; i < P->nfam; ++i)
        if (P->fam[i].eps == eps) {
            *out = &P->fam[i];
            return HPADI_OK;
        }
    if (P->nfam >= hpadi_plan_s::kMaxFam) return HPADI_OK;
    ShiftFamily& F = P->fam[P->nfam];
    const int rc = build_family(P, P->dx.op, P->dy.op, eps, F);
    if (rc != HPADI_OK) {
        family_free(F);
        return rc;
    }
    P->nfam++;
    *out = &F;
    return HPADI_OK;
}

int hpadi_plan_create_ex(hpadi_op1d x, hpadi_op1d y, double omega2, double tol, int precision,
                         const double* interval, void* hip_stream, const hpadi_options* opts, hpadi_plan* out) {
    if (!out) return HPADI_EINVAL;
    *out = nullptr;
    if (!std::isfinite(omega2)) return HPADI_EINVAL;
    if (omega2 < 0.0) return HPADI_ESINGULAR;
    const double coef[4] = {1.0, omega2 / 2.0, 1.0, omega2 / 2.0};
    const int rc = hpadi_plan_create_general(x, y, coef, tol, precision, interval, hip_stream, opts, out);
    if (rc == HPADI_OK) (*out)->omega2 = omega2;
    return rc;
}

int hpadi_plan_create_general(hpadi_op1d x, hpadi_op1d y, const double coef[4], double tol, int precision,
                              const double* interval, void* hip_stream, const hpadi_options* opts,
                              hpadi_plan* out) {
    if (!out) return HPADI_EINVAL;
    *out = nullptr;
    if (!x || !y || !coef || !(tol > 0.0 && tol < 1.0) || (precision != HPADI_FP64 && precision != HPADI_MIXED))
        return HPADI_EINVAL;
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(coef[i])) return HPADI_EINVAL;
    if (!(coef[0] > 0.0) || !(coef[2] > 0.0)) return HPADI_EINVAL;
    // both axis operators must be positive definite: K is singular only with Neumann at both ends
    if (coef[1] < 0.0 || coef[3] < 0.0 || (x->k_singular() && !(coef[1] > 0.0)) ||
        (y->k_singular() && !(coef[3] > 0.0)))
        return HPADI_ESINGULAR;
    if (x->p / 2 > 64 || y->p / 2 > 64 || x->nh > kMaxHats || y->nh > kMaxHats) return HPADI_EINVAL;
    hpadi_plan_s* P = new (std::nothrow) hpadi_plan_s;
    if (!P) return HPADI_ENOMEM;
    if (opts) P->opt = *opts;
    if (!(P->opt.inner_tol > 0.0)) P->opt.inner_tol = 3e-7;
    if (P->opt.fp32_rounds <= 0) P->opt.fp32_rounds = 1;
    if (P->opt.max_rounds <= 0) P->opt.max_rounds = 8;
    P->kx = coef[0];
    P->sx = coef[1];
    P->ky = coef[2];
    P->sy = coef[3];
    P->omega2 = 2.0 * coef[1];  // the screened problem's omega^2 when sx = sy (Burgers, batch keys)
    P->tol = tol;
    P->precision = precision;
    P->stream = (hipStream_t)hip_stream;
    int rc;
    // interval of Alg. 2: [a, b] for (A_Y^x, M^x), [c, d] = [-b_y, -a_y] for (-A_Y^y, M^y)
    if (interval) {
        for (int i = 0; i < 4; ++i) P->interval[i] = interval[i];
    } else {
        double ix[2], iy[2];
        if ((rc = interval_of(*x, P->kx, P->sx, ix)) != HPADI_OK) { plan_free(P); return rc; }
        if (same_op(*x, *y) && P->kx == P->ky && P->sx == P->sy) { iy[0] = ix[0]; iy[1] = ix[1]; }
        else if ((rc = interval_of(*y, P->ky, P->sy, iy)) != HPADI_OK) { plan_free(P); return rc; }
        P->interval[0] = ix[0];
        P->interval[1] = ix[1];
        P->interval[2] = -iy[1];
        P->interval[3] = -iy[0];
    }
    if ((rc = make_dim(P->dx, *x)) != HPADI_OK || (rc = make_dim(P->dy, *y)) != HPADI_OK) { plan_free(P); return rc; }
    // FP64 plans: one family for tol.  Mixed plans: the FP32 rounds use inner_tol; the
    // first FP64 refinement round needs eps <= tol / e (ADI lemma), e the error left by the
    // FP32 round, which follows inner_tol down to the FP32 rounding floor: a family for
    // tol / inner_tol meets tol after two rounds when e <= inner_tol (measured fastest at
    // n = p = 64 against 1e-4 and 1e-3), and a later round takes a looser ladder family.
    const double eps0 = precision == HPADI_FP64 ? tol : std::max(P->opt.inner_tol, tol);
    if ((rc = build_family(P, *x, *y, eps0, P->fam[0])) != HPADI_OK) { plan_free(P); return rc; }
    if (precision == HPADI_MIXED) {
        double eps1 = P->opt.refine_tol > 0.0 ? P->opt.refine_tol : tol / eps0;
        eps1 = std::min(0.1, std::max(eps1, tol));
        if (eps1 != eps0) {
            if ((rc = build_family(P, *x, *y, eps1, P->fam[1])) != HPADI_OK) { plan_free(P); return rc; }
            P->nfam = 2;
            P->iref = 1;
        }
    }
    // workspace: internal panel layout (8-column panels, hats padded to a multiple of 8)
    const int Nx = x->N, Ny = y->N;
    P->ldw = ((long)Ny + 63) / 64 * 64;
    hpadi::Layout& L = P->lint;
    // panel width of the internal layout: 8 when 8-line (or 1-line) workgroups are asked
    // for, else 4 (measured fastest for FP64 at n = p = 64, equal for FP32); lines per
    // workgroup of the ADI half-sweeps: 1, 4 or 8 per direction
    const int pw = (P->opt.lines_per_block == 8 || P->opt.lines_per_block == 1) ? 8 : 4;
    auto lines = [&](int req, int n_line_axis, int p_line_axis) {
        if (req == 1 && n_line_axis % 64 == 0) return 1;
        // 8 lines over 4-column panels: a wavefront reads 8 chains x 8 lines, whole 128-byte
        // lines of FP32 in both directions (2n / 8 wavefronts, within the kernel's limit)
        if (req == 8 && pw == 4 && n_line_axis % 8 == 0 &&
            64 * (2 * n_line_axis / 8) <= (p_line_axis / 2 <= 32 ? 1024 : 512))
            return 8;
        // a wavefront holds 64 / lines chains of one parity: small n needs more lines
        if (n_line_axis % (64 / pw) != 0 && n_line_axis % 4 == 0) return 16;
        return pw;
    };
    // a column pass runs along x (chains of the x basis), a row pass along y
    P->lpb_col = lines(P->opt.col_lines_per_block > 0 ? P->opt.col_lines_per_block : P->opt.lines_per_block, x->n,
                       x->p);
    P->lpb_row = lines(P->opt.row_lines_per_block > 0 ? P->opt.row_lines_per_block : P->opt.lines_per_block, y->n,
                       y->p);
    L.panel = pw;
    L.nhr = x->nh;
    L.nhc = y->nh;
    L.offr = P->dx.hpad - x->nh;
    L.offc = P->dy.hpad - y->nh;
    L.ld = (long)P->dx.Npad * pw;
    const long panels = (P->dy.Npad + pw - 1) / pw;
    P->nint = (size_t)panels * L.ld;
    // 8-byte elements in both modes: mixed plans run FP64 refinement rounds as well
    bool ok = hipMalloc(&P->Wk, P->nint * 8) == hipSuccess && hipMalloc(&P->Gt, P->nint * 8) == hipSuccess &&
              dmalloc(&P->T64, P->nint) == hipSuccess;
    ok = ok && dmalloc(&P->acc, 8) == hipSuccess && hipHostMalloc((void**)&P->acc_host, 8 * sizeof(double)) == hipSuccess;
    ok = ok && dmalloc(&P->part, (size_t)hpadi::residual_partials(P->dx.dev, P->dy.op.N)) == hipSuccess;
    if (!ok) { plan_free(P); return HPADI_ENOMEM; }
    (void)Nx;
    (void)Ny;
    *out = P;
    return HPADI_OK;
}

int hpadi_plan_create(hpadi_op1d x, hpadi_op1d y, double omega2, double tol, int precision, const double* interval,
                      void* hip_stream, hpadi_plan* out) {
    return hpadi_plan_create_ex(x, y, omega2, tol, precision, interval, hip_stream, nullptr, out);
}

int hpadi_plan_info(hpadi_plan P, int* J, double* p, double* q, double interval[4]) {
    if (!P) return HPADI_EINVAL;
    const ShiftFamily& F = P->first();
    if (J) *J = F.J;
    for (int j = 0; j < F.J; ++j) {
        if (p) p[j] = F.P[j];
        if (q) q[j] = F.Q[j];
    }
    if (interval)
        for (int i = 0; i < 4; ++i) interval[i] = P->interval[i];
    return HPADI_OK;
}

int hpadi_plan_export_factor(hpadi_plan P, int j, int axis, double* buf, size_t len) {
    if (!P || !buf || (axis != 0 && axis != 1)) return HPADI_EINVAL;
    const FactorLayout& fl = axis == 0 ? P->flx : P->fly;
    const ShiftFamily& F = P->first();
    const double* base = axis == 0 ? F.facx64 : F.facy64;
    const int idx = j == -1 ? F.J : j;
    const size_t doc = (size_t)fl.off_link0 + (fl.off_link0 - fl.off_invd0);  // documented prefix
    if (idx < 0 || idx > F.J || len < doc) return HPADI_EINVAL;
    if (hipMemcpyAsync(buf, base + (size_t)idx * fl.stride, doc * sizeof(double), hipMemcpyDeviceToHost,
                       P->stream) != hipSuccess ||
        hipStreamSynchronize(P->stream) != hipSuccess)
        return HPADI_EHIP;
    return HPADI_OK;
}

int hpadi_load(hpadi_plan P, const double* F, int ldf, double* G, int ldg) {
    if (!P || !F || !G || ldf < P->dy.op.Nleg || ldg < P->dy.op.N) return HPADI_EINVAL;
    if (!P->H) {
        P->ldh = ((long)P->dy.op.N + 63) / 64 * 64;
        if (dmalloc(&P->H, (size_t)P->dx.op.Nleg * P->ldh) != hipSuccess) return HPADI_ENOMEM;
    }
    return hpadi::launch_load(P->dx.dev, P->dy.dev, F, ldf, P->H, P->ldh, G, ldg, P->stream) == hipSuccess
               ? HPADI_OK
               : HPADI_EHIP;
}

int hpadi_load_noalloc(hpadi_plan P, const double* F, int ldf, double* G, int ldg) {
    if (!P || !F || !G || ldf < P->dy.op.Nleg || ldg < P->dy.op.N) return HPADI_EINVAL;
    // column blocks of w columns: the intermediate of one block, Nleg_x x w doubles, fills
    // at most the fixed scratch
    const long nleg = P->dx.op.Nleg;
    long w = hpadi::kLoadScratchWords / nleg / 64 * 64;
    if (w < 64) return HPADI_EINVAL;
    if (w > P->dy.op.N) w = P->dy.op.N;
    double* H = nullptr;
    if (hpadi::load_scratch(&H) != hipSuccess) return HPADI_EHIP;
    for (long j0 = 0; j0 < P->dy.op.N; j0 += w) {
        const int nc = (int)std::min<long>(w, P->dy.op.N - j0);
        if (hpadi::launch_load_cols(P->dx.dev, P->dy.dev, F, ldf, H, w, G, ldg, (int)j0, nc, P->stream) !=
            hipSuccess)
            return HPADI_EHIP;
    }
    return HPADI_OK;
}

int hpadi_apply(hpadi_plan P, const double* U, int ldu, double* Y, int ldy) {
    if (!P || !U || !Y || ldu < P->dy.op.N || ldy < P->dy.op.N) return HPADI_EINVAL;
    int rc = ensure_fp64_work(P);
    if (rc != HPADI_OK) return rc;
    if ((rc = row_products(P, U, ldu)) != HPADI_OK) return rc;
    hpadi::Residual r{};
    r.G = nullptr;
    r.T1 = P->T12;
    r.T2 = nullptr;
    r.t_ld = P->ldw;
    r.r64 = Y;
    r.r64_ld = ldy;
    r.ax_k = P->kx;
    r.ax_t = P->sx;
    r.alpha = 0.0;
    r.beta = 1.0;
    r.ncols = P->dy.op.N;
    return hpadi::launch_residual(P->dx.dev, r, P->stream) == hipSuccess ? HPADI_OK : HPADI_EHIP;
}

int hpadi_solve(hpadi_plan P, const double* G, int ldg, double* U, int ldu, hpadi_stats* stats) {
    if (!P || !G || !U || ldg < P->dy.op.N || ldu < P->dy.op.N) return HPADI_EINVAL;
    hpadi_stats st{};
    st.J = P->first().J;
    st.J_refine = P->refine().J;
    for (int i = 0; i < 4; ++i) st.interval[i] = P->interval[i];
    hipStream_t s = P->stream;
    const int Nx = P->dx.op.N, Ny = P->dy.op.N;
    int rc = HPADI_OK;
    if (P->precision == HPADI_FP64) {
        if ((rc = transform_rhs(P, G, ldg, 8)) != HPADI_OK) return rc;
        if ((rc = run_adi(P, P->first(), 8, U, ldu, false, false)) != HPADI_OK) return rc;
        st.rounds = 1;
        st.iters = P->first().J;
        st.est_rel_err = P->tol;
    } else {
        // Iterative refinement: U = 0; repeat { delta = ADI(r); U += delta; r = G - A U (FP64) }.
        // The first fp32_rounds rounds run the ADI sweeps in FP32 storage; the later ones in
        // FP64, where the ADI lemma bounds the error of the round: with e the error before
        // the round and delta its correction, ||e - delta|| <= eps ||e|| and ||e|| <= ||delta||
        // / (1 - eps), so ||U* - U|| <= eps / (1 - eps) ||delta|| (eps: tolerance of the
        // shift family of the round), all in the lemma's norm (lemma_bound).  FP32 rounds
        // have no such bound (their rounding floor depends on the spectrum of the residual)
        // and never end the solve.  FP32 rounds take the first shift family, the first FP64
        // round the refinement family, later FP64 rounds the loosest family that the bound
        // of the round before allows (ladder_family).
        if ((rc = ensure_fp64_work(P)) != HPADI_OK) return rc;
        if (!P->R64 && dmalloc(&P->R64, (size_t)Nx * P->ldw) != hipSuccess) return HPADI_ENOMEM;
        double est = 1.0, last_bound = 0.0;
        const int maxr = P->opt.fixed_rounds > 0 ? P->opt.fixed_rounds : P->opt.max_rounds;
        int k = 0, nfp32 = P->opt.fp32_rounds, k0 = 0;
        bool done = false;
        // phase times (stats t_ms): three events per round, before it, after its ADI sweeps
        // and after the residual that follows; read once the last round has been synchronised
        while ((int)P->phase_ev.size() < 3 * maxr) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return HPADI_EHIP;
            P->phase_ev.push_back(e);
        }
        std::vector<int> round_fp32, round_res;
        for (k = 1; k <= maxr; ++k) {
            // k0: rounds discarded by a restart in FP64 (an FP32 round that overflowed)
            const bool fp32 = k - k0 <= nfp32;
            const int ts = fp32 ? 4 : 8;
            const ShiftFamily* Fp = fp32 ? &P->first() : &P->refine();
            if (!fp32 && P->opt.fixed_rounds <= 0 && std::isfinite(last_bound) && last_bound > 0.0 &&
                (rc = ladder_family(P, last_bound, &Fp)) != HPADI_OK)
                return rc;
            const ShiftFamily& F = *Fp;
            const double eps = F.eps;
            // round 1 starts from U = 0 (acc[4], the norm of U before the round, stays 0)
            const bool first = k == k0 + 1;
            hipEvent_t* ev = P->phase_ev.data() + 3 * (k - 1);
            if (hipEventRecord(ev[0], s) != hipSuccess) return HPADI_EHIP;
            round_fp32.push_back(fp32 ? 1 : 0);
            round_res.push_back(0);
            if (hpadi::launch_zero_f64(P->acc, first ? 5 : 1, 1, first ? 5 : 1, s) != hipSuccess) return HPADI_EHIP;
            if ((rc = transform_rhs(P, first ? G : P->R64, first ? ldg : P->ldw, ts)) != HPADI_OK) return rc;
            // the first round writes U, later rounds add their correction to it
            if ((rc = run_adi(P, F, ts, U, ldu, !first, true)) != HPADI_OK) return rc;
            if (hipEventRecord(ev[1], s) != hipSuccess) return HPADI_EHIP;
            st.iters += F.J;
            if (fp32) st.fp32_rounds++;
            const bool decide = P->opt.fixed_rounds <= 0 && !fp32;
            if (decide || k == maxr) {
                if (hipMemcpyAsync(P->acc_host, P->acc, 5 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess)
                    return HPADI_EHIP;
                if (k > 1) {
                    const double gnorm = std::sqrt(std::max(P->acc_host[3], 0.0));
                    st.res_rel = gnorm > 0 ? std::sqrt(std::max(P->acc_host[2], 0.0)) / gnorm : 0.0;
                }
                est = fp32 ? 1.0 : lemma_bound(eps, P->acc_host[0], P->acc_host[4]);
                if (!fp32) last_bound = est;
                const bool finite = std::isfinite(P->acc_host[0]) && std::isfinite(P->acc_host[4]);
                if (!finite && nfp32 > 0 && k < maxr) {
                    // data beyond the FP32 range (or a non-finite FP32 round): start again
                    // with FP64 rounds only; a non-finite input fails again and ends ENOCONV
                    nfp32 = 0;
                    k0 = k;
                    last_bound = 0.0;
                    st.fp32_rounds = 0;
                    continue;
                }
                if (!finite) break;
                if (decide && est <= P->tol) {
                    done = true;
                    break;
                }
                if (k == maxr) break;
            }
            // r = G - A U in FP64
            if ((rc = residual_into_r64(P, G, ldg, U, ldu)) != HPADI_OK) return rc;
            if (hipEventRecord(ev[2], s) != hipSuccess) return HPADI_EHIP;
            round_res.back() = 1;
        }
        if (k > maxr) k = maxr;
        // every recorded event precedes the last synchronisation
        for (size_t r = 0; r < round_fp32.size(); ++r) {
            const hipEvent_t* ev = P->phase_ev.data() + 3 * r;
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) st.t_ms[round_fp32[r] ? 0 : 1] += ms;
            if (round_res[r] && hipEventElapsedTime(&ms, ev[1], ev[2]) == hipSuccess) st.t_ms[2] += ms;
        }
        st.rounds = k;
        st.est_rel_err = est;
        if (P->opt.fixed_rounds <= 0 && !done) rc = HPADI_ENOCONV;
    }
    st.status = rc;
    if (stats) *stats = st;
    return rc;
}

namespace {
// On-disk autotune results: one line per key, "arch n_x p_x n_y p_y mask_x mask_y lines".
void load_tune_cache(const char* path, const std::string& arch, std::vector<std::pair<std::vector<int>, int>>& out) {
    std::FILE* f = std::fopen(path, "r");
    if (!f) return;
    char a[64];
    int v[7];
    while (std::fscanf(f, "%63s %d %d %d %d %d %d %d", a, &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6]) == 8)
        if (arch == a && (v[6] == 4 || v[6] == 8)) out.push_back({{v[0], v[1], v[2], v[3], v[4], v[5]}, v[6]});
    std::fclose(f);
}
void save_tune_cache(const char* path, const std::string& arch, const std::vector<std::pair<std::vector<int>, int>>& t,
                     size_t from) {
    std::FILE* f = std::fopen(path, "a");
    if (!f) return;  // the cache is an optimisation: a read-only location is not an error
    for (size_t i = from; i < t.size(); ++i) {
        const std::vector<int>& k = t[i].first;
        std::fprintf(f, "%s %d %d %d %d %d %d %d\n", arch.c_str(), k[0], k[1], k[2], k[3], k[4], k[5], t[i].second);
    }
    std::fclose(f);
}
}  // namespace

int hpadi_batch_create(int count, const hpadi_op1d* xs, const hpadi_op1d* ys, const double* omega2, double tol,
                       const double* const* G, const int* ldg, double* const* U, const int* ldu, int autotune,
                       int nstreams, void* hip_stream, hpadi_batch* out) {
    if (count < 1 || !xs || !ys || !omega2 || !G || !ldg || !U || !ldu || !out || !(tol > 0.0 && tol < 1.0))
        return HPADI_EINVAL;
    *out = nullptr;
    // every instance is checked before the first HIP call
    for (int i = 0; i < count; ++i)
        if (!xs[i] || !ys[i] || !G[i] || !U[i] || ldg[i] < ys[i]->N || ldu[i] < ys[i]->N ||
            xs[i]->nh > kMaxHats || ys[i]->nh > kMaxHats)
            return HPADI_EINVAL;
    hpadi_batch_s* B = new (std::nothrow) hpadi_batch_s();
    if (!B) return HPADI_ENOMEM;
    B->count = count;
    B->tol = tol;
    B->origin = (hipStream_t)hip_stream;
    if (!B->origin) {
        // the legacy default stream cannot be captured: launch the graph on a stream of our own
        if (hipStreamCreateWithFlags(&B->origin, hipStreamNonBlocking) != hipSuccess) {
            delete B;
            return HPADI_EHIP;
        }
        B->own_origin = true;
    }
    (void)nstreams;
    // autotuner: lines per workgroup (4 or 8) per distinct (n_x, p_x, n_y, p_y, hat masks), by
    // timing one fixed-schedule solve of each candidate on the instance's own data; results
    // persist in the file named by HPADI_TUNE_CACHE (if set), keyed by the GPU architecture
    std::vector<std::pair<std::vector<int>, int>> tuned;
    const char* cache_path = std::getenv("HPADI_TUNE_CACHE");
    std::string arch = "gpu";
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            arch = prop.gcnArchName;
            arch = arch.substr(0, arch.find(':'));
        }
    }
    if (autotune && cache_path) load_tune_cache(cache_path, arch, tuned);
    const size_t ncached = tuned.size();
    B->plans.assign(count, nullptr);
    B->lw.assign(count, 4);
    B->G.assign(G, G + count);
    B->U.assign(U, U + count);
    B->ldg.assign(ldg, ldg + count);
    B->ldu.assign(ldu, ldu + count);
    auto make_plan = [&](int i, int lw, hpadi_plan* pl) -> int {
        hpadi_options o{};
        o.lines_per_block = lw;
        // FP32 round at 3e-6, FP64 round at 1e-6: the batch's small, rough instances leave
        // FP32 errors well above 3e-7, and the FP64 family must take them to tol in one
        // round, or they need a further round outside the graph
        o.inner_tol = 3e-6;
        o.refine_tol = 1e-6;
        int rc = hpadi_plan_create_ex(xs[i], ys[i], omega2[i], tol, HPADI_MIXED, nullptr, B->origin, &o, pl);
        if (rc != HPADI_OK) return rc;
        hpadi_plan_s* P = *pl;
        if ((rc = ensure_fp64_work(P)) != HPADI_OK) return rc;
        if (!P->R64 && dmalloc(&P->R64, (size_t)P->dx.op.N * P->ldw) != hipSuccess) return HPADI_ENOMEM;
        return HPADI_OK;
    };
    for (int i = 0; i < count; ++i) {
        const std::vector<int> key = {xs[i]->n, xs[i]->p, ys[i]->n, ys[i]->p, xs[i]->bc, ys[i]->bc};
        int lw = 4;
        bool found = false;
        for (auto& kv : tuned)
            if (kv.first == key) {
                lw = kv.second;
                found = true;
            }
        int rc = HPADI_OK;
        if (!found && autotune) {
            double best = 1e300;
            for (int cand : {4, 8}) {
                hpadi_plan pl = nullptr;
                if ((rc = make_plan(i, cand, &pl)) != HPADI_OK) {
                    hpadi_plan_destroy(pl);
                    delete B;
                    return rc;
                }
                hipStream_t st = pl->stream;
                hipEvent_t e0 = nullptr, e1 = nullptr;
                float ms = 0.0f;
                bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
                ok = ok && enqueue_fixed_solve(pl, G[i], ldg[i], U[i], ldu[i], 1, 1) == HPADI_OK;  // warm-up
                ok = ok && hipEventRecord(e0, st) == hipSuccess &&
                     enqueue_fixed_solve(pl, G[i], ldg[i], U[i], ldu[i], 1, 1) == HPADI_OK &&
                     hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                if (e0) (void)hipEventDestroy(e0);
                if (e1) (void)hipEventDestroy(e1);
                if (!ok) {
                    hpadi_plan_destroy(pl);
                    delete B;
                    return HPADI_EHIP;
                }
                if (ms < best) {
                    best = ms;
                    lw = cand;
                    if (B->plans[i]) hpadi_plan_destroy(B->plans[i]);
                    B->plans[i] = pl;
                } else {
                    hpadi_plan_destroy(pl);
                }
            }
            tuned.push_back({key, lw});
        }
        B->lw[i] = lw;
        if (!B->plans[i] && (rc = make_plan(i, lw, &B->plans[i])) != HPADI_OK) {
            delete B;
            return rc;
        }
    }
    if (autotune && cache_path && tuned.size() > ncached) save_tune_cache(cache_path, arch, tuned, ncached);
    // device table of accumulator pointers and their gathered copy
    std::vector<double*> accs(count);
    for (int i = 0; i < count; ++i) accs[i] = B->plans[i]->acc;
    if (dmalloc(&B->acc_ptrs, (size_t)count) != hipSuccess || dmalloc(&B->acc_all, 2 * (size_t)count) != hipSuccess ||
        hipHostMalloc((void**)&B->acc_host, 2 * (size_t)count * sizeof(double)) != hipSuccess ||
        hipMemcpy(B->acc_ptrs, accs.data(), count * sizeof(double*), hipMemcpyHostToDevice) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        delete B;
        return HPADI_ENOMEM;
    }
    // the schedule: both rounds of every instance in lock step, every kind of half-sweep
    // of one iteration as few grouped launches as there are (chain length, width) pairs
    std::vector<BatchStep> steps;
    std::vector<hpadi::GroupTask> table;
    // phases: the steps appended since the last seal touch disjoint instances
    int nphase = 0;
    size_t mark = 0;
    auto seal = [&]() {
        for (size_t k = mark; k < steps.size(); ++k) steps[k].phase = nphase;
        ++nphase;
        mark = steps.size();
    };
    for (int round = 1; round <= 2; ++round) {
        const int ts = round == 1 ? 4 : 8;
        // round 1: FP32 sweeps with the first shift family; round 2: FP64 sweeps with the
        // refinement family
        auto fam = [&](const hpadi_plan_s* P) -> const ShiftFamily& { return round == 1 ? P->first() : P->refine(); };
        int jmax = 0;
        for (int i = 0; i < count; ++i) jmax = std::max(jmax, fam(B->plans[i]).J);
        // round 1 writes U (no zeroing pass); round 2 starts from the FP64 residual of every
        // instance; one launch clears the correction norms of all instances
        if (round == 2)
            for (int i = 0; i < count; ++i) {
                BatchStep st;
                st.kind = 2;
                st.inst = i;
                steps.push_back(st);
            }
        {
            BatchStep st;
            st.kind = 4;
            steps.push_back(st);
        }
        seal();
        std::vector<std::pair<int, hpadi::SweepArgs>> items;
        for (int i = 0; i < count; ++i) {
            hpadi_plan_s* P = B->plans[i];
            items.push_back({i, transform_row_args(P, round == 1 ? G[i] : P->R64, round == 1 ? ldg[i] : P->ldw)});
        }
        add_sweeps(steps, table, B->plans, items, hpadi::SWEEP_TRANSFORM, 8, 8, false);
        seal();
        items.clear();
        for (int i = 0; i < count; ++i) items.push_back({i, transform_col_args(B->plans[i])});
        add_sweeps(steps, table, B->plans, items, hpadi::SWEEP_TRANSFORM, 8, ts, true);
        seal();
        for (int jj = 0; jj < jmax; ++jj) {
            std::vector<std::pair<int, hpadi::SweepArgs>> rows, cols, last;
            for (int i = 0; i < count; ++i) {
                hpadi_plan_s* P = B->plans[i];
                const ShiftFamily& F = fam(P);
                if (jj >= F.J) continue;
                rows.push_back({i, adi_row_args(P, F, jj)});
                if (jj + 1 == F.J) last.push_back({i, last_col_args(P, F, true)});
                else cols.push_back({i, adi_col_args(P, F, jj)});
            }
            add_sweeps(steps, table, B->plans, rows, hpadi::SWEEP_FULL, ts, ts, false);
            seal();
            add_sweeps(steps, table, B->plans, cols, hpadi::SWEEP_FULL, ts, ts, true);
            add_sweeps(steps, table, B->plans, last, hpadi::SWEEP_SOLVE, ts, ts, true);
            seal();
        }
        items.clear();
        for (int i = 0; i < count; ++i) items.push_back({i, final_args(B->plans[i], U[i], ldu[i], round > 1)});
        add_sweeps(steps, table, B->plans, items, hpadi::SWEEP_FINAL, ts, 8, false);
        seal();
    }
    if (!table.empty() &&
        (dmalloc(&B->table, table.size()) != hipSuccess ||
         hipMemcpy(B->table, table.data(), table.size() * sizeof(hpadi::GroupTask), hipMemcpyHostToDevice) != hipSuccess)) {
        delete B;
        return HPADI_ENOMEM;
    }
    // capture the schedule on the origin stream (every plan works on that stream)
    for (hpadi_plan p : B->plans) p->stream = B->origin;
    // capture lanes: the origin stream plus kLanes - 1 side streams that join the capture
    // through the fork event of each phase
    bool ok = hipEventCreateWithFlags(&B->fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k + 1 < hpadi_batch_s::kLanes && ok; ++k)
        ok = hipStreamCreateWithFlags(&B->side[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&B->join[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        delete B;
        return HPADI_EHIP;
    }
    auto lane = [&](int k) -> hipStream_t { return k == 0 ? B->origin : B->side[k - 1]; };
    auto launch_step = [&](const BatchStep& st, hipStream_t q) -> bool {
        hpadi_plan_s* P = st.inst >= 0 ? B->plans[st.inst] : nullptr;
        switch (st.kind) {
            case 0: {
                hpadi::GroupLaunch g = st.g;
                g.tasks = B->table + st.task_off;
                return hpadi::launch_sweep_uni_grouped(g, q) == hipSuccess;
            }
            case 1:
                return hpadi::launch_sweep(st.column ? P->dx.dev : P->dy.dev, st.a, st.mode, st.tin, st.tout,
                                           st.column, q) == hipSuccess;
            case 2: {
                P->stream = q;
                const bool r = residual_into_r64(P, G[st.inst], ldg[st.inst], U[st.inst], ldu[st.inst]) == HPADI_OK;
                P->stream = B->origin;
                return r;
            }
            case 4:
                return hpadi::launch_zero_accs(B->acc_ptrs, count, q) == hipSuccess;
            default:
                return false;
        }
    };
    ok = hipStreamBeginCapture(B->origin, hipStreamCaptureModeRelaxed) == hipSuccess;
    for (size_t a = 0; a < steps.size() && ok;) {
        size_t b = a;
        while (b < steps.size() && steps[b].phase == steps[a].phase) ++b;
        const int nl = (int)std::min<size_t>(b - a, hpadi_batch_s::kLanes);
        // fork: the side lanes of this phase wait for everything before it on the origin
        if (nl > 1) {
            ok = hipEventRecord(B->fork, B->origin) == hipSuccess;
            for (int k = 1; k < nl && ok; ++k) ok = hipStreamWaitEvent(lane(k), B->fork, 0) == hipSuccess;
        }
        for (size_t t = a; t < b && ok; ++t) {
            ok = launch_step(steps[t], lane((int)((t - a) % nl)));
            ++B->nlaunch;
        }
        // join: the origin waits for every side lane before the next phase
        for (int k = 1; k < nl && ok; ++k)
            ok = hipEventRecord(B->join[k - 1], lane(k)) == hipSuccess &&
                 hipStreamWaitEvent(B->origin, B->join[k - 1], 0) == hipSuccess;
        a = b;
    }
    ok = ok && hpadi::launch_gather_acc(B->acc_ptrs, count, B->acc_all, B->origin) == hipSuccess;
    const bool ended = hipStreamEndCapture(B->origin, &B->graph) == hipSuccess;
    ok = ok && ended && hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {
        delete B;
        return HPADI_EHIP;
    }
    *out = B;
    return HPADI_OK;
}

int hpadi_batch_solve(hpadi_batch B, hpadi_stats* stats, int* n_extra) {
    if (!B) return HPADI_EINVAL;
    if (hipGraphLaunch(B->exec, B->origin) != hipSuccess ||
        hipMemcpyAsync(B->acc_host, B->acc_all, 2 * (size_t)B->count * sizeof(double), hipMemcpyDeviceToHost,
                       B->origin) != hipSuccess ||
        hipStreamSynchronize(B->origin) != hipSuccess)
        return HPADI_EHIP;
    // lemma bound of the FP64 round; instances above the tolerance get further FP64 rounds
    int extra = 0, status = HPADI_OK;
    for (int i = 0; i < B->count; ++i) {
        hpadi_plan_s* P = B->plans[i];
        const double eps = P->refine().eps;
        double est = lemma_bound(eps, B->acc_host[2 * i], B->acc_host[2 * i + 1]);
        int rounds = 2, iters = P->first().J + P->refine().J;
        while (est > B->tol && rounds < P->opt.max_rounds) {
            const ShiftFamily* F = &P->refine();
            int rc = std::isfinite(est) ? ladder_family(P, est, &F) : HPADI_OK;
            if (rc == HPADI_OK) rc = residual_into_r64(P, B->G[i], B->ldg[i], B->U[i], B->ldu[i]);
            if (rc == HPADI_OK && hpadi::launch_zero_f64(P->acc, 1, 1, 1, P->stream) != hipSuccess) rc = HPADI_EHIP;
            if (rc == HPADI_OK) rc = transform_rhs(P, P->R64, P->ldw, 8);
            if (rc == HPADI_OK) rc = run_adi(P, *F, 8, B->U[i], B->ldu[i], true, true);
            if (rc == HPADI_OK &&
                (hipMemcpyAsync(P->acc_host, P->acc, 5 * sizeof(double), hipMemcpyDeviceToHost, P->stream) != hipSuccess ||
                 hipStreamSynchronize(P->stream) != hipSuccess))
                rc = HPADI_EHIP;
            if (rc != HPADI_OK) return rc;
            est = lemma_bound(F->eps, P->acc_host[0], P->acc_host[4]);
            iters += F->J;
            ++rounds;
            ++extra;
        }
        if (!(est <= B->tol)) status = HPADI_ENOCONV;
        if (stats) {
            hpadi_stats st{};
            st.J = P->first().J;
            st.J_refine = P->refine().J;
            st.rounds = rounds;
            st.fp32_rounds = 1;
            st.iters = iters;
            st.status = est <= B->tol ? HPADI_OK : HPADI_ENOCONV;
            st.est_rel_err = est;
            for (int k = 0; k < 4; ++k) st.interval[k] = P->interval[k];
            stats[i] = st;
        }
    }
    if (n_extra) *n_extra = extra;
    return status;
}

int hpadi_batch_info(hpadi_batch B, int i, int* lines_per_block, int* J, int* stream_index) {
    if (!B || i < 0 || i >= B->count) return HPADI_EINVAL;
    if (lines_per_block) *lines_per_block = B->lw[i];
    if (J) *J = B->plans[i]->first().J;
    if (stream_index) *stream_index = 0;
    return HPADI_OK;
}

void hpadi_batch_destroy(hpadi_batch B) { delete B; }

int hpadi_plan_timing(hpadi_plan P, int enable) {
    if (!P) return HPADI_EINVAL;
    if (enable) P->nrec = 0;
    P->timing = enable != 0;
    return HPADI_OK;
}

int hpadi_plan_timing_read(hpadi_plan P, double ms[6], double bytes[6], int count[6]) {
    if (!P) return HPADI_EINVAL;
    if (hipStreamSynchronize(P->stream) != hipSuccess) return HPADI_EHIP;
    double t[6] = {0, 0, 0, 0, 0, 0}, b[6] = {0, 0, 0, 0, 0, 0};
    int c[6] = {0, 0, 0, 0, 0, 0};
    for (size_t i = 0; i < P->nrec; ++i) {
        float e = 0.0f;
        if (hipEventElapsedTime(&e, P->recs[i].a, P->recs[i].b) != hipSuccess) return HPADI_EHIP;
        const int k = P->recs[i].kind;
        t[k] += e;
        b[k] += P->recs[i].bytes;
        c[k] += 1;
    }
    for (int k = 0; k < 6; ++k) {
        if (ms) ms[k] = t[k];
        if (bytes) bytes[k] = b[k];
        if (count) count[k] = c[k];
    }
    return HPADI_OK;
}

void hpadi_plan_destroy(hpadi_plan P) {
    if (P && P->stream) hipStreamSynchronize(P->stream);
    else if (P) hipDeviceSynchronize();
    plan_free(P);
}

}  // extern "C"
