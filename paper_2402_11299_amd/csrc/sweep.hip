// ADI half-sweeps in mass-balanced coordinates (gfx950).
//
// The generalised ADI of Sec. 5 (Alg. 2) is, by the lemma that proves its error
// bound, the standard ADI for X = V U L^T, where M^x = V^T V and M^y = L^T L are
// the reverse Cholesky factors of the two mass matrices (Sec. 4).  In these
// coordinates a half-sweep along one direction, with S = K + sigma M and mass
// factor Lm of that direction, is
//
//   z = Lm^T y,   w = S^{-1} z,   out = g - Lm^{-T} (kappa K + tau M) w,
//
// (kappa K + tau M) being the product of the next half-step.  Every stored array
// (y, g, out) is then balanced: a relative rounding of its entries is a relative
// error in the norm of the ADI lemma, which is what lets the bulk of the data
// live in FP32 without the mass matrix amplifying the rounding.  All arithmetic
// here is FP64 (registers are not the bottleneck of a bandwidth-bound sweep).
//
// Work decomposition: a workgroup owns LW = 4 or 8 lines (one panel of the
// internal layout) and one thread owns one bubble chain (element e, parity pi)
// of one line, kept in registers.  Chain c = pi n + e of a line holds positions
// nh + 2 s n + c, s = 0, 1, ..., so the 2n chains of a step are consecutive and
// each wavefront reads LW lines x 64/LW consecutive positions: 256 bytes (FP32)
// in contiguous runs of at least 64 bytes, in both sweep directions.  The hat block of each line (the Schur
// complement of Alg. 1, n_h <= 65 unknowns) is solved by one wavefront per line
// as one 64-lane prefix composition of affine maps built from DPP row shifts and
// row broadcasts (the backward solve with its hats in reverse lane order), with the
// hat factors staged in LDS.

#include <hip/hip_runtime.h>

#include "internal.h"
#include "sweep_common.h"

namespace hpadi {

using namespace sweep_detail;

namespace {

template <typename TIN, typename TOUT, int CL, int MODE, bool COL, bool UNI, int LW>
__global__ void __launch_bounds__(sweep_max_threads(CL)) sweep_kernel(DimDev d, SweepArgs a) {
    // LW lines per workgroup (the panel width of the internal layout); CW chains per
    // wavefront, so that a wavefront touches LW lines x CW consecutive positions.
    constexpr int CW = 64 / LW;
    extern __shared__ double sm[];
    const int n = d.n, p = d.p, nh = d.nh;
    const int hs = nh + 1;
    // LDS: per line A, B (hats), H1, H2 (chain heads); then staged hat factors
    double* sA = sm;
    double* sB = sA + LW * hs;
    double* sH1 = sB + LW * hs;
    double* sH2 = sH1 + LW * 2 * n;
    double* fbase = sH2 + LW * 2 * n;
    HatF FS, FM;
    FS.invd0 = fbase;
    FS.d0 = FS.invd0 + hs;
    FS.link0 = FS.d0 + hs;
    FS.cpl = FS.link0 + hs;
    FM.invd0 = FS.cpl + 4 * n;
    FM.d0 = FM.invd0 + hs;
    FM.link0 = FM.d0 + hs;
    FM.cpl = FM.link0 + hs;
    double* scf = FM.cpl + 4 * n;  // uniform meshes: per-degree records, 8 (p-1) doubles

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wavefront-uniform: scalar registers
    const int nwaves = blockDim.x >> 6;
    int c, l;
    if (COL) {
        c = wave * CW + lane / LW;
        l = lane % LW;
    } else {
        c = wave * CW + lane % CW;
        l = lane / CW;
    }
    const FactorLayout& fl = a.fl;
    const double* S = a.facS;
    const double* Mf = a.facM;
    const bool useS = (MODE == SWEEP_FULL || MODE == SWEEP_SOLVE);

    // ---- stage the hat factors
    for (int i = tid; i < hs; i += blockDim.x) {
        const bool inr = i < nh;
        if (useS) {
            FS.invd0[i] = inr ? S[fl.off_invd0 + i] : 0.0;
            FS.d0[i] = inr ? S[fl.off_d0 + i] : 0.0;
            FS.link0[i] = inr ? S[fl.off_link0 + i] : 0.0;
        }
        FM.invd0[i] = inr ? Mf[fl.off_invd0 + i] : 0.0;
        FM.d0[i] = inr ? Mf[fl.off_d0 + i] : 0.0;
        FM.link0[i] = inr ? Mf[fl.off_link0 + i] : 0.0;
    }
    for (int i = tid; i < 4 * n; i += blockDim.x) {
        if (useS) FS.cpl[i] = S[fl.off_cpl + i];
        FM.cpl[i] = Mf[fl.off_cpl + i];
    }
    if (UNI)
        for (int i = tid; i < 8 * p; i += blockDim.x) scf[i] = a.coef[i];

    auto line_of = [&](int ll) -> int {
        const int lint = blockIdx.x * LW + ll;
        if (lint < a.nh_lines) return lint;
        if (lint < a.hpad_lines) return -1;
        return lint - (a.hpad_lines - a.nh_lines);
    };
    const int line = line_of(l);
    const bool lact = line >= 0 && line < a.nlines;
    const bool act = lact && c < 2 * n;
    // On a uniform mesh with n % CW == 0 the CW chains of a wavefront share their parity,
    // so degree-dependent coefficients are wavefront-uniform (scalar loads).
    const int pi = UNI ? __builtin_amdgcn_readfirstlane(c >= n ? 1 : 0) : (c >= n ? 1 : 0);
    const int e = c - pi * n;
    const int len = pi ? (p - 1) / 2 : p / 2;

    double* A = sA + l * hs;
    double* B = sB + l * hs;
    double* H1 = sH1 + l * 2 * n;
    double* H2 = sH2 + l * 2 * n;

    // per-degree coefficients (App. A entries and factor entries at degree m)
    const double* kd = d.tab64;
    const double* md = d.tab64 + d.tabstride;
    const double* mo = d.tab64 + 2 * d.tabstride;
    const double de = d.delta[e < n ? e : 0], ide = d.invdelta[e < n ? e : 0];
    const double* cf = scf;
    auto S_inv = [&](int m) { return UNI ? cf[m * 8 + 0] : S[fl.off_invd + m * n + e]; };
    auto S_lnk = [&](int m) { return UNI ? cf[m * 8 + 1] : S[fl.off_link + m * n + e]; };
    auto M_d = [&](int m) { return UNI ? cf[m * 8 + 2] : Mf[fl.off_d + m * n + e]; };
    auto M_lnk = [&](int m) { return UNI ? cf[m * 8 + 3] : Mf[fl.off_link + m * n + e]; };
    auto M_inv = [&](int m) { return UNI ? cf[m * 8 + 4] : Mf[fl.off_invd + m * n + e]; };
    auto K_dg = [&](int m) { return UNI ? cf[m * 8 + 5] : kd[m] * ide; };
    auto M_dg = [&](int m) { return UNI ? cf[m * 8 + 6] : md[m] * de; };
    auto M_of = [&](int m) { return UNI ? cf[m * 8 + 7] : mo[m] * de; };

    // addresses: chain step s of this thread sits at offset o + s * st (uniform meshes,
    // n % 8 == 0: the layouts map a chain step to a constant stride); general case per step
    auto IDX = [&](const Layout& L, int ln, int pos) -> long { return COL ? addr(L, pos, ln) : addr(L, ln, pos); };
    auto chain_off = [&](const Layout& L, int s) -> long {
        return IDX(L, line, nh + 2 * s * n + c);
    };
    const TIN* in = reinterpret_cast<const TIN*>(a.in);
    long oi = 0, si = 0;
    if (act) {
        oi = chain_off(a.lin, 0);
        si = UNI ? chain_off(a.lin, 1) - oi : 0;
    }
    auto in_at = [&](int s) -> long { return UNI ? oi + s * si : chain_off(a.lin, s); };

    // the hat entry first, then the chain; no load sits in a branch of its own (its wait
    // would come before the next load is issued): steps past the chain read step 0 and
    // are set to zero
    const bool has_hat = act && c < nh;
    const TIN hat_in = in[has_hat ? IDX(a.lin, line, c) : 0];
    double y[CL];
    if (act) {
#pragma unroll
        for (int s = 0; s < CL; ++s) {
            const TIN v = in[s < len ? in_at(s) : in_at(0)];
            y[s] = s < len ? (double)v : 0.0;
        }
    }
    if (has_hat) A[c] = (double)hat_in;
    if (UNI) __syncthreads();  // staged per-degree records

    // The scanning wavefront of a line: wave w handles lines w, w + nwaves, ...
    auto for_my_lines = [&](auto&& body) {
        for (int ll = wave; ll < LW; ll += nwaves) {
            const int ln = line_of(ll);
            if (ln >= 0 && ln < a.nlines) body(ll);
        }
    };

    if (MODE == SWEEP_FULL || MODE == SWEEP_SOLVE) {
        // ---- z = Lm^T y and the back substitution of S^{-1} z, fused (highest degree first)
        if (act) {
            double yo_next = 0.0, yp_next = 0.0;
#pragma unroll
            for (int s = CL - 1; s >= 0; --s) {
                if (s < len) {
                    const int m = pi + 2 * s;
                    const double yo = y[s];
                    double z = M_d(m) * yo;
                    double v = 0.0;
                    if (s + 1 < CL) {
                        if (s + 1 < len) {
                            z += M_lnk(m + 2) * yo_next;
                            v = S_lnk(m + 2) * yp_next;
                        }
                    }
                    const double yp = (z - v) * S_inv(m);
                    y[s] = yp;
                    yo_next = yo;
                    yp_next = yp;
                }
            }
            H1[c] = len > 0 ? yo_next : 0.0;  // heads of y
            H2[c] = len > 0 ? yp_next : 0.0;  // heads of L_S^{-T} z
        }
        __syncthreads();
        // ---- hats of z, right-hand side of the hat block of S, and its solve
        for_my_lines([&](int ll) {
            double* A2 = sA + ll * hs;
            const double* h1 = sH1 + ll * 2 * n;
            const double* h2 = sH2 + ll * 2 * n;
            for (int h = lane; h < nh; h += 64) {
                const double z = FM.d0[h] * A2[h] + FM.link0[h + 1] * (h + 1 < nh ? A2[h + 1] : 0.0) +
                                 head_coupling(FM.cpl, h1, d.bc, n, h);
                sB[ll * hs + h] = z - head_coupling(FS.cpl, h2, d.bc, n, h);
            }
            __builtin_amdgcn_wave_barrier();
            for (int h = lane; h < nh; h += 64) A2[h] = sB[ll * hs + h];
            __builtin_amdgcn_wave_barrier();
            hat_backward(A2, FS, nh, lane);
            __builtin_amdgcn_wave_barrier();
            hat_forward(A2, FS, nh, lane);
        });
        __syncthreads();
        // ---- forward substitution x = L_S^{-1} (y' - C x_h) (lowest degree first)
        double xl = 0.0, xr = 0.0;
        if (act) {
            if (vhat(d.bc, n, e)) xl = A[hov(d.bc, e)];
            if (vhat(d.bc, n, e + 1)) xr = A[hov(d.bc, e + 1)];
            double prev = 0.0;
#pragma unroll
            for (int s = 0; s < CL; ++s) {
                if (s < len) {
                    const int m = pi + 2 * s;
                    double v = y[s];
                    if (s == 0) v -= FS.cpl[4 * e + 2 * pi] * xl + FS.cpl[4 * e + 2 * pi + 1] * xr;
                    else v -= S_lnk(m) * prev;
                    prev = v * S_inv(m);
                    y[s] = prev;
                }
            }
            H1[c] = len > 0 ? y[0] : 0.0;  // heads of x
        }
        if (MODE == SWEEP_SOLVE) {
            TOUT* out = reinterpret_cast<TOUT*>(a.out);
            double sq = 0.0;
            if (act) {
                long oo = chain_off(a.lout, 0);
                const long so = UNI ? chain_off(a.lout, 1) - oo : 0;
#pragma unroll
                for (int s = 0; s < CL; ++s)
                    if (s < len) out[UNI ? oo + s * so : chain_off(a.lout, s)] = (TOUT)y[s];
                if (c < nh) out[IDX(a.lout, line, c)] = (TOUT)A[c];
                if (a.norm_acc) {
                    // |Lm w|^2 of this chain (and of hat c): the line's share of the squared
                    // norm of the correction in the norm of the ADI error lemma
#pragma unroll
                    for (int s = 0; s < CL; ++s)
                        if (s < len) {
                            const int m = pi + 2 * s;
                            double v = M_d(m) * y[s];
                            if (s == 0) v += FM.cpl[4 * e + 2 * pi] * xl + FM.cpl[4 * e + 2 * pi + 1] * xr;
                            else v += M_lnk(m) * y[s - 1];
                            sq += v * v;
                        }
                    if (c < nh) {
                        const double v = FM.d0[c] * A[c] + (c > 0 ? FM.link0[c] * A[c - 1] : 0.0);
                        sq += v * v;
                    }
                }
            }
            if (a.norm_acc) block_sum_atomic(sq, sm, a.norm_acc);
            return;
        }
        // ---- product v = (kappa K + tau M) x and u = Lm^{-T} v, fused (highest degree first)
        const double kap = a.kappa, tau = a.tau;
        if (act) {
            double x_next = 0.0, u_next = 0.0;
#pragma unroll
            for (int s = CL - 1; s >= 0; --s) {
                if (s < len) {
                    const int m = pi + 2 * s;
                    const double x = y[s];
                    double v = (kap * K_dg(m) + tau * M_dg(m)) * x;
                    double w = 0.0;
                    if (s > 0) v += tau * M_of(m - 2) * y[s - 1];
                    if (s + 1 < CL) {
                        if (s + 1 < len) {
                            v += tau * M_of(m) * x_next;
                            w = M_lnk(m + 2) * u_next;
                        }
                    }
                    if (s == 0) v += pi == 0 ? (tau * de) * (xl + xr) * (1.0 / 6.0) : (tau * de) * (xr - xl) * (1.0 / 30.0);
                    const double u = (v - w) * M_inv(m);
                    y[s] = u;
                    x_next = x;
                    u_next = u;
                }
            }
            H2[c] = len > 0 ? u_next : 0.0;  // heads of u
        }
        __syncthreads();
        // ---- hat rows of the product, right-hand side of the Lm^T hat block, its solve
        for_my_lines([&](int ll) {
            double* A2 = sA + ll * hs;
            double* B2 = sB + ll * hs;
            const double* hx = sH1 + ll * 2 * n;
            const double* hu = sH2 + ll * 2 * n;
            for (int h = lane; h < nh; h += 64) {
                const int v = voh(d.bc, h);
                const double xh = A2[h];
                double r = kap * robin_at(d, v) * xh;
                if (v >= 1) {
                    const int q = v - 1;
                    const double dq = d.delta[q], idq = d.invdelta[q];
                    r += (kap * idq + tau * dq * (1.0 / 3.0)) * xh;
                    if (vhat(d.bc, n, v - 1)) r += (-kap * idq + tau * dq * (1.0 / 6.0)) * A2[h - 1];
                    r += tau * dq * (hx[q] * (1.0 / 6.0) + hx[n + q] * (1.0 / 30.0));
                }
                if (v <= n - 1) {
                    const int q = v;
                    const double dq = d.delta[q], idq = d.invdelta[q];
                    r += (kap * idq + tau * dq * (1.0 / 3.0)) * xh;
                    if (vhat(d.bc, n, v + 1)) r += (-kap * idq + tau * dq * (1.0 / 6.0)) * A2[h + 1];
                    r += tau * dq * (hx[q] * (1.0 / 6.0) - hx[n + q] * (1.0 / 30.0));
                }
                B2[h] = r - head_coupling(FM.cpl, hu, d.bc, n, h);
            }
            __builtin_amdgcn_wave_barrier();
            hat_backward(B2, FM, nh, lane);
        });
        __syncthreads();
        const TIN* g = reinterpret_cast<const TIN*>(a.g);
        TOUT* out = reinterpret_cast<TOUT*>(a.out);
        if (act) {
            const long og = chain_off(a.lg, 0), oo = chain_off(a.lout, 0);
            const long sg = UNI ? chain_off(a.lg, 1) - og : 0, so = UNI ? chain_off(a.lout, 1) - oo : 0;
#pragma unroll
            for (int s = 0; s < CL; ++s)
                if (s < len) {
                    const long ig = UNI ? og + s * sg : chain_off(a.lg, s);
                    const long io = UNI ? oo + s * so : chain_off(a.lout, s);
                    out[io] = (TOUT)((double)g[ig] - y[s]);
                }
            if (c < nh) out[IDX(a.lout, line, c)] = (TOUT)((double)g[IDX(a.lg, line, c)] - B[c]);
        }
        return;
    }

    if (MODE == SWEEP_TRANSFORM) {
        // ---- u = Lm^{-T} y: chain back substitution, then the hat block
        if (act) {
            double u_next = 0.0;
#pragma unroll
            for (int s = CL - 1; s >= 0; --s) {
                if (s < len) {
                    const int m = pi + 2 * s;
                    double v = y[s];
                    if (s + 1 < CL) {
                        if (s + 1 < len) v -= M_lnk(m + 2) * u_next;
                    }
                    u_next = v * M_inv(m);
                    y[s] = u_next;
                }
            }
            H2[c] = len > 0 ? y[0] : 0.0;
        }
        __syncthreads();
        for_my_lines([&](int ll) {
            double* A2 = sA + ll * hs;
            const double* hu = sH2 + ll * 2 * n;
            for (int h = lane; h < nh; h += 64) A2[h] -= head_coupling(FM.cpl, hu, d.bc, n, h);
            __builtin_amdgcn_wave_barrier();
            hat_backward(A2, FM, nh, lane);
        });
        __syncthreads();
        TOUT* out = reinterpret_cast<TOUT*>(a.out);
        if (act) {
            const long oo = chain_off(a.lout, 0);
            const long so = UNI ? chain_off(a.lout, 1) - oo : 0;
#pragma unroll
            for (int s = 0; s < CL; ++s)
                if (s < len) out[UNI ? oo + s * so : chain_off(a.lout, s)] = (TOUT)y[s];
            if (c < nh) out[IDX(a.lout, line, c)] = (TOUT)A[c];
        }
        return;
    }

    if (MODE == SWEEP_FINAL) {
        // ---- u = Lm^{-1} w: hat block first (forward), then the chains (lowest degree first)
        __syncthreads();
        for_my_lines([&](int ll) { hat_forward(sA + ll * hs, FM, nh, lane); });
        __syncthreads();
        if (act) {
            double xl = 0.0, xr = 0.0;
            if (vhat(d.bc, n, e)) xl = A[hov(d.bc, e)];
            if (vhat(d.bc, n, e + 1)) xr = A[hov(d.bc, e + 1)];
            double* out = reinterpret_cast<double*>(a.out);
            double prev = 0.0;
#pragma unroll
            for (int s = 0; s < CL; ++s) {
                if (s < len) {
                    const int m = pi + 2 * s;
                    double v = y[s];
                    if (s == 0) v -= FM.cpl[4 * e + 2 * pi] * xl + FM.cpl[4 * e + 2 * pi + 1] * xr;
                    else v -= M_lnk(m) * prev;
                    prev = v * M_inv(m);
                    const long o = chain_off(a.lout, s);
                    out[o] = a.accumulate ? out[o] + prev : prev;
                }
            }
            if (c < nh) {
                const long o = IDX(a.lout, line, c);
                out[o] = a.accumulate ? out[o] + A[c] : A[c];
            }
        }
    }
}

// Per-degree coefficient records of a uniform mesh (see internal.h).
__global__ void coef_kernel(DimDev d, const double* facS, int stride, const double* facM, FactorLayout fl, double* out) {
    const int f = blockIdx.x;
    const int n = d.n, p = d.p;
    const double* S = facS + (size_t)f * stride;
    const double de = d.delta[0], ide = d.invdelta[0];
    for (int m = threadIdx.x; m < p; m += blockDim.x) {
        double* r = out + ((size_t)f * p + m) * 8;
        if (m == p - 1) {  // phantom degree p-1: zero coefficients make it inert in the recurrences
            for (int k = 0; k < 8; ++k) r[k] = 0.0;
            continue;
        }
        r[0] = S[fl.off_invd + m * n];
        r[1] = S[fl.off_link + m * n];
        r[2] = facM[fl.off_d + m * n];
        r[3] = facM[fl.off_link + m * n];
        r[4] = facM[fl.off_invd + m * n];
        r[5] = d.tab64[m] * ide;
        r[6] = d.tab64[d.tabstride + m] * de;
        r[7] = d.tab64[2 * d.tabstride + m] * de;
    }
}

template <typename TIN, typename TOUT, int CL, int MODE, bool COL, int LW>
hipError_t launch_lw(const DimDev& d, const SweepArgs& a, hipStream_t s) {
    constexpr int CW = 64 / LW;
    const int threads = 64 * ((2 * d.n + CW - 1) / CW);
    if (threads > sweep_max_threads(CL) || d.nh > 65) return hipErrorInvalidValue;
    const int blocks = (a.hpad_lines + a.nlines - a.nh_lines + LW - 1) / LW;
    const size_t lds = sweep_lds_bytes(d, threads, MODE);
    if (a.coef && d.n % CW == 0)
        hipLaunchKernelGGL((sweep_kernel<TIN, TOUT, CL, MODE, COL, true, LW>), dim3(blocks), dim3(threads), lds, s, d, a);
    else
        hipLaunchKernelGGL((sweep_kernel<TIN, TOUT, CL, MODE, COL, false, LW>), dim3(blocks), dim3(threads), lds, s, d, a);
    return hipGetLastError();
}

template <typename TIN, typename TOUT, int CL, int MODE, bool COL>
hipError_t launch_s(const DimDev& d, const SweepArgs& a, hipStream_t s) {
    return a.lpb == 4 ? launch_lw<TIN, TOUT, CL, MODE, COL, 4>(d, a, s) : launch_lw<TIN, TOUT, CL, MODE, COL, 8>(d, a, s);
}

template <typename TIN, typename TOUT, int MODE>
hipError_t by_cl(const DimDev& d, const SweepArgs& a, bool col, hipStream_t s) {
    const int need = d.p / 2;
#define HPADI_CASE(CLV)                                                                                   \
    if (need <= CLV)                                                                                      \
        return col ? launch_s<TIN, TOUT, CLV, MODE, true>(d, a, s) : launch_s<TIN, TOUT, CLV, MODE, false>(d, a, s);
    HPADI_CASE(4)
    HPADI_CASE(8)
    HPADI_CASE(16)
    HPADI_CASE(32)
    HPADI_CASE(64)
#undef HPADI_CASE
    return hipErrorInvalidValue;
}

}  // namespace

namespace sweep_detail {
size_t sweep_lds_bytes(const DimDev& d, int threads, int mode) {
    const int hs = d.nh + 1;
    size_t words = (size_t)8 * (2 * hs + 4 * d.n) + 2 * (3 * hs + 4 * d.n) + 8 * d.p;  // LW <= 8
    if (mode == SWEEP_FINAL && words < (size_t)threads * 2) words = (size_t)threads * 2;
    return words * sizeof(double);
}

}  // namespace sweep_detail

hipError_t launch_sweep(const DimDev& d, const SweepArgs& a, int mode, int tin, int tout, bool column,
                        hipStream_t s) {
    if (a.nlines <= 0) return hipSuccess;
    if (a.ptab && a.idx32 && sweep_uni_available(d, a.lpb)) return launch_sweep_uni(d, a, mode, tin, tout, column, s);
    switch (mode) {
        case SWEEP_FULL:
            if (tin == 4 && tout == 4) return by_cl<float, float, SWEEP_FULL>(d, a, column, s);
            if (tin == 8 && tout == 8) return by_cl<double, double, SWEEP_FULL>(d, a, column, s);
            break;
        case SWEEP_SOLVE:
            if (tin == 4 && tout == 4) return by_cl<float, float, SWEEP_SOLVE>(d, a, column, s);
            if (tin == 8 && tout == 8) return by_cl<double, double, SWEEP_SOLVE>(d, a, column, s);
            break;
        case SWEEP_TRANSFORM:
            if (tin == 8 && tout == 8) return by_cl<double, double, SWEEP_TRANSFORM>(d, a, column, s);
            if (tin == 8 && tout == 4) return by_cl<double, float, SWEEP_TRANSFORM>(d, a, column, s);
            break;
        case SWEEP_FINAL:
            if (tin == 4 && tout == 8) return by_cl<float, double, SWEEP_FINAL>(d, a, column, s);
            if (tin == 8 && tout == 8) return by_cl<double, double, SWEEP_FINAL>(d, a, column, s);
            break;
        default:
            break;
    }
    return hipErrorInvalidValue;
}

int sweep_threads(int n, int lines_per_block) {
    const int cw = 64 / lines_per_block;
    return 64 * ((2 * n + cw - 1) / cw);
}

namespace {
__global__ void pass_table_kernel(DimDev d, const double* facS, int stride, const double* facM, FactorLayout fl,
                                  const double* tau_dev, double kappa, double* out) {
    const int f = blockIdx.x;
    const int n = d.n, p = d.p;
    const double* S = facS + (size_t)f * stride;
    const double de = d.delta[0], ide = d.invdelta[0];
    const double tau = tau_dev ? tau_dev[f] : 0.0;
    const double* kd = d.tab64;
    const double* md = d.tab64 + d.tabstride;
    const double* mo = d.tab64 + 2 * d.tabstride;
    for (int m = threadIdx.x; m < p; m += blockDim.x) {
        double* r = out + ((size_t)f * p + m) * 16;
        for (int k = 0; k < 16; ++k) r[k] = 0.0;
        if (m > p - 2) continue;  // phantom degree p-1
        const bool up = m + 2 <= p - 2;
        const double sinv = S[fl.off_invd + m * n], minv = facM[fl.off_invd + m * n];
        const double slnk_up = up ? S[fl.off_link + (m + 2) * n] : 0.0;
        const double mlnk_up = up ? facM[fl.off_link + (m + 2) * n] : 0.0;
        const double slnk = m >= 2 ? S[fl.off_link + m * n] : 0.0;
        const double mlnk = m >= 2 ? facM[fl.off_link + m * n] : 0.0;
        r[0] = facM[fl.off_d + m * n] * sinv;
        r[1] = mlnk_up * sinv;
        r[2] = -slnk_up * sinv;
        r[3] = sinv;
        r[4] = -slnk * sinv;
        r[5] = minv * (kappa * kd[m] * ide + tau * md[m] * de);
        r[6] = m >= 2 ? minv * tau * mo[m - 2] * de : 0.0;
        r[7] = up ? minv * tau * mo[m] * de : 0.0;
        r[8] = -minv * mlnk_up;
        r[9] = minv;
        r[10] = -mlnk * minv;
        r[11] = -mlnk_up * minv;
        r[12] = minv * tau * de;
        r[13] = md[m] * de;  // diagonal of M at degree m
        r[14] = facM[fl.off_d + m * n];  // mass factor: diagonal and link to degree m - 2
        r[15] = mlnk;
    }
}
}  // namespace

hipError_t launch_pass_tables(const DimDev& d, int nf, const double* facS, int stride, const double* facM,
                              FactorLayout fl, const double* tau_dev, double kappa, double* out, hipStream_t s) {
    if (nf <= 0 || d.p < 2) return hipSuccess;
    hipLaunchKernelGGL(pass_table_kernel, dim3(nf), dim3(64), 0, s, d, facS, stride, facM, fl, tau_dev, kappa, out);
    return hipGetLastError();
}

hipError_t launch_coef_tables(const DimDev& d, int nf, const double* facS, int stride, const double* facM,
                              FactorLayout fl, double* out, hipStream_t s) {
    if (nf <= 0 || d.p < 2) return hipSuccess;
    hipLaunchKernelGGL(coef_kernel, dim3(nf), dim3(64), 0, s, d, facS, stride, facM, fl, out);
    return hipGetLastError();
}

}  // namespace hpadi
