// Uniform-mesh fast path of the mass-balanced half-sweeps (see sweep.hip for the
// method and the general kernel).
//
// On a mesh of equal elements the factor and operator entries depend only on the
// degree m, so they are read from one per-degree record table through the scalar
// cache; with n a multiple of the chains per wavefront every wavefront has one
// parity, so those reads are wavefront-uniform.  The chain length is a
// compile-time constant CL = p/2; a chain one degree shorter (odd parity, even
// p) is padded by a phantom degree whose coefficients are zero, which makes it
// inert in every recurrence, so the unrolled chain loops carry no per-step
// branches.  Offsets are 32-bit (the host only selects this path when every
// array has fewer than 2^31 entries).

#include <hip/hip_runtime.h>

#include "internal.h"
#include "sweep_common.h"

namespace hpadi {

using namespace sweep_detail;

namespace {

typedef const __attribute__((address_space(4))) double* cptr;

template <typename TIN, typename TOUT, int CL, int MODE, bool COL, int LW>
__global__ void __launch_bounds__(sweep_max_threads(CL)) sweep_uni_kernel(DimDev d, SweepArgs a) {
    constexpr int CW = 64 / LW;
    extern __shared__ double sm[];
    const int n = d.n, p = d.p, nh = d.nh;
    const int hs = nh + 1;
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

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
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

    auto line_of = [&](int ll) -> int {
        const int lint = blockIdx.x * LW + ll;
        if (lint < a.nh_lines) return lint;
        if (lint < a.hpad_lines) return -1;
        return lint - (a.hpad_lines - a.nh_lines);
    };
    const int line = line_of(l);
    const bool lact = line >= 0 && line < a.nlines;
    const bool act = lact && c < 2 * n;
    const int pi = __builtin_amdgcn_readfirstlane(c >= n ? 1 : 0);
    const int e = c - pi * n;
    const bool full = (pi ? (p - 1) / 2 : p / 2) == CL;  // else the last step is the phantom degree
    const cptr cf = (cptr)(a.coef);
    auto CF = [&](int m, int k) -> double { return cf[m * 8 + k]; };

    auto IDX = [&](const Layout& L, int ln, int pos) -> long { return COL ? addr(L, pos, ln) : addr(L, ln, pos); };
    auto chain0 = [&](const Layout& L, int& o, int& st) {
        const long o0 = IDX(L, line, nh + c);
        o = (int)o0;
        st = (int)(IDX(L, line, nh + 2 * n + c) - o0);
    };

    const TIN* in = reinterpret_cast<const TIN*>(a.in);
    double y[CL];
    if (act) {
        // issued highest degree first: the first recurrence consumes them in that order
        int o, st;
        chain0(a.lin, o, st);
        o += (CL - 1) * st;
        y[CL - 1] = full ? (double)in[o] : 0.0;
#pragma unroll
        for (int s = CL - 2; s >= 0; --s) {
            o -= st;
            y[s] = (double)in[o];
        }
    }
    double* A = sA + l * hs;
    double* B = sB + l * hs;
    double* H1 = sH1 + l * 2 * n;
    double* H2 = sH2 + l * 2 * n;
    if (act && c < nh) A[c] = (double)in[IDX(a.lin, line, c)];

    auto for_my_lines = [&](auto&& body) {
        for (int ll = wave; ll < LW; ll += nwaves) {
            const int ln = line_of(ll);
            if (ln >= 0 && ln < a.nlines) body(ll);
        }
    };
    auto store_chain = [&](TOUT* out, const Layout& L, auto&& value) {
        int o, st;
        chain0(L, o, st);
#pragma unroll
        for (int s = 0; s < CL - 1; ++s) {
            out[o] = (TOUT)value(s, o);
            o += st;
        }
        if (full) out[o] = (TOUT)value(CL - 1, o);
    };

    if (MODE == SWEEP_FULL || MODE == SWEEP_SOLVE) {
        // z = Lm^T y and the back substitution of S^{-1} z, fused (highest degree first)
        if (act) {
            double yo_n = 0.0, yp_n = 0.0;
#pragma unroll
            for (int s = CL - 1; s >= 0; --s) {
                const int m = pi + 2 * s;
                const double yo = y[s];
                double z = CF(m, 2) * yo;
                double v = 0.0;
                if (s + 1 < CL) {
                    z += CF(m + 2, 3) * yo_n;
                    v = CF(m + 2, 1) * yp_n;
                }
                const double yp = (z - v) * CF(m, 0);
                y[s] = yp;
                yo_n = yo;
                yp_n = yp;
            }
            H1[c] = yo_n;
            H2[c] = yp_n;
        }
        __syncthreads();
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
        double xl = 0.0, xr = 0.0;
        if (act) {
            if (vhat(d.bc, n, e)) xl = A[hov(d.bc, e)];
            if (vhat(d.bc, n, e + 1)) xr = A[hov(d.bc, e + 1)];
            double prev = 0.0;
#pragma unroll
            for (int s = 0; s < CL; ++s) {
                const int m = pi + 2 * s;
                double v = y[s];
                if (s == 0) v -= FS.cpl[4 * e + 2 * pi] * xl + FS.cpl[4 * e + 2 * pi + 1] * xr;
                else v -= CF(m, 1) * prev;
                prev = v * CF(m, 0);
                y[s] = prev;
            }
            H1[c] = y[0];
        }
        if (MODE == SWEEP_SOLVE) {
            if (act) {
                TOUT* out = reinterpret_cast<TOUT*>(a.out);
                store_chain(out, a.lout, [&](int s, int) { return y[s]; });
                if (c < nh) out[IDX(a.lout, line, c)] = (TOUT)A[c];
            }
            return;
        }
        const double kap = a.kappa, tau = a.tau;
        // product v = (kappa K + tau M) x and u = Lm^{-T} v on the chains, highest degree
        // first; a bubble entry of u is final once computed (the hat block of Lm^T does not
        // feed back into the bubbles), so g - u is stored as it is produced.
        if (act) {
            const TIN* g = reinterpret_cast<const TIN*>(a.g);
            TOUT* out = reinterpret_cast<TOUT*>(a.out);
            int og, sg, oo, so;
            chain0(a.lg, og, sg);
            chain0(a.lout, oo, so);
            og += (CL - 1) * sg;
            oo += (CL - 1) * so;
            const double tde = tau * d.delta[0];
            double x_n = 0.0, u_n = 0.0;
#pragma unroll
            for (int s = CL - 1; s >= 0; --s) {
                const int m = pi + 2 * s;
                const double x = y[s];
                double v = (kap * CF(m, 5) + tau * CF(m, 6)) * x;
                double w = 0.0;
                if (s > 0) v += tau * CF(m - 2, 7) * y[s - 1];
                if (s + 1 < CL) {
                    v += tau * CF(m, 7) * x_n;
                    w = CF(m + 2, 3) * u_n;
                }
                if (s == 0) v += pi == 0 ? tde * (xl + xr) * (1.0 / 6.0) : tde * (xr - xl) * (1.0 / 30.0);
                const double u = (v - w) * CF(m, 4);
                if (s < CL - 1 || full) out[oo] = (TOUT)((double)g[og] - u);
                og -= sg;
                oo -= so;
                x_n = x;
                u_n = u;
            }
            H2[c] = u_n;
        }
        __syncthreads();
        for_my_lines([&](int ll) {
            double* A2 = sA + ll * hs;
            double* B2 = sB + ll * hs;
            const double* hx = sH1 + ll * 2 * n;
            const double* hu = sH2 + ll * 2 * n;
            for (int h = lane; h < nh; h += 64) {
                const int v = voh(d.bc, h);
                const double xh = A2[h];
                double r = 0.0;
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
        if (act && c < nh) {
            const TIN* g = reinterpret_cast<const TIN*>(a.g);
            TOUT* out = reinterpret_cast<TOUT*>(a.out);
            out[IDX(a.lout, line, c)] = (TOUT)((double)g[IDX(a.lg, line, c)] - B[c]);
        }
        return;
    }

    if (MODE == SWEEP_TRANSFORM) {
        // u = Lm^{-T} y: chain back substitution (entries final as computed, stored at once),
        // then the hat block
        if (act) {
            TOUT* out = reinterpret_cast<TOUT*>(a.out);
            int oo, so;
            chain0(a.lout, oo, so);
            oo += (CL - 1) * so;
            double u_n = 0.0;
#pragma unroll
            for (int s = CL - 1; s >= 0; --s) {
                const int m = pi + 2 * s;
                double v = y[s];
                if (s + 1 < CL) v -= CF(m + 2, 3) * u_n;
                u_n = v * CF(m, 4);
                if (s < CL - 1 || full) out[oo] = (TOUT)u_n;
                oo -= so;
            }
            H2[c] = u_n;
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
        if (act && c < nh) {
            TOUT* out = reinterpret_cast<TOUT*>(a.out);
            out[IDX(a.lout, line, c)] = (TOUT)A[c];
        }
        return;
    }

    if (MODE == SWEEP_FINAL) {
        __syncthreads();
        for_my_lines([&](int ll) { hat_forward(sA + ll * hs, FM, nh, lane); });
        __syncthreads();
        double sdx = 0.0, su = 0.0;
        if (act) {
            double xl = 0.0, xr = 0.0;
            if (vhat(d.bc, n, e)) xl = A[hov(d.bc, e)];
            if (vhat(d.bc, n, e + 1)) xr = A[hov(d.bc, e + 1)];
            double prev = 0.0;
#pragma unroll
            for (int s = 0; s < CL; ++s) {
                const int m = pi + 2 * s;
                double v = y[s];
                if (s == 0) v -= FM.cpl[4 * e + 2 * pi] * xl + FM.cpl[4 * e + 2 * pi + 1] * xr;
                else v -= CF(m, 3) * prev;
                prev = v * CF(m, 4);
                y[s] = prev;
            }
            double* out = reinterpret_cast<double*>(a.out);
            const double* w = d.mdiag;
            int o, st;
            chain0(a.lout, o, st);
#pragma unroll
            for (int s = 0; s < CL; ++s) {
                if (s < CL - 1 || full) {
                    const int pos = nh + 2 * s * n + c;
                    const double u = a.accumulate ? out[o] + y[s] : y[s];
                    out[o] = u;
                    sdx += w[pos] * y[s] * y[s];
                    su += w[pos] * u * u;
                }
                o += st;
            }
            if (c < nh) {
                const long oh = IDX(a.lout, line, c);
                const double dx = A[c];
                const double u = a.accumulate ? out[oh] + dx : dx;
                out[oh] = u;
                sdx += w[c] * dx * dx;
                su += w[c] * u * u;
            }
            if (a.norm_acc) {
                const double wl = a.wline[line];
                sdx *= wl;
                su *= wl;
            }
        }
        if (a.norm_acc) {
            __syncthreads();
            sm[2 * tid] = sdx;
            sm[2 * tid + 1] = su;
            __syncthreads();
            for (int w2 = blockDim.x; w2 > 1; w2 = (w2 + 1) / 2) {
                const int half = (w2 + 1) / 2;
                if (tid + half < w2) {
                    sm[2 * tid] += sm[2 * (tid + half)];
                    sm[2 * tid + 1] += sm[2 * (tid + half) + 1];
                }
                __syncthreads();
            }
            if (tid == 0) {
                atomicAdd(a.norm_acc + 0, sm[0]);
                atomicAdd(a.norm_acc + 1, sm[1]);
            }
        }
    }
}

template <typename TIN, typename TOUT, int CL, int MODE, bool COL, int LW>
hipError_t launch_u(const DimDev& d, const SweepArgs& a, hipStream_t s) {
    constexpr int CW = 64 / LW;
    const int threads = 64 * ((2 * d.n + CW - 1) / CW);
    if (threads > sweep_max_threads(CL) || d.nh > 65) return hipErrorInvalidValue;
    const int blocks = (a.hpad_lines + a.nlines - a.nh_lines + LW - 1) / LW;
    hipLaunchKernelGGL((sweep_uni_kernel<TIN, TOUT, CL, MODE, COL, LW>), dim3(blocks), dim3(threads),
                       sweep_lds_bytes(d, threads, MODE), s, d, a);
    return hipGetLastError();
}

template <typename TIN, typename TOUT, int CL, int MODE>
hipError_t by_dir(const DimDev& d, const SweepArgs& a, bool col, hipStream_t s) {
    if (a.lpb == 4) return col ? launch_u<TIN, TOUT, CL, MODE, true, 4>(d, a, s) : launch_u<TIN, TOUT, CL, MODE, false, 4>(d, a, s);
    return col ? launch_u<TIN, TOUT, CL, MODE, true, 8>(d, a, s) : launch_u<TIN, TOUT, CL, MODE, false, 8>(d, a, s);
}

template <typename TIN, typename TOUT, int MODE>
hipError_t by_cl(const DimDev& d, const SweepArgs& a, bool col, hipStream_t s) {
    switch (d.p / 2) {
        case 4: return by_dir<TIN, TOUT, 4, MODE>(d, a, col, s);
        case 8: return by_dir<TIN, TOUT, 8, MODE>(d, a, col, s);
        case 16: return by_dir<TIN, TOUT, 16, MODE>(d, a, col, s);
        case 32: return by_dir<TIN, TOUT, 32, MODE>(d, a, col, s);
        case 64: return by_dir<TIN, TOUT, 64, MODE>(d, a, col, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool sweep_uni_available(const DimDev& d, int lines_per_block) {
    const int cw = 64 / lines_per_block;
    const int cl = d.p / 2;
    return d.n % cw == 0 && (cl == 4 || cl == 8 || cl == 16 || cl == 32 || cl == 64) && d.nh <= 65;
}

hipError_t launch_sweep_uni(const DimDev& d, const SweepArgs& a, int mode, int tin, int tout, bool column,
                            hipStream_t s) {
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

}  // namespace hpadi
