// Uniform-mesh fast path of the mass-balanced half-sweeps (see sweep.hip for the
// method and the general kernel).
//
// On a mesh of equal elements the factor and operator entries depend only on the
// degree m, so they come from one per-degree record table; with n a multiple of the
// chains per wavefront every wavefront has one parity, so they are wavefront-uniform
// (read through the scalar cache, or from lane copies in the chain recurrences of the
// full half-sweeps and the transform passes).  The chain length is a
// compile-time constant CL = p/2; a chain one degree shorter (odd parity, even
// p) is padded by a phantom degree whose coefficients are zero, which makes it
// inert in every recurrence, so the unrolled chain loops carry no per-step
// branches.  Offsets are 32-bit (the host only selects this path when every
// array has fewer than 2^31 entries).

#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"
#include "sweep_common.h"

namespace hpadi {

using namespace sweep_detail;

namespace {

typedef const __attribute__((address_space(4))) double* cptr;

// The half-sweep of workgroup bid (of nblk) of one problem; d and a may live in kernel
// arguments or in a device task table (grouped launches).
// standalone: the workgroup index is the hardware one (workgroup b runs on XCD b mod 8),
// so the line-to-workgroup mapping may be made XCD-aware.
template <typename TIN, typename TOUT, int CL, int MODE, bool COL, int LW>
__device__ __forceinline__ void sweep_uni_body(const DimDev& d, const SweepArgs& a, int bid, int nblk,
                                               bool standalone) {
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

    // Workgroups that share cache lines (a row pass covering only part of each 128-byte
    // line of a panel, e.g. 4 rows of 16 bytes in FP32; a column pass covering fewer
    // columns than a panel holds, whose workgroups share every sector) are xcd_group
    // consecutive workgroups: they run on one XCD (workgroup b runs on XCD b mod 8) in
    // consecutive dispatch slots, so each line is fetched into that XCD's L2 once
    // instead of once per XCD.
    int blk = bid;
    if (standalone && a.xcd_group > 1) {
        const int g = a.xcd_group;
        const int full = (nblk / (8 * g)) * (8 * g);
        if (blk < full) {
            const int xcd = blk % 8, slot = blk / 8;
            blk = (slot / g) * (8 * g) + xcd * g + slot % g;
        }
    }
    auto line_of = [&](int ll) -> int {
        const int lint = blk * LW + ll;
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
    const cptr pt = (cptr)(a.ptab);
    auto PT = [&](int m, int k) -> double { return pt[m * 16 + k]; };

    // Full half-sweeps with chains of 32 or more steps: the two chain recurrences take their
    // per-step coefficients from lane copies (lane s holds the coefficient of chain step s,
    // degree pi + 2s, read back with readlane), so the unrolled chains do not wait on a
    // scalar load at every step.  A copy is valid only where the whole wavefront wrote it:
    // the copies are loaded outside every lane-dependent branch and pinned there by an
    // empty asm that consumes them, so the compiler cannot sink the loads into a branch
    // that masks off lanes (lanes of missing lines would then keep stale copies).  Shorter
    // chains keep the scalar loads (the compiler hoists all their readlanes and spills
    // scalar registers).
    constexpr bool kLaneCoef = MODE == SWEEP_FULL && CL >= 32;
    auto lane_coef = [&](int k) -> double { return lane < CL ? a.ptab[(pi + 2 * lane) * 16 + k] : 0.0; };
    auto pin = [](double& v) { asm volatile("" : "+v"(v)); };
    auto lane_read = [](double v, int s) -> double {
        const int lo = __builtin_amdgcn_readlane(__double2loint(v), s);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(v), s);
        return __hiloint2double(hi, lo);
    };
    auto RL = [&](double v, int s, int k) -> double {
        if constexpr (!kLaneCoef) {
            (void)v;
            return PT(pi + 2 * s, k);
        } else {
            return lane_read(v, s);
        }
    };
    // the transform passes take the two coefficients of their one recurrence the same way
    // (the final pass keeps the scalar loads: its registers hold the previous solution too)
    constexpr bool kLaneT = MODE == SWEEP_TRANSFORM && CL >= 32;
    auto RT = [&](double v, int s, int k) -> double {
        if constexpr (!kLaneT) {
            (void)v;
            return PT(pi + 2 * s, k);
        } else {
            return lane_read(v, s);
        }
    };
    // issued ahead of the chain loads: loads complete in order, so waiting for these
    // does not wait for the chains
    double cb0 = 0.0, cb1 = 0.0, cb2 = 0.0;
    if constexpr (kLaneCoef) {
        cb0 = lane_coef(0);
        cb1 = lane_coef(1);
        cb2 = lane_coef(2);
    }
    double ct0 = 0.0, ct1 = 0.0;
    if constexpr (kLaneT) {
        ct0 = lane_coef(9);
        ct1 = lane_coef(11);
    }

    auto IDX = [&](const Layout& L, int ln, int pos) -> long { return COL ? addr(L, pos, ln) : addr(L, ln, pos); };
    // byte offset of chain step 0 and byte stride per step (32-bit: loads and stores
    // address a uniform base plus a per-lane 32-bit offset)
    auto chain0 = [&](const Layout& L, unsigned& o, unsigned& st, unsigned esz) {
        const long o0 = IDX(L, line, nh + c);
        o = (unsigned)(o0 * esz);
        st = (unsigned)((IDX(L, line, nh + 2 * n + c) - o0) * esz);
    };

    const char* inb = reinterpret_cast<const char*>(a.in);
    const TIN* in = reinterpret_cast<const TIN*>(a.in);
    // the hat entry of the lane, issued ahead of the chains (loads complete in order, so
    // its LDS write below waits for it alone); lanes without one read entry 0
    const bool has_hat = act && c < nh;
    const TIN hat_in = in[has_hat ? IDX(a.lin, line, c) : 0];
    double y[CL];
    if (act) {
        // issued highest degree first: the first recurrence consumes them in that order;
        // no load sits in a branch of its own (its wait would come before the next issue):
        // the phantom degree reads the step below it and drops the value
        unsigned o, st;
        chain0(a.lin, o, st, sizeof(TIN));
        o += (CL - 1) * st;
        const TIN top = *reinterpret_cast<const TIN*>(inb + (full ? o : o - st));
        y[CL - 1] = full ? (double)top : 0.0;
#pragma unroll
        for (int s = CL - 2; s >= 0; --s) {
            o -= st;
            y[s] = (double)*reinterpret_cast<const TIN*>(inb + o);
        }
    }
    double* A = sA + l * hs;
    double* B = sB + l * hs;
    double* H1 = sH1 + l * 2 * n;
    double* H2 = sH2 + l * 2 * n;
    if (has_hat) A[c] = (double)hat_in;

    auto for_my_lines = [&](auto&& body) {
        for (int ll = wave; ll < LW; ll += nwaves) {
            const int ln = line_of(ll);
            if (ln >= 0 && ln < a.nlines) body(ll);
        }
    };
    auto store_chain = [&](TOUT* out, const Layout& L, auto&& value) {
        unsigned o, st;
        chain0(L, o, st, sizeof(TOUT));
        char* ob = reinterpret_cast<char*>(out);
#pragma unroll
        for (int s = 0; s < CL - 1; ++s) {
            *reinterpret_cast<TOUT*>(ob + o) = (TOUT)value(s);
            o += st;
        }
        if (full) *reinterpret_cast<TOUT*>(ob + o) = (TOUT)value(CL - 1);
    };

    if (MODE == SWEEP_FULL || MODE == SWEEP_SOLVE) {
        if constexpr (kLaneCoef) {
            pin(cb0);
            pin(cb1);
            pin(cb2);
        }
        // z = Lm^T y and the back substitution of S^{-1} z, fused (highest degree first):
        // y'_s = b1 y_s + b2 y_{s+1} + b3 y'_{s+1}
        if (act) {
            double yo_n = 0.0, yp_n = 0.0;
#pragma unroll
            for (int s = CL - 1; s >= 0; --s) {
                const int m = pi + 2 * s;
                const double yo = y[s];
                double yp = RL(cb0, s, 0) * yo;
                if (s + 1 < CL) yp += RL(cb1, s, 1) * yo_n + RL(cb2, s, 2) * yp_n;
                y[s] = yp;
                yo_n = yo;
                yp_n = yp;
            }
            H1[c] = yo_n;
            H2[c] = yp_n;
        }
        double cf3 = 0.0, cf4 = 0.0;
        if constexpr (kLaneCoef) {
            cf3 = lane_coef(3);
            cf4 = lane_coef(4);
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
        if constexpr (kLaneCoef) {
            pin(cf3);
            pin(cf4);
        }
        double xl = 0.0, xr = 0.0;
        if (act) {
            if (vhat(d.bc, n, e)) xl = A[hov(d.bc, e)];
            if (vhat(d.bc, n, e + 1)) xr = A[hov(d.bc, e + 1)];
            // x_s = c1 y'_s + c2 x_{s-1}; the head also removes the hat coupling
            double prev = 0.0;
#pragma unroll
            for (int s = 0; s < CL; ++s) {
                const int m = pi + 2 * s;
                if (s == 0) prev = (y[0] - FS.cpl[4 * e + 2 * pi] * xl - FS.cpl[4 * e + 2 * pi + 1] * xr) * RL(cf3, 0, 3);
                else prev = RL(cf3, s, 3) * y[s] + RL(cf4, s, 4) * prev;
                y[s] = prev;
            }
            H1[c] = y[0];
        }
        if (MODE == SWEEP_SOLVE) {
            double sq = 0.0;
            if (act) {
                TOUT* out = reinterpret_cast<TOUT*>(a.out);
                store_chain(out, a.lout, [&](int s) { return y[s]; });
                if (c < nh) out[IDX(a.lout, line, c)] = (TOUT)A[c];
                if (a.norm_acc) {
                    // |Lm w|^2 of this chain (and of hat c): the line's share of the squared
                    // norm of the correction in the norm of the ADI error lemma
                    double prev = 0.0;
#pragma unroll
                    for (int s = 0; s < CL; ++s) {
                        const int m = pi + 2 * s;
                        double v = PT(m, 14) * y[s];
                        if (s == 0) v += FM.cpl[4 * e + 2 * pi] * xl + FM.cpl[4 * e + 2 * pi + 1] * xr;
                        else v += PT(m, 15) * prev;
                        sq += v * v;
                        prev = y[s];
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
        const double kap = a.kappa, tau = a.tau;
        // product v = (kappa K + tau M) x and u = Lm^{-T} v on the chains, highest degree
        // first; a bubble entry of u is final once computed (the hat block of Lm^T does not
        // feed back into the bubbles), so g - u is stored as it is produced.
        // G~ of the chain is loaded ahead of the recurrence (all of it for FP32, in two
        // halves for FP64), so the loads do not wait one by one behind the output stores.
        constexpr int PF = (sizeof(TIN) == 4 || CL < 16) ? CL : CL / 2;
        TIN gv[CL];
        const char* gb = reinterpret_cast<const char*>(a.g);
        unsigned og0, sg;
        chain0(a.lg, og0, sg, sizeof(TIN));
        auto load_g = [&](int s) {
            // the phantom step and inactive lanes read the array's first entry (unused)
            const bool real = act && (s < CL - 1 || full);
            gv[s] = *reinterpret_cast<const TIN*>(gb + (real ? og0 + (unsigned)s * sg : 0u));
        };
#pragma unroll
        for (int s = CL - 1; s >= CL - PF; --s) load_g(s);  // in the order they are consumed
        if (act) {
            char* ob = reinterpret_cast<char*>(a.out);
            unsigned oo, so;
            chain0(a.lout, oo, so, sizeof(TOUT));
            oo += (CL - 1) * so;
            const double hterm = pi == 0 ? (xl + xr) * (1.0 / 6.0) : (xr - xl) * (1.0 / 30.0);
            double x_n = 0.0, u_n = 0.0;
            // u_s = a1 x_s + a2 x_{s-1} + a3 x_{s+1} + a4 u_{s+1} (+ the hat term at the head)
#pragma unroll
            for (int s = CL - 1; s >= 0; --s) {
                if (PF < CL && s == CL - PF) {
#pragma unroll
                    for (int s2 = CL - PF - 1; s2 >= 0; --s2) load_g(s2);
                }
                const int m = pi + 2 * s;
                const double x = y[s];
                double u = PT(m, 5) * x;
                if (s > 0) u += PT(m, 6) * y[s - 1];
                if (s + 1 < CL) u += PT(m, 7) * x_n + PT(m, 8) * u_n;
                if (s == 0) u += PT(m, 12) * hterm;
                if (s < CL - 1 || full) *reinterpret_cast<TOUT*>(ob + oo) = (TOUT)((double)gv[s] - u);
                oo -= so;
                x_n = x;
                u_n = u;
            }
            H2[c] = u_n;
        }
        // G~ of the lane's hat, issued before the hat block (its latency hides there)
        const TIN g_hat = reinterpret_cast<const TIN*>(a.g)[has_hat ? IDX(a.lg, line, c) : 0];
        // equal elements: one width (through the scalar cache, so that the hat block
        // waits on no vector load, which would also wait for the stores above)
        const double dq = ((cptr)d.delta)[0], idq = ((cptr)d.invdelta)[0];
        __syncthreads();
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
                    r += (kap * idq + tau * dq * (1.0 / 3.0)) * xh;
                    if (vhat(d.bc, n, v - 1)) r += (-kap * idq + tau * dq * (1.0 / 6.0)) * A2[h - 1];
                    r += tau * dq * (hx[q] * (1.0 / 6.0) + hx[n + q] * (1.0 / 30.0));
                }
                if (v <= n - 1) {
                    const int q = v;
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
        if (has_hat) {
            TOUT* out = reinterpret_cast<TOUT*>(a.out);
            out[IDX(a.lout, line, c)] = (TOUT)((double)g_hat - B[c]);
        }
        return;
    }

    if constexpr (kLaneT) {
        pin(ct0);
        pin(ct1);
    }
    if (MODE == SWEEP_TRANSFORM) {
        // u = Lm^{-T} y: chain back substitution (entries final as computed, stored at once),
        // then the hat block
        if (act) {
            char* ob = reinterpret_cast<char*>(a.out);
            unsigned oo, so;
            chain0(a.lout, oo, so, sizeof(TOUT));
            oo += (CL - 1) * so;
            double u_n = 0.0;
#pragma unroll
            for (int s = CL - 1; s >= 0; --s) {
                const int m = pi + 2 * s;
                u_n = RT(ct0, s, 9) * y[s] + (s + 1 < CL ? RT(ct1, s, 11) * u_n : 0.0);
                if (s < CL - 1 || full) *reinterpret_cast<TOUT*>(ob + oo) = (TOUT)u_n;
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
        if (act) {
            double xl = 0.0, xr = 0.0;
            if (vhat(d.bc, n, e)) xl = A[hov(d.bc, e)];
            if (vhat(d.bc, n, e + 1)) xr = A[hov(d.bc, e + 1)];
            double prev = 0.0;
            double* out = reinterpret_cast<double*>(a.out);
            char* ob = reinterpret_cast<char*>(a.out);
            unsigned o0, st;
            chain0(a.lout, o0, st, sizeof(double));
            // previous U of the chain, loaded in two halves ahead of the stores
            constexpr int PH = CL < 16 ? CL : CL / 2;
            double uo[CL];
            auto load_u = [&](int s) {
                const bool real = a.accumulate && (s < CL - 1 || full);
                uo[s] = real ? *reinterpret_cast<const double*>(ob + o0 + (unsigned)s * st) : 0.0;
            };
#pragma unroll
            for (int s = 0; s < PH; ++s) load_u(s);
#pragma unroll
            for (int s = 0; s < CL; ++s) {
                if (PH < CL && s == PH / 2) {
#pragma unroll
                    for (int s2 = PH; s2 < CL; ++s2) load_u(s2);
                }
                const int m = pi + 2 * s;
                if (s == 0) prev = (y[0] - FM.cpl[4 * e + 2 * pi] * xl - FM.cpl[4 * e + 2 * pi + 1] * xr) * PT(m, 9);
                else prev = PT(m, 9) * y[s] + PT(m, 10) * prev;
                if (s < CL - 1 || full) *reinterpret_cast<double*>(ob + o0 + (unsigned)s * st) = uo[s] + prev;
            }
            if (c < nh) {
                const long oh = IDX(a.lout, line, c);
                out[oh] = a.accumulate ? out[oh] + A[c] : A[c];
            }
        }
    }
}

}  // namespace
}  // namespace hpadi
