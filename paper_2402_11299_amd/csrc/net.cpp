// Host side of the learned correction: parameters, workspace, forward and
// backward passes, Adam training, training pairs from the Krylov iterates and
// the correction applied inside the Krylov loop.  Declared in include/hpadi.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "hpadi.h"
#include "krylov.h"
#include "krylov_internal.h"
#include "net.h"

using hpadi::bf16_t;
using hpadi::ImgShape;
using hpadi_host::dmalloc;

namespace {

// splitmix64 (Steele, Lea and Flood 2014): a counter-based 64-bit generator
uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
double uniform01(uint64_t seed, uint64_t ctr) { return (splitmix64(seed ^ splitmix64(ctr)) >> 11) * 0x1.0p-53; }

}  // namespace

struct hpadi_net_s {
    hipStream_t stream = nullptr;
    float* params = nullptr;
    float* grads = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    bf16_t *wf1 = nullptr, *wb1 = nullptr, *wf2 = nullptr, *wb2 = nullptr;
    int step = 0;
    // workspace for up to cap pixels
    size_t cap = 0;
    bool train_ws = false;
    float *x = nullptr, *zn = nullptr, *t = nullptr, *w = nullptr, *out = nullptr, *g = nullptr;
    float *pre0 = nullptr, *pre1 = nullptr, *pre2 = nullptr;
    bf16_t *a0 = nullptr, *a1 = nullptr, *a2 = nullptr, *ga = nullptr, *gb = nullptr;
    double* num_den = nullptr;
    double* num_den_host = nullptr;
    int nd_cap = 0;
    int* idx = nullptr;
    int idx_cap = 0;
    double damping = 0.0;         // > 0: z <- z + damping c; 0: energy-optimal combination
    int period = 1;               // correct the preconditioned residual at every period-th iteration

    void free_ws() {
        for (void* p : {(void*)x, (void*)zn, (void*)t, (void*)w, (void*)out, (void*)g, (void*)pre0, (void*)pre1,
                        (void*)pre2, (void*)a0, (void*)a1, (void*)a2, (void*)ga, (void*)gb})
            (void)hipFree(p);
        x = zn = t = w = out = g = pre0 = pre1 = pre2 = nullptr;
        a0 = a1 = a2 = ga = gb = nullptr;
        cap = 0;
    }
    ~hpadi_net_s() {
        if (stream) (void)hipStreamSynchronize(stream);
        free_ws();
        for (void* p : {(void*)params, (void*)grads, (void*)m, (void*)v, (void*)wf1, (void*)wb1, (void*)wf2,
                        (void*)wb2, (void*)num_den, (void*)idx})
            (void)hipFree(p);
        if (num_den_host) (void)hipHostFree(num_den_host);
    }
};

namespace {

// Workspace for npix pixels; training needs the pre-activations and gradient images.
int ensure_ws(hpadi_net_s* N, size_t npix, bool train) {
    if (npix <= N->cap && (!train || N->train_ws)) return HPADI_OK;
    if (N->stream) (void)hipStreamSynchronize(N->stream);
    N->free_ws();
    const size_t C = hpadi::kNetC;
    bool ok = dmalloc(&N->out, npix) == hipSuccess && dmalloc(&N->a0, C * npix) == hipSuccess &&
              dmalloc(&N->a1, C * npix) == hipSuccess;
    if (ok && train)
        ok = dmalloc(&N->x, 3 * npix) == hipSuccess && dmalloc(&N->zn, npix) == hipSuccess &&
             dmalloc(&N->t, npix) == hipSuccess && dmalloc(&N->w, npix) == hipSuccess &&
             dmalloc(&N->g, npix) == hipSuccess && dmalloc(&N->pre0, C * npix) == hipSuccess &&
             dmalloc(&N->pre1, C * npix) == hipSuccess && dmalloc(&N->pre2, C * npix) == hipSuccess &&
             dmalloc(&N->a2, C * npix) == hipSuccess && dmalloc(&N->ga, C * npix) == hipSuccess &&
             dmalloc(&N->gb, C * npix) == hipSuccess;
    if (!ok) {
        N->free_ws();
        return HPADI_ENOMEM;
    }
    N->cap = npix;
    N->train_ws = train;
    return HPADI_OK;
}

int ensure_nd(hpadi_net_s* N, int B) {
    if (B <= N->nd_cap) return HPADI_OK;
    (void)hipFree(N->num_den);
    if (N->num_den_host) (void)hipHostFree(N->num_den_host);
    N->num_den = nullptr;
    N->num_den_host = nullptr;
    if (dmalloc(&N->num_den, 2 * (size_t)B) != hipSuccess ||
        hipHostMalloc((void**)&N->num_den_host, 2 * (size_t)B * sizeof(double)) != hipSuccess)
        return HPADI_ENOMEM;
    N->nd_cap = B;
    return HPADI_OK;
}

#define HIPCHK(call)                              \
    do {                                          \
        if ((call) != hipSuccess) return HPADI_EHIP; \
    } while (0)

// Forward pass; train = keep pre-activations and all activations for the backward pass.
int forward(hpadi_net_s* N, const float* x, ImgShape s, float* out, bool train) {
    hipStream_t st = N->stream;
    const float* P = N->params;
    if (train) {
        HIPCHK(hpadi::launch_conv_in(x, s, P, N->pre0, N->a0, st));
        HIPCHK(hpadi::launch_conv32(N->a0, s, N->wf1, P + hpadi::kOffB1, nullptr, N->pre1, N->a1, 0, st));
        HIPCHK(hpadi::launch_conv32(N->a1, s, N->wf2, P + hpadi::kOffB2, nullptr, N->pre2, N->a2, 0, st));
        HIPCHK(hpadi::launch_conv_out(N->a2, s, P, out, st));
    } else {
        HIPCHK(hpadi::launch_conv_in(x, s, P, nullptr, N->a0, st));
        HIPCHK(hpadi::launch_conv32(N->a0, s, N->wf1, P + hpadi::kOffB1, nullptr, nullptr, N->a1, 0, st));
        HIPCHK(hpadi::launch_conv32(N->a1, s, N->wf2, P + hpadi::kOffB2, nullptr, nullptr, N->a0, 0, st));
        HIPCHK(hpadi::launch_conv_out(N->a0, s, P, out, st));
    }
    return HPADI_OK;
}

// Loss and gradients (into N->grads) of the batch held in N->x, zn, t, w; *loss on the host.
int loss_backward(hpadi_net_s* N, ImgShape s, double* loss) {
    hipStream_t st = N->stream;
    const float* P = N->params;
    int rc = forward(N, N->x, s, N->out, true);
    if (rc != HPADI_OK) return rc;
    if ((rc = ensure_nd(N, s.B)) != HPADI_OK) return rc;
    HIPCHK(hipMemsetAsync(N->num_den, 0, 2 * (size_t)s.B * sizeof(double), st));
    HIPCHK(hpadi::launch_zero_f32(N->grads, hpadi::kNetParams, st));
    HIPCHK(hpadi::launch_loss(N->out, N->zn, N->t, N->w, s, N->g, N->num_den, st));
    HIPCHK(hpadi::launch_conv_out_backward(N->a2, N->g, N->pre2, s, P, N->grads, N->ga, st));  // ga = dL/dpre2
    HIPCHK(hpadi::launch_conv32_wgrad(N->a1, N->ga, s, N->grads + hpadi::kOffW2, st));
    HIPCHK(hpadi::launch_bias_grad(N->ga, s, N->grads + hpadi::kOffB2, st));
    HIPCHK(hpadi::launch_conv32(N->ga, s, N->wb2, nullptr, N->pre1, nullptr, N->gb, 1, st));  // gb = dL/dpre1
    HIPCHK(hpadi::launch_conv32_wgrad(N->a0, N->gb, s, N->grads + hpadi::kOffW1, st));
    HIPCHK(hpadi::launch_bias_grad(N->gb, s, N->grads + hpadi::kOffB1, st));
    HIPCHK(hpadi::launch_conv32(N->gb, s, N->wb1, nullptr, N->pre0, nullptr, N->ga, 1, st));  // ga = dL/dpre0
    HIPCHK(hpadi::launch_conv_in_wgrad(N->x, N->ga, s, N->grads + hpadi::kOffW0, st));
    HIPCHK(hpadi::launch_bias_grad(N->ga, s, N->grads + hpadi::kOffB0, st));
    if (loss) {
        HIPCHK(hipMemcpyAsync(N->num_den_host, N->num_den, 2 * (size_t)s.B * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        double L = 0.0;
        for (int b = 0; b < s.B; ++b)
            L += N->num_den_host[2 * b + 1] > 0 ? N->num_den_host[2 * b] / N->num_den_host[2 * b + 1] : 0.0;
        *loss = L / s.B;
    }
    return HPADI_OK;
}

int upload_params(hpadi_net_s* N, const float* h) {
    HIPCHK(hipMemcpyAsync(N->params, h, hpadi::kNetParams * sizeof(float), hipMemcpyHostToDevice, N->stream));
    HIPCHK(hpadi::launch_pack_weights(N->params, N->wf1, N->wb1, N->wf2, N->wb2, N->stream));
    HIPCHK(hipStreamSynchronize(N->stream));
    return HPADI_OK;
}

}  // namespace

extern "C" {

int hpadi_net_num_params(void) { return hpadi::kNetParams; }

int hpadi_net_create(const float* params, unsigned long long seed, void* hip_stream, hpadi_net* out) {
    if (!out) return HPADI_EINVAL;
    *out = nullptr;
    hpadi_net_s* N = new (std::nothrow) hpadi_net_s();
    if (!N) return HPADI_ENOMEM;
    N->stream = (hipStream_t)hip_stream;
    const size_t P = hpadi::kNetParams, WW = 9 * hpadi::kNetC * hpadi::kNetC;
    if (dmalloc(&N->params, P) != hipSuccess || dmalloc(&N->grads, P) != hipSuccess || dmalloc(&N->m, P) != hipSuccess ||
        dmalloc(&N->v, P) != hipSuccess || dmalloc(&N->wf1, WW) != hipSuccess || dmalloc(&N->wb1, WW) != hipSuccess ||
        dmalloc(&N->wf2, WW) != hipSuccess || dmalloc(&N->wb2, WW) != hipSuccess) {
        delete N;
        return HPADI_ENOMEM;
    }
    std::vector<float> h(P, 0.0f);
    if (params) {
        std::memcpy(h.data(), params, P * sizeof(float));
    } else {
        // normal(0, sqrt(2 / fan_in)) by Box-Muller on the counter-based uniforms
        const int cin[4] = {hpadi::kNetCin, hpadi::kNetC, hpadi::kNetC, hpadi::kNetC};
        const int cout[4] = {hpadi::kNetC, hpadi::kNetC, hpadi::kNetC, 1};
        const int offw[4] = {hpadi::kOffW0, hpadi::kOffW1, hpadi::kOffW2, hpadi::kOffW3};
        uint64_t ctr = 0;
        for (int l = 0; l < 4; ++l) {
            const int n = 9 * cin[l] * cout[l];
            const double sd = std::sqrt(2.0 / (9.0 * cin[l])) * (l == 3 ? 0.1 : 1.0);
            for (int i = 0; i < n; ++i) {
                const double u1 = std::max(uniform01(seed, ctr++), 1e-300), u2 = uniform01(seed, ctr++);
                h[offw[l] + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2));
            }
        }
    }
    if (hipMemsetAsync(N->m, 0, P * sizeof(float), N->stream) != hipSuccess ||
        hipMemsetAsync(N->v, 0, P * sizeof(float), N->stream) != hipSuccess || upload_params(N, h.data()) != HPADI_OK) {
        delete N;
        return HPADI_EHIP;
    }
    *out = N;
    return HPADI_OK;
}

int hpadi_net_get_params(hpadi_net N, float* params) {
    if (!N || !params) return HPADI_EINVAL;
    if (hipMemcpyAsync(params, N->params, hpadi::kNetParams * sizeof(float), hipMemcpyDeviceToHost, N->stream) !=
            hipSuccess ||
        hipStreamSynchronize(N->stream) != hipSuccess)
        return HPADI_EHIP;
    return HPADI_OK;
}

int hpadi_net_set_params(hpadi_net N, const float* params) {
    if (!N || !params) return HPADI_EINVAL;
    return upload_params(N, params);
}

int hpadi_net_set_period(hpadi_net N, int period) {
    if (!N || period < 1) return HPADI_EINVAL;
    N->period = period;
    return HPADI_OK;
}

int hpadi_net_set_damping(hpadi_net N, double omega) {
    if (!N || !(omega >= 0.0) || !std::isfinite(omega)) return HPADI_EINVAL;
    N->damping = omega;
    return HPADI_OK;
}

int hpadi_net_forward(hpadi_net N, const float* x, int B, int H, int W, float* out) {
    if (!N || !x || !out || B < 1 || H < 1 || W < 1) return HPADI_EINVAL;
    int rc = ensure_ws(N, (size_t)B * H * W, false);
    if (rc != HPADI_OK) return rc;
    return forward(N, x, ImgShape{B, H, W}, out, false);
}

int hpadi_net_loss_grad(hpadi_net N, const float* x, const float* zn, const float* t, const float* w, int B, int H,
                        int W, double* loss, float* grad) {
    if (!N || !x || !zn || !t || !w || B < 1 || H < 1 || W < 16 || W % 16 != 0) return HPADI_EINVAL;
    const size_t np = (size_t)B * H * W;
    int rc = ensure_ws(N, np, true);
    if (rc != HPADI_OK) return rc;
    hipStream_t st = N->stream;
    if (hipMemcpyAsync(N->x, x, 3 * np * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(N->zn, zn, np * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(N->t, t, np * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(N->w, w, np * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return HPADI_EHIP;
    if ((rc = loss_backward(N, ImgShape{B, H, W}, loss)) != HPADI_OK) return rc;
    if (grad) {
        if (hipMemcpyAsync(grad, N->grads, hpadi::kNetParams * sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return HPADI_EHIP;
    }
    return HPADI_OK;
}

int hpadi_net_train(hpadi_net N, const float* X, const float* ZN, const float* T, const float* Wt, int npairs, int c,
                    int batch, int steps, double lr, unsigned long long seed, float* loss_hist) {
    if (!N || !X || !ZN || !T || !Wt || npairs < 1 || c < 16 || c % 16 != 0 || batch < 1 || steps < 0 || !(lr > 0))
        return HPADI_EINVAL;
    const size_t np = (size_t)batch * c * c;
    int rc = ensure_ws(N, np, true);
    if (rc != HPADI_OK) return rc;
    hipStream_t st = N->stream;
    if (batch > N->idx_cap) {
        (void)hipFree(N->idx);
        N->idx = nullptr;
        if (dmalloc(&N->idx, (size_t)batch) != hipSuccess) return HPADI_ENOMEM;
        N->idx_cap = batch;
    }
    std::vector<int> idx(batch);
    for (int it = 0; it < steps; ++it) {
        for (int b = 0; b < batch; ++b)
            idx[b] = std::min(npairs - 1, (int)(uniform01(seed, (uint64_t)it * batch + b) * npairs));
        if (hipMemcpyAsync(N->idx, idx.data(), batch * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
            hpadi::launch_gather_batch(X, ZN, T, Wt, c, N->idx, batch, N->x, N->zn, N->t, N->w, st) != hipSuccess)
            return HPADI_EHIP;
        double L = 0.0;
        if ((rc = loss_backward(N, ImgShape{batch, c, c}, loss_hist ? &L : nullptr)) != HPADI_OK) return rc;
        if (loss_hist) loss_hist[it] = (float)L;
        ++N->step;
        if (hpadi::launch_adam(N->params, N->grads, N->m, N->v, hpadi::kNetParams, (float)lr, 0.9f, 0.999f, 1e-8f,
                               N->step, st) != hipSuccess ||
            hpadi::launch_pack_weights(N->params, N->wf1, N->wb1, N->wf2, N->wb2, st) != hipSuccess)
            return HPADI_EHIP;
    }
    return hipStreamSynchronize(st) == hipSuccess ? HPADI_OK : HPADI_EHIP;
}

void hpadi_net_destroy(hpadi_net N) { delete N; }

int hpadi_net_pairs(hpadi_varcoef V, hpadi_plan precond, const double* b, int ldb, const double* xstar, int ldxs,
                    double tol, int max_iters, int c, int crops_per_iter, unsigned long long seed, float* X, float* ZN,
                    float* T, float* Wt, int cap, int* count) {
    if (!V || !b || !xstar || !X || !ZN || !T || !Wt || !count || cap < 1 || crops_per_iter < 1 || c < 1 ||
        max_iters < 1 || ldxs < V->Ny)
        return HPADI_EINVAL;
    *count = 0;
    int rc = hpadi_host::ensure_slots(V);
    if (rc != HPADI_OK) return rc;
    if (c > V->H || c > V->W) return HPADI_EINVAL;
    hipStream_t st = V->stream;
    const long n = (long)V->Nx * V->Ny;
    // x* in compact layout
    double* xs = nullptr;
    int* pos = nullptr;
    if (dmalloc(&xs, (size_t)n) != hipSuccess || dmalloc(&pos, 2 * (size_t)crops_per_iter) != hipSuccess) {
        (void)hipFree(xs);
        return HPADI_ENOMEM;
    }
    if (hpadi::launch_copy2d(xstar, ldxs, xs, V->Ny, V->Nx, V->Ny, st) != hipSuccess) rc = HPADI_EHIP;
    hpadi::SlotMap mp{V->H, V->W, V->sx, V->sy, V->loga};
    std::vector<int> hp(2 * crops_per_iter);
    const size_t cc = (size_t)c * c;
    auto observe = [&](int k, const double* r, const double* z, const double* x) -> int {
        if (*count >= cap) return HPADI_OK;
        double nz = 0.0;
        {
            hpadi::MultiB mb{};
            mb.nb = 1;
            mb.b[0] = z;
            if (hpadi::launch_multidot(z, mb, n, V->part, V->dots, st) != hipSuccess ||
                hipMemcpyAsync(V->dots_host, V->dots, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return HPADI_EHIP;
            nz = V->dots_host[0];
        }
        const double sz = std::sqrt(std::max(nz, 1e-300) / n);
        if (hpadi::launch_pack_image(mp, z, V->Ny, 1.0 / sz, V->img, st) != hipSuccess ||
            hpadi::launch_target_image(mp, xs, x, z, V->Ny, 1.0 / sz, V->wx, V->wy, V->img_zn, V->img_t, V->img_w,
                                       st) != hipSuccess)
            return HPADI_EHIP;
        const int ncrop = std::min(crops_per_iter, cap - *count);
        for (int i = 0; i < ncrop; ++i) {
            const uint64_t ctr = ((uint64_t)k * crops_per_iter + i) * 2;
            hp[2 * i] = std::min(V->H - c, (int)(uniform01(seed, ctr) * (V->H - c + 1)));
            hp[2 * i + 1] = std::min(V->W - c, (int)(uniform01(seed, ctr + 1) * (V->W - c + 1)));
        }
        const size_t off = (size_t)(*count) * cc;
        if (hipMemcpyAsync(pos, hp.data(), 2 * ncrop * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
            hpadi::launch_crop(V->img, V->img_zn, V->img_t, V->img_w, V->H, V->W, c, pos, ncrop, X + 3 * off,
                               ZN + off, T + off, Wt + off, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return HPADI_EHIP;
        *count += ncrop;
        return HPADI_OK;
    };
    if (rc == HPADI_OK) {
        double* xout = nullptr;
        if (dmalloc(&xout, (size_t)n) != hipSuccess) {
            rc = HPADI_ENOMEM;
        } else {
            hpadi_krylov_stats kst{};
            rc = hpadi_host::fcg_core(V, precond, nullptr, b, ldb, xout, V->Ny, tol, max_iters, 0, nullptr, 0, &kst,
                                      observe);
            if (rc == HPADI_ENOCONV) rc = HPADI_OK;
            (void)hipFree(xout);
        }
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(xs);
    (void)hipFree(pos);
    return rc;
}

}  // extern "C"

namespace hpadi_host {

int net_correct(hpadi_net N, hpadi_varcoef_s* V, const double* r, double* z, int iter, bool* applied) {
    *applied = false;
    if (iter % N->period != 0) return HPADI_OK;  // corrections at iterations 0, period, 2 period, ...
    hipStream_t st = V->stream;
    const long n = (long)V->Nx * V->Ny;
    int rc = ensure_slots(V);
    if (rc != HPADI_OK) return rc;
    if ((rc = ensure_ws(N, (size_t)V->H * V->W, N->train_ws)) != HPADI_OK) return rc;
    auto fetch = [&](int cnt) -> int {
        if (hipMemcpyAsync(V->dots_host, V->dots, cnt * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return HPADI_EHIP;
        return HPADI_OK;
    };
    hpadi::MultiB mb{};
    mb.nb = 1;
    mb.b[0] = z;
    if (hpadi::launch_multidot(z, mb, n, V->part, V->dots, st) != hipSuccess) return HPADI_EHIP;
    hpadi::SlotMap mp{V->H, V->W, V->sx, V->sy, V->loga};
    if (N->damping > 0.0) {
        // z <- z + damping c: the scale of z stays on the device, no host round trip
        if (hpadi::launch_pack_image(mp, z, V->Ny, 0.0, V->img, st, V->dots, 1.0 / (double)n) != hipSuccess)
            return HPADI_EHIP;
        if (N->stream != st && hipStreamSynchronize(st) != hipSuccess) return HPADI_EHIP;
        if ((rc = forward(N, V->img, ImgShape{1, V->H, V->W}, V->img_out, false)) != HPADI_OK) return rc;
        if (N->stream != st && hipStreamSynchronize(N->stream) != hipSuccess) return HPADI_EHIP;
        if (hpadi::launch_unpack_add(mp, V->img_out, N->damping, z, V->Ny, st, V->dots, 1.0 / (double)n) !=
            hipSuccess)
            return HPADI_EHIP;
        *applied = true;
        return HPADI_OK;
    }
    if ((rc = fetch(1)) != HPADI_OK) return rc;
    const double zz = V->dots_host[0];
    if (!(zz > 0.0)) return HPADI_OK;
    const double sz = std::sqrt(zz / n);
    double* c = V->zs;
    if (hpadi::launch_pack_image(mp, z, V->Ny, 1.0 / sz, V->img, st) != hipSuccess) return HPADI_EHIP;
    if (N->stream != st && hipStreamSynchronize(st) != hipSuccess) return HPADI_EHIP;
    if ((rc = forward(N, V->img, ImgShape{1, V->H, V->W}, V->img_out, false)) != HPADI_OK) return rc;
    if (N->stream != st && hipStreamSynchronize(N->stream) != hipSuccess) return HPADI_EHIP;
    if (hipMemsetAsync(c, 0, n * sizeof(double), st) != hipSuccess ||
        hpadi::launch_unpack_add(mp, V->img_out, sz, c, V->Ny, st) != hipSuccess ||
        hpadi::launch_vc_apply(V->dev, z, V->Ny, V->Az, V->Ny, st) != hipSuccess ||
        hpadi::launch_vc_apply(V->dev, c, V->Ny, V->Ac, V->Ny, st) != hipSuccess)
        return HPADI_EHIP;
    // z.Az, z.Ac, z.r, c.Ac, c.r
    mb.nb = 3;
    mb.b[0] = V->Az;
    mb.b[1] = V->Ac;
    mb.b[2] = r;
    if (hpadi::launch_multidot(z, mb, n, V->part, V->dots, st) != hipSuccess) return HPADI_EHIP;
    mb.nb = 2;
    mb.b[0] = V->Ac;
    mb.b[1] = r;
    if (hpadi::launch_multidot(c, mb, n, V->part, V->dots + 3, st) != hipSuccess) return HPADI_EHIP;
    if ((rc = fetch(5)) != HPADI_OK) return rc;
    const double zAz = V->dots_host[0], zAc = V->dots_host[1], zr = V->dots_host[2];
    const double cAc = V->dots_host[3], cr = V->dots_host[4];
    // minimise [a b] G [a b]^T - 2 [a b] g with G = [[zAz, zAc], [zAc, cAc]], g = [zr, cr]
    const double det = zAz * cAc - zAc * zAc;
    if (!(zAz > 0.0) || !(cAc > 0.0) || !(det > 1e-12 * zAz * cAc) || !std::isfinite(det)) return HPADI_OK;
    const double alpha = (cAc * zr - zAc * cr) / det, beta = (zAz * cr - zAc * zr) / det;
    if (!(alpha > 0.0) || !std::isfinite(beta)) return HPADI_OK;
    hpadi::MultiB xs{};
    hpadi::Coefs cc{};
    xs.nb = 1;
    xs.b[0] = c;
    cc.c[0] = beta / alpha;
    if (hpadi::launch_axpys(z, xs, cc, n, st) != hipSuccess) return HPADI_EHIP;
    *applied = true;
    return HPADI_OK;
}

}  // namespace hpadi_host
