// Declarations shared by the learned-correction kernels (net.hip) and their host
// code (net.cpp).  The network: 3x3 convolutions with zero padding, channels
// 3 -> 32 -> 32 -> 32 -> 1, tanh-form GELU after the hidden layers.  Images are
// NHWC; hidden activations are BF16, pre-activations and gradients of the
// parameters FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstddef>
#include <cstdint>

namespace hpadi {

constexpr int kNetC = 32;      // hidden channels
constexpr int kNetCin = 3;     // input channels: z/s_z, (z/s_z)/a, log a
// parameter vector (FP32): W0[3][3][3][32] b0[32] W1[3][3][32][32] b1[32] W2[...] b2[32] W3[3][3][32][1] b3[1]
constexpr int kOffW0 = 0;
constexpr int kOffB0 = kOffW0 + 9 * kNetCin * kNetC;
constexpr int kOffW1 = kOffB0 + kNetC;
constexpr int kOffB1 = kOffW1 + 9 * kNetC * kNetC;
constexpr int kOffW2 = kOffB1 + kNetC;
constexpr int kOffB2 = kOffW2 + 9 * kNetC * kNetC;
constexpr int kOffW3 = kOffB2 + kNetC;
constexpr int kOffB3 = kOffW3 + 9 * kNetC;
constexpr int kNetParams = kOffB3 + 1;

typedef uint16_t bf16_t;  // storage type of BF16 arrays

struct ImgShape { int B, H, W; };

// first layer (VALU): pre = conv(x, W0) + b0 (FP32, optional), act = bf16(gelu(pre))
hipError_t launch_conv_in(const float* x, ImgShape s, const float* params, float* pre, bf16_t* act, hipStream_t st);
// 32 -> 32 layer on MFMA.  wt: [9][32 n][32 k] BF16 (n: output channel of this conv,
// k: input channel).  mode 0: pre = conv + bias (FP32, optional), act = bf16(gelu(pre));
// mode 1 (data gradient): act = bf16(conv * gelu'(pre_prev)).
hipError_t launch_conv32(const bf16_t* in, ImgShape s, const bf16_t* wt, const float* bias, const float* pre_prev,
                         float* pre, bf16_t* act, int mode, hipStream_t st);
// last layer (VALU): out = conv(a, W3) + b3 (FP32)
hipError_t launch_conv_out(const bf16_t* a, ImgShape s, const float* params, float* out, hipStream_t st);
// loss of a batch: den[b] = sum w t^2, num[b] = sum w (zn + o - t)^2; g = 2/B w (zn + o - t) / den[b]
hipError_t launch_loss(const float* o, const float* zn, const float* t, const float* w, ImgShape s, float* g,
                       double* num_den, hipStream_t st);
// backward of the last layer: grads[W3, b3] += ..., gact = bf16(W3^T-conv(g) * gelu'(pre2))
hipError_t launch_conv_out_backward(const bf16_t* a, const float* g, const float* pre2, ImgShape s,
                                    const float* params, float* grads, bf16_t* gact, hipStream_t st);
// weight gradient of a 32 -> 32 layer on MFMA: dW[tap][ci][co] += sum_p a[p + off][ci] g[p][co]
hipError_t launch_conv32_wgrad(const bf16_t* a, const bf16_t* g, ImgShape s, float* dW, hipStream_t st);
// weight gradient of the first layer (FP32 input)
hipError_t launch_conv_in_wgrad(const float* x, const bf16_t* g, ImgShape s, float* dW0, hipStream_t st);
// bias gradient: db[c] += sum_p g[p][c] (32 channels)
hipError_t launch_bias_grad(const bf16_t* g, ImgShape s, float* db, hipStream_t st);
// Adam step on the parameters, then the BF16 layouts of the two hidden layers
// (forward [tap][co][ci], data gradient [tap][ci][co] with the tap flipped).
hipError_t launch_adam(float* params, const float* grads, float* m, float* v, int n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t st);
hipError_t launch_pack_weights(const float* params, bf16_t* wf1, bf16_t* wb1, bf16_t* wf2, bf16_t* wb2,
                               hipStream_t st);
hipError_t launch_zero_f32(float* p, size_t n, hipStream_t st);

// Coefficient <-> image maps for the Krylov correction (one image, H = (n_x p_x + 1),
// W = (n_y p_y + 1)); slot2g*[s] = global index of slot s or -1.
struct SlotMap {
    int H, W;
    const int* sx;   // [H]
    const int* sy;   // [W]
    const float* loga;  // [H W] log a at the slots
};
// x[p] = [z/s_z, (z/s_z) exp(-log a), log a] at every slot p, with 1/s_z = inv_sz, or, when zz
// is given, 1/s_z = 1/sqrt(zz[0] inv_n) from the device sum of squares zz[0] of z (no host
// round trip).
hipError_t launch_pack_image(const SlotMap& m, const double* z, long ld, double inv_sz, float* x, hipStream_t st,
                             const double* zz = nullptr, double inv_n = 0.0);
// z[slot] += sz o[p]; when zz is given the factor is sz sqrt(zz[0] inv_n).
hipError_t launch_unpack_add(const SlotMap& m, const float* o, double sz, double* z, long ld, hipStream_t st,
                             const double* zz = nullptr, double inv_n = 0.0);
// training pairs: crops (y0, x0) of size c from full images (H x W): inputs (3 ch), zn, t, w
hipError_t launch_crop(const float* x, const float* zn, const float* t, const float* w, int H, int W, int c,
                       const int* pos /* [n][2] */, int n, float* cx, float* czn, float* ct, float* cw, hipStream_t st);
// target and weight images: t = (xs - x) / s_z at the slots, zn = z / s_z and the loss
// weight w = a (k_x m_y + m_x k_y), the diagonal of the energy form at the slot
// (wx = [m_x | k_x], wy = [m_y | k_y]: mass and stiffness diagonals of the slot functions)
hipError_t launch_target_image(const SlotMap& m, const double* xs, const double* x, const double* z, long ld,
                               double inv_sz, const float* wx, const float* wy, float* zn, float* t, float* w,
                               hipStream_t st);
// gather batch items idx[0..B) of crops (c x c) into contiguous arrays
hipError_t launch_gather_batch(const float* X, const float* ZN, const float* T, const float* Wt, int c,
                               const int* idx, int B, float* x, float* zn, float* t, float* w, hipStream_t st);

}  // namespace hpadi
