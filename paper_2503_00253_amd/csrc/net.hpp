// Internal view of the warm-start network handle.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace infoesrf {

// Trunk 1 -> H -> H -> H -> D channels, kernel K (odd, <= 15), "same" zero padding, GELU after the
// first three layers; per member it maps bh = sqrt(m) b / ||b|| to Y (D x m), and the head gives the
// system at shift s the output sum_d c^(d+1) Y[d], c = 1 / (1 + s).  FP32 parameters, Adam moments
// and a gradient buffer live on the device (allocated when the handle is created or loaded, never
// on the update path).
constexpr int kNetD = 4;  // output channels of the trunk (terms of the shift head)
struct Net {
  int H = 64;
  int K = 9;
  int D = kNetD;
  int64_t count = 0;         // FP32 parameters
  float* params = nullptr;   // device, layout W1 b1 W2 b2 W3 b3 W4 b4 (W row-major Cout x Cin x K)
  float* adam_m = nullptr;   // device
  float* adam_v = nullptr;   // device
  float* grads = nullptr;    // device
  int64_t step = 0;          // Adam steps taken
};

int64_t net_param_count(int H, int K, int D);
// Offsets (in floats) of layer l's weights and bias, and its channel counts.
void net_layer(const Net& n, int l, int64_t* w_off, int64_t* b_off, int* cin, int* cout);
// Bytes of workspace for a batch of B members (Q shifts each when training) of length m.
size_t net_ws_bytes(const Net& n, int64_t B, int64_t Q, int64_t m, bool training);
// Trunk output Y (B x D x m) of member inputs X (B x m) in FP32; ws as sized by net_ws_bytes(.., false).
int net_forward(const Net& n, const float* X, int64_t B, int64_t m, float* Y, void* ws, size_t ws_bytes,
                hipStream_t st);
// The same with BF16 weights and activations on MFMA, FP32 accumulation (H <= 64, H % 8 == 0);
// the inference workspace covers both.
int net_forward_bf16(const Net& n, const float* X, int64_t B, int64_t m, float* Y, void* ws, size_t ws_bytes,
                     hipStream_t st);

hipError_t launch_conv_fwd(const float* in, int Cin, const float* W, const float* bias, int Cout, int K, int m,
                           int64_t B, float* pre, float* act, int gelu, hipStream_t st);
// BF16 inference: packed weights (round_up(Cout, 16) rows of bf16_kd(Cin, K) entries), and the
// MFMA correlation (inputs (B, Cin, m) FP32 or (B, m, Cin) BF16 with Cin a multiple of 8; outputs
// (B, m) FP32 when Cout = 1 or (B, m, Cout) BF16).  Cin, Cout <= 64.
int bf16_cp(int Cin);
int bf16_kd(int Cin, int K);
int bf16_opad(int Cout);
hipError_t launch_pack_weights_bf16(const float* W, int Cout, int Cin, int K, __hip_bfloat16* out, hipStream_t st);
hipError_t launch_conv_bf16(const void* in, bool in_f32, int Cin, const __hip_bfloat16* Wp, const float* bias, int Cout,
                            int K, int m, int64_t B, void* out, bool out_f32, int gelu, hipStream_t st);
hipError_t launch_conv_wgrad(const float* a, int Cin, const float* g, int Cout, int K, int m, int64_t B, float* gW,
                             float* gb, hipStream_t st);
hipError_t launch_flip_transpose(const float* W, int Cout, int Cin, int K, float* Wt, hipStream_t st);
hipError_t launch_gelu_bwd(float* g, const float* z, int64_t n, hipStream_t st);
// The shift head's loss and gradient for B members x Q shifts (cq: Q values c = 1 / (1 + s)):
// per-system relative L2 errors against T (B x Q x m) into per (B Q), their mean into *mean,
// the gradient factors into scale (B Q) and dL/dY (B x D x m) into gY.
hipError_t launch_head_loss_grad(const float* Y, int D, const float* cq, int Q, const float* T, int m, int64_t B,
                                 float* per, float* scale, float* mean, float* gY, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* mo, float* ve, int64_t n, float lr, int64_t t,
                       hipStream_t st);

}  // namespace infoesrf
