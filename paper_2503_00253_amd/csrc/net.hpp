// Internal view of the warm-start network handle.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace infoesrf {

// 3 -> H -> H -> H -> 1 channels, kernel K (odd, <= 15), "same" zero padding, GELU after the
// first three layers.  FP32 parameters, Adam moments and a gradient buffer live on the device
// (allocated when the handle is created or loaded, never on the update path).
struct Net {
  int H = 64;
  int K = 9;
  int64_t count = 0;         // FP32 parameters
  float* params = nullptr;   // device, layout W1 b1 W2 b2 W3 b3 W4 b4 (W row-major Cout x Cin x K)
  float* adam_m = nullptr;   // device
  float* adam_v = nullptr;   // device
  float* grads = nullptr;    // device
  int64_t step = 0;          // Adam steps taken
};

int64_t net_param_count(int H, int K);
// Offsets (in floats) of layer l's weights and bias, and its channel counts.
void net_layer(const Net& n, int l, int64_t* w_off, int64_t* b_off, int* cin, int* cout);
// Bytes of workspace for a batch of B samples of length m (training keeps every activation).
size_t net_ws_bytes(const Net& n, int64_t B, int64_t m, bool training);
// Network output Y (B x m) of inputs X (B x 3 x m) in FP32; ws as sized by net_ws_bytes(.., false).
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
hipError_t launch_rel_l2(const float* y, const float* t, int m, int64_t B, float* gy, float* per, float* mean,
                         hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* mo, float* ve, int64_t n, float lr, int64_t t,
                       hipStream_t st);

}  // namespace infoesrf
