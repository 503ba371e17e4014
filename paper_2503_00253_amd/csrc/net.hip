// Warm-start network handle: creation, file I/O, inference and training steps.
//
// File format (little endian):
//   8 bytes  magic "IENET002"
//   5 int32  layers (4), input channels (1), hidden channels H, kernel width K, output channels D
//   float32  parameters in order W1 (H x 1 x K), b1 (H), W2 (H x H x K), b2 (H),
//            W3 (H x H x K), b3 (H), W4 (D x H x K), b4 (D)
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.hpp"
#include "net.hpp"

namespace infoesrf {

int64_t net_param_count(int H, int K, int D) {
  return (int64_t)H * 1 * K + H + 2 * ((int64_t)H * H * K + H) + (int64_t)D * H * K + D;
}

void net_layer(const Net& n, int l, int64_t* w_off, int64_t* b_off, int* cin, int* cout) {
  const int ci[4] = {1, n.H, n.H, n.H};
  const int co[4] = {n.H, n.H, n.H, n.D};
  int64_t off = 0;
  for (int j = 0; j < l; ++j) off += (int64_t)co[j] * ci[j] * n.K + co[j];
  *w_off = off;
  *b_off = off + (int64_t)co[l] * ci[l] * n.K;
  *cin = ci[l];
  *cout = co[l];
}

namespace {

// Training workspace (floats): z1 a1 z2 a2 z3 a3 (B H m each), the trunk output y and its gradient
// gy (B D m), per-system errors and gradient factors (B Q each), loss (1), two gradient buffers
// (B H m) and the flipped weights (H H K).  Inference: two (B H m) buffers.
struct NetWs {
  float *z[3], *a[3], *y, *gy, *per, *scale, *loss, *g0, *g1, *wt;
  float *p0, *p1;                // inference ping-pong (FP32)
  __hip_bfloat16 *q0, *q1;       // inference ping-pong (BF16, position-major)
  __hip_bfloat16* wpk[4];        // packed BF16 weights of the four layers
};

int64_t al(int64_t n) { return (n + 63) / 64 * 64; }

NetWs carve(const Net& n, int64_t B, int64_t Q, int64_t m, bool training, void* ws, size_t* bytes) {
  NetWs w{};
  float* base = static_cast<float*>(ws);
  int64_t off = 0;
  auto take = [&](int64_t cnt) {
    float* p = base ? base + off : nullptr;
    off += al(cnt);
    return p;
  };
  const int64_t act = B * n.H * m;
  if (training) {
    for (int l = 0; l < 3; ++l) {
      w.z[l] = take(act);
      w.a[l] = take(act);
    }
    w.y = take(B * n.D * m);
    w.gy = take(B * n.D * m);
    w.per = take(B * Q);
    w.scale = take(B * Q);
    w.loss = take(1);
    w.g0 = take(act);
    w.g1 = take(act);
    w.wt = take((int64_t)n.H * n.H * n.K);
  } else {
    w.p0 = take(act);
    w.p1 = take(act);
    const int64_t actb = B * (int64_t)bf16_cp(n.H) * m;  // BF16 elements
    w.q0 = reinterpret_cast<__hip_bfloat16*>(take((actb + 1) / 2));
    w.q1 = reinterpret_cast<__hip_bfloat16*>(take((actb + 1) / 2));
    for (int l = 0; l < 4; ++l) {
      int64_t wo, bo;
      int ci, co;
      net_layer(n, l, &wo, &bo, &ci, &co);
      const int64_t cnt = (int64_t)bf16_opad(co) * bf16_kd(ci, n.K);
      w.wpk[l] = reinterpret_cast<__hip_bfloat16*>(take((cnt + 1) / 2));
    }
  }
  *bytes = (size_t)off * sizeof(float) + 256;
  return w;
}

int check_net_io(const Net* n, int64_t B, int64_t m) {
  IE_CHECK(n && n->params, INFOESRF_ERR_INVALID_ARG, "network handle is NULL");
  IE_CHECK(B >= 1 && B <= 65535, INFOESRF_ERR_INVALID_ARG, "batch B must be in [1, 65535]");
  IE_CHECK(m >= 1 && m <= (1 << 24), INFOESRF_ERR_INVALID_ARG, "length m out of range");
  return 0;
}

int check_shifts(int64_t B, int64_t Q) {
  IE_CHECK(Q >= 1 && Q <= 64 && B * Q <= (int64_t)1 << 31, INFOESRF_ERR_INVALID_ARG, "shifts Q must be in [1, 64]");
  return 0;
}

// forward through all layers, keeping z and a (training) or ping-ponging (inference)
int forward_layers(const Net& n, const float* X, int64_t B, int64_t m, const NetWs& w, bool training, float* Y,
                   hipStream_t st) {
  const float* in = X;
  for (int l = 0; l < 4; ++l) {
    int64_t wo, bo;
    int ci, co;
    net_layer(n, l, &wo, &bo, &ci, &co);
    const bool last = (l == 3);
    float* pre = training && !last ? w.z[l] : nullptr;
    float* act = last ? Y : (training ? w.a[l] : (l % 2 == 0 ? w.p0 : w.p1));
    IE_HIP(launch_conv_fwd(in, ci, n.params + wo, n.params + bo, co, n.K, (int)m, B, pre, act, last ? 0 : 1, st));
    in = act;
  }
  return 0;
}

// BF16 inference: weights packed on every call (they may have been trained since), activations in
// BF16 between layers, the last layer writes FP32
int forward_layers_bf16(const Net& n, const float* X, int64_t B, int64_t m, const NetWs& w, float* Y,
                        hipStream_t st) {
  const void* in = X;
  for (int l = 0; l < 4; ++l) {
    int64_t wo, bo;
    int ci, co;
    net_layer(n, l, &wo, &bo, &ci, &co);
    IE_HIP(launch_pack_weights_bf16(n.params + wo, co, ci, n.K, w.wpk[l], st));
    const bool last = (l == 3);
    void* out = last ? static_cast<void*>(Y) : static_cast<void*>(l % 2 == 0 ? w.q0 : w.q1);
    IE_HIP(launch_conv_bf16(in, l == 0, ci, w.wpk[l], n.params + bo, co, n.K, (int)m, B, out, last, last ? 0 : 1,
                            st));
    in = out;
  }
  return 0;
}

// gradients of the mean relative L2 loss of the B x Q systems (shift factors cq) into grads (and
// the loss into *loss_dev): the trunk forward, the head's loss and gradient, the trunk backward
int gradients(const Net& n, const float* X, const float* cq, const float* T, int64_t B, int64_t Q, int64_t m,
              const NetWs& w, float* grads, float* loss_dev, hipStream_t st) {
  IE_TRY(forward_layers(n, X, B, m, w, true, w.y, st));
  IE_HIP(launch_head_loss_grad(w.y, n.D, cq, (int)Q, T, (int)m, B, w.per, w.scale, loss_dev ? loss_dev : w.loss,
                               w.gy, st));
  const float* g = w.gy;  // gradient w.r.t. layer l's output
  for (int l = 3; l >= 0; --l) {
    int64_t wo, bo;
    int ci, co;
    net_layer(n, l, &wo, &bo, &ci, &co);
    const float* a_in = (l == 0) ? X : w.a[l - 1];
    IE_HIP(launch_conv_wgrad(a_in, ci, g, co, n.K, (int)m, B, grads + wo, grads + bo, st));
    if (l == 0) break;
    // gradient w.r.t. the input activation a_{l-1}, then through GELU to z_{l-1}
    float* gin = (l % 2 == 1) ? w.g0 : w.g1;
    IE_HIP(launch_flip_transpose(n.params + wo, co, ci, n.K, w.wt, st));
    IE_HIP(launch_conv_fwd(g, co, w.wt, nullptr, ci, n.K, (int)m, B, nullptr, gin, 0, st));
    IE_HIP(launch_gelu_bwd(gin, w.z[l - 1], B * (int64_t)ci * m, st));
    g = gin;
  }
  return 0;
}

// splitmix64: a counter-based generator for the initial weights
uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

int alloc_state(Net* h) {
  const size_t b = sizeof(float) * (size_t)h->count;
  IE_HIP(hipMalloc(&h->params, b));
  IE_HIP(hipMalloc(&h->adam_m, b));
  IE_HIP(hipMalloc(&h->adam_v, b));
  IE_HIP(hipMalloc(&h->grads, b));
  IE_HIP(hipMemset(h->adam_m, 0, b));
  IE_HIP(hipMemset(h->adam_v, 0, b));
  IE_HIP(hipMemset(h->grads, 0, b));
  return 0;
}

void free_state(Net* h) {
  for (float* p : {h->params, h->adam_m, h->adam_v, h->grads})
    if (p) (void)hipFree(p);
  h->params = h->adam_m = h->adam_v = h->grads = nullptr;
}

}  // namespace

size_t net_ws_bytes(const Net& n, int64_t B, int64_t Q, int64_t m, bool training) {
  size_t b = 0;
  (void)carve(n, B, Q, m, training, nullptr, &b);
  return b;
}

int net_forward(const Net& n, const float* X, int64_t B, int64_t m, float* Y, void* ws, size_t ws_bytes,
                hipStream_t st) {
  size_t need = 0;
  const NetWs w = carve(n, B, 1, m, false, ws, &need);
  IE_CHECK(ws && ws_bytes >= need, INFOESRF_ERR_WORKSPACE, "network workspace too small");
  return forward_layers(n, X, B, m, w, false, Y, st);
}

int net_forward_bf16(const Net& n, const float* X, int64_t B, int64_t m, float* Y, void* ws, size_t ws_bytes,
                     hipStream_t st) {
  size_t need = 0;
  const NetWs w = carve(n, B, 1, m, false, ws, &need);
  IE_CHECK(ws && ws_bytes >= need, INFOESRF_ERR_WORKSPACE, "network workspace too small");
  IE_CHECK(n.H <= 64 && n.H % 8 == 0, INFOESRF_ERR_INVALID_ARG, "BF16 inference needs H <= 64, H % 8 == 0");
  return forward_layers_bf16(n, X, B, m, w, Y, st);
}

}  // namespace infoesrf

using namespace infoesrf;

extern "C" int infoesrf_net_create(int32_t hidden, int32_t kernel, uint64_t seed, void** net) {
  clear_error();
  IE_CHECK(net != nullptr, INFOESRF_ERR_INVALID_ARG, "net must be non-NULL");
  *net = nullptr;
  IE_CHECK(hidden >= 1 && hidden <= 256, INFOESRF_ERR_INVALID_ARG, "hidden channels must be in [1, 256]");
  IE_CHECK(kernel >= 1 && kernel <= 15 && kernel % 2 == 1, INFOESRF_ERR_INVALID_ARG,
           "kernel width must be odd and <= 15");
  Net* h = new Net();
  h->H = hidden;
  h->K = kernel;
  h->D = kNetD;
  h->count = net_param_count(hidden, kernel, h->D);
  std::vector<float> host((size_t)h->count, 0.f);
  // uniform(-a, a) weights with a = sqrt(6 / (Cin K)), zero biases; the output layer starts at
  // zero, so an untrained network predicts the zero start
  uint64_t ctr = seed * 0x100000001B3ULL;
  for (int l = 0; l < 3; ++l) {
    int64_t wo, bo;
    int ci, co;
    net_layer(*h, l, &wo, &bo, &ci, &co);
    const double a = std::sqrt(6.0 / ((double)ci * kernel));
    for (int64_t i = 0; i < (int64_t)co * ci * kernel; ++i) {
      const double u = (double)(splitmix64(ctr++) >> 11) * (1.0 / 9007199254740992.0);
      host[(size_t)(wo + i)] = (float)((2.0 * u - 1.0) * a);
    }
  }
  if (alloc_state(h) < 0 ||
      hipMemcpy(h->params, host.data(), sizeof(float) * host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    free_state(h);
    delete h;
    set_error("device allocation or copy failed for the network");
    return INFOESRF_ERR_HIP;
  }
  *net = h;
  return INFOESRF_OK;
}

extern "C" int infoesrf_net_load(const char* path, void** net) {
  clear_error();
  IE_CHECK(path && net, INFOESRF_ERR_INVALID_ARG, "path and net must be non-NULL");
  *net = nullptr;
  FILE* f = std::fopen(path, "rb");
  IE_CHECK(f != nullptr, INFOESRF_ERR_INVALID_ARG, std::string("cannot open ") + path);
  char magic[8];
  int32_t hdr[5];
  const bool ok_hdr = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "IENET002", 8) == 0 &&
                      std::fread(hdr, sizeof(int32_t), 5, f) == 5;
  if (!ok_hdr || hdr[0] != 4 || hdr[1] != 1 || hdr[4] < 1 || hdr[4] > 16 || hdr[2] < 1 || hdr[2] > 256 ||
      hdr[3] < 1 || hdr[3] > 15 || (hdr[3] % 2) == 0) {
    std::fclose(f);
    set_error("not a warm-start network file (bad magic or header)");
    return INFOESRF_ERR_INVALID_ARG;
  }
  const int H = hdr[2], K = hdr[3], D = hdr[4];
  const int64_t cnt = net_param_count(H, K, D);
  std::vector<float> host((size_t)cnt);
  const size_t got = std::fread(host.data(), sizeof(float), (size_t)cnt, f);
  std::fclose(f);
  IE_CHECK(got == (size_t)cnt, INFOESRF_ERR_INVALID_ARG, "truncated network file");
  Net* h = new Net();
  h->H = H;
  h->K = K;
  h->D = D;
  h->count = cnt;
  if (alloc_state(h) < 0 ||
      hipMemcpy(h->params, host.data(), sizeof(float) * cnt, hipMemcpyHostToDevice) != hipSuccess) {
    free_state(h);
    delete h;
    set_error("device allocation or copy failed for the network");
    return INFOESRF_ERR_HIP;
  }
  *net = h;
  return INFOESRF_OK;
}

extern "C" int infoesrf_net_save(const void* net, const char* path) {
  clear_error();
  IE_CHECK(path && net, INFOESRF_ERR_INVALID_ARG, "path and net must be non-NULL");
  const Net* h = static_cast<const Net*>(net);
  std::vector<float> host((size_t)h->count);
  IE_HIP(hipMemcpy(host.data(), h->params, sizeof(float) * h->count, hipMemcpyDeviceToHost));
  FILE* f = std::fopen(path, "wb");
  IE_CHECK(f != nullptr, INFOESRF_ERR_INVALID_ARG, std::string("cannot write ") + path);
  const int32_t hdr[5] = {4, 1, h->H, h->K, h->D};
  bool ok = std::fwrite("IENET002", 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int32_t), 5, f) == 5 &&
            std::fwrite(host.data(), sizeof(float), host.size(), f) == host.size();
  ok = (std::fclose(f) == 0) && ok;
  IE_CHECK(ok, INFOESRF_ERR_INVALID_ARG, std::string("write failed: ") + path);
  return INFOESRF_OK;
}

extern "C" void infoesrf_net_free(void* net) {
  if (!net) return;
  Net* h = static_cast<Net*>(net);
  free_state(h);
  delete h;
}

extern "C" int64_t infoesrf_net_param_count(const void* net) {
  return net ? static_cast<const Net*>(net)->count : 0;
}

extern "C" int infoesrf_net_get_params(const void* net, float* host) {
  clear_error();
  IE_CHECK(net && host, INFOESRF_ERR_INVALID_ARG, "net and host must be non-NULL");
  const Net* h = static_cast<const Net*>(net);
  IE_HIP(hipMemcpy(host, h->params, sizeof(float) * h->count, hipMemcpyDeviceToHost));
  return INFOESRF_OK;
}

extern "C" int infoesrf_net_set_params(void* net, const float* host) {
  clear_error();
  IE_CHECK(net && host, INFOESRF_ERR_INVALID_ARG, "net and host must be non-NULL");
  Net* h = static_cast<Net*>(net);
  IE_HIP(hipMemcpy(h->params, host, sizeof(float) * h->count, hipMemcpyHostToDevice));
  h->step = 0;
  IE_HIP(hipMemset(h->adam_m, 0, sizeof(float) * h->count));
  IE_HIP(hipMemset(h->adam_v, 0, sizeof(float) * h->count));
  return INFOESRF_OK;
}

extern "C" size_t infoesrf_net_workspace_bytes(const void* net, int64_t B, int64_t Q, int64_t m, int32_t training) {
  clear_error();
  if (check_net_io(static_cast<const Net*>(net), B, m) < 0) return 0;
  if (training && check_shifts(B, Q) < 0) return 0;
  return net_ws_bytes(*static_cast<const Net*>(net), B, training ? Q : 1, m, training != 0);
}

extern "C" int infoesrf_net_forward(const void* net, const float* X, int64_t B, int64_t m, float* Y, void* ws,
                                    size_t ws_bytes, void* stream) {
  clear_error();
  const Net* h = static_cast<const Net*>(net);
  IE_TRY(check_net_io(h, B, m));
  IE_CHECK(X && Y, INFOESRF_ERR_INVALID_ARG, "X and Y must be non-NULL");
  return net_forward(*h, X, B, m, Y, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

extern "C" int infoesrf_net_forward_bf16(const void* net, const float* X, int64_t B, int64_t m, float* Y, void* ws,
                                         size_t ws_bytes, void* stream) {
  clear_error();
  const Net* h = static_cast<const Net*>(net);
  IE_TRY(check_net_io(h, B, m));
  IE_CHECK(X && Y, INFOESRF_ERR_INVALID_ARG, "X and Y must be non-NULL");
  return net_forward_bf16(*h, X, B, m, Y, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

extern "C" int infoesrf_net_gradients(const void* net, const float* X, const float* cq, const float* T, int64_t B,
                                      int64_t Q, int64_t m, float* grads, float* loss, void* ws, size_t ws_bytes,
                                      void* stream) {
  clear_error();
  const Net* h = static_cast<const Net*>(net);
  IE_TRY(check_net_io(h, B, m));
  IE_TRY(check_shifts(B, Q));
  IE_CHECK(X && cq && T && grads, INFOESRF_ERR_INVALID_ARG, "X, cq, T and grads must be non-NULL");
  size_t need = 0;
  const NetWs w = carve(*h, B, Q, m, true, ws, &need);
  IE_CHECK(ws && ws_bytes >= need, INFOESRF_ERR_WORKSPACE, "network workspace too small");
  return gradients(*h, X, cq, T, B, Q, m, w, grads, loss, static_cast<hipStream_t>(stream));
}

extern "C" int infoesrf_net_train_step(void* net, const float* X, const float* cq, const float* T, int64_t B,
                                       int64_t Q, int64_t m, float lr, float* loss, void* ws, size_t ws_bytes,
                                       void* stream) {
  clear_error();
  Net* h = static_cast<Net*>(net);
  IE_TRY(check_net_io(h, B, m));
  IE_TRY(check_shifts(B, Q));
  IE_CHECK(X && cq && T, INFOESRF_ERR_INVALID_ARG, "X, cq and T must be non-NULL");
  IE_CHECK(lr > 0.f && std::isfinite(lr), INFOESRF_ERR_INVALID_ARG, "learning rate must be positive");
  size_t need = 0;
  const NetWs w = carve(*h, B, Q, m, true, ws, &need);
  IE_CHECK(ws && ws_bytes >= need, INFOESRF_ERR_WORKSPACE, "network workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  IE_TRY(gradients(*h, X, cq, T, B, Q, m, w, h->grads, loss, st));
  h->step += 1;
  IE_HIP(launch_adam(h->params, h->grads, h->adam_m, h->adam_v, h->count, lr, h->step, st));
  return INFOESRF_OK;
}
