// Kernels of the warm-start network (a 1-D convolutional net over the m observation rows; the
// method's extension for initial guesses of the shifted systems, Appendix E, eq. E.1).
//
// Layout: activations of a batch are (B, C, m) row-contiguous, element (b, c, x) at
// (b * C + c) * m + x.  Weights (Cout, Cin, K) row-contiguous, K odd, "same" zero padding:
//
//   y[b, o, x] = bias[o] + sum_c sum_k W[o, c, k] a[b, c, x + k - K/2].
//
// All arithmetic is FP32 (accumulation in FP32, reductions in a fixed order).
#include <cmath>

#include "internal.hpp"

namespace infoesrf {

namespace {

constexpr int kTX = 64;    // positions per block (one per lane)
constexpr int kCIC = 16;   // input channels staged per chunk

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float z) {
  const float Phi = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float phi = 0.39894228040143268f * expf(-0.5f * z * z);
  return Phi + z * phi;
}

// Direct correlation.  Block: 64 positions (lanes) x 4 * CPW output channels (CPW per wave).
// Input window and weight chunk in LDS; weights are read as wave-uniform broadcasts.
template <int CPW>
__global__ __launch_bounds__(256) void k_conv_fwd(const float* __restrict__ in, int Cin, const float* __restrict__ W,
                                                  const float* __restrict__ bias, int Cout, int K, int m,
                                                  float* __restrict__ pre, float* __restrict__ act, int gelu) {
  extern __shared__ float sm[];
  const int h = K / 2;
  const int WX = kTX + K - 1;
  float* win = sm;                      // kCIC x WX
  float* wts = sm + kCIC * WX;          // (4 CPW) x kCIC x K
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x0 = blockIdx.x * kTX;
  const int o0 = blockIdx.y * 4 * CPW;
  const int64_t b = blockIdx.z;
  const float* inb = in + b * (int64_t)Cin * m;
  float acc[CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) acc[j] = 0.f;
  for (int c0 = 0; c0 < Cin; c0 += kCIC) {
    const int cc = min(kCIC, Cin - c0);
    __syncthreads();
    for (int t = threadIdx.x; t < kCIC * WX; t += 256) {
      const int ci = t / WX, u = t % WX;
      const int x = x0 - h + u;
      win[t] = (ci < cc && x >= 0 && x < m) ? inb[(int64_t)(c0 + ci) * m + x] : 0.f;
    }
    for (int t = threadIdx.x; t < 4 * CPW * kCIC * K; t += 256) {
      const int o = t / (kCIC * K), rem = t % (kCIC * K), ci = rem / K, k = rem % K;
      wts[t] = (o0 + o < Cout && ci < cc) ? W[((int64_t)(o0 + o) * Cin + c0 + ci) * K + k] : 0.f;
    }
    __syncthreads();
    for (int ci = 0; ci < cc; ++ci)
      for (int k = 0; k < K; ++k) {
        const float v = win[ci * WX + lane + k];
#pragma unroll
        for (int j = 0; j < CPW; ++j) acc[j] = fmaf(wts[((wave * CPW + j) * kCIC + ci) * K + k], v, acc[j]);
      }
  }
  const int x = x0 + lane;
  if (x >= m) return;
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int o = o0 + wave * CPW + j;
    if (o >= Cout) continue;
    const float z = acc[j] + (bias ? bias[o] : 0.f);
    const int64_t at = (b * Cout + o) * (int64_t)m + x;
    if (pre) pre[at] = z;
    act[at] = gelu ? gelu_f(z) : z;
  }
}

// ---- BF16 inference on MFMA (FP32 accumulation) --------------------------------------------
// The same correlation as an implicit GEMM: y[o, x] = bias[o] + sum_kd Wp[o, kd] A[kd, x] with
// kd = k Cp + c (Cp = input channels rounded up to 8, so the 8 values a lane feeds to one MFMA
// share k and are consecutive channels), A[kd, x] = a[c, x + k - K/2].  Weights are packed once
// per call to BF16 rows of KD = round_up(K Cp, 32) entries (Cout rounded up to 16 rows, zeros in
// the padding).  Activations between layers are BF16, position-major (b, x, c).
typedef __bf16 nbf8 __attribute__((ext_vector_type(8)));
typedef float nf4 __attribute__((ext_vector_type(4)));

__global__ void k_pack_weights_bf16(const float* __restrict__ W, int Cout, int Cin, int K, int Cp, int KD, int Opad,
                                    __hip_bfloat16* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)Opad * KD) return;
  const int o = (int)(t / KD), kd = (int)(t % KD);
  const int k = kd / Cp, c = kd % Cp;
  const float v = (o < Cout && k < K && c < Cin) ? W[((int64_t)o * Cin + c) * K + k] : 0.f;
  out[t] = __float2bfloat16(v);
}

// Block: 64 positions x 64 output channels (wavefront w: channels o0 + 16 w .. + 15, four
// 16-position tiles).  The input window (64 + K - 1 positions x Cp channels) is staged in LDS as
// BF16, rows padded by 8 channels (16 bytes) against bank conflicts.
// IN_F32: input (B, Cin, m) FP32, else (B, m, Cp) BF16.  OUT_F32: output (B, Cout, m) FP32, else
// (B, m, Cout) BF16.
template <bool IN_F32, bool OUT_F32>
__global__ __launch_bounds__(256) void k_conv_bf16(const void* __restrict__ in, int Cin, int Cp,
                                                   const __hip_bfloat16* __restrict__ Wp, int KD,
                                                   const float* __restrict__ bias, int Cout, int K, int m,
                                                   void* __restrict__ out, int gelu) {
  extern __shared__ __attribute__((aligned(16))) unsigned char nsm[];
  __hip_bfloat16* win = reinterpret_cast<__hip_bfloat16*>(nsm);
  const int h = K / 2;
  const int WX = 64 + K - 1;
  const int Cs = Cp + 8;  // LDS row stride (channels)
  const int x0 = blockIdx.x * 64;
  const int o0 = blockIdx.y * 64;
  const int64_t b = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lrow = lane & 15, lk = lane >> 4;
  for (int t = tid; t < WX * Cp; t += 256) {
    const int u = t / Cp, c = t % Cp;
    const int x = x0 - h + u;
    float v = 0.f;
    if (x >= 0 && x < m && c < Cin) {
      if (IN_F32) v = static_cast<const float*>(in)[(b * Cin + c) * (int64_t)m + x];
      else v = __bfloat162float(static_cast<const __hip_bfloat16*>(in)[(b * m + x) * (int64_t)Cp + c]);
    }
    win[u * Cs + c] = __float2bfloat16(v);
  }
  __syncthreads();
  const int ob = o0 + 16 * wave;
  if (ob >= Cout) return;  // no channels for this wavefront (after the only barrier)
  nf4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = nf4{0.f, 0.f, 0.f, 0.f};
  const __hip_bfloat16* wrow = Wp + (int64_t)(ob + lrow) * KD + 8 * lk;
  for (int kd0 = 0; kd0 < KD; kd0 += 32) {
    const nbf8 a = *reinterpret_cast<const nbf8*>(wrow + kd0);
    const int kd = kd0 + 8 * lk;
    const int k = kd / Cp, c0 = kd % Cp;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      nbf8 bv;
      if (k < K) {
        bv = *reinterpret_cast<const nbf8*>(win + (16 * t + lrow + k) * Cs + c0);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) bv[i] = (__bf16)0.f;
      }
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc[t], 0, 0, 0);
    }
  }
  // D register v of lane l: channel ob + 4 (l / 16) + v, position x0 + 16 t + l % 16
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int x = x0 + 16 * t + lrow;
    if (x >= m) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int o = ob + 4 * lk + v;
      if (o >= Cout) continue;
      const float z = acc[t][v] + (bias ? bias[o] : 0.f);
      const float y = gelu ? gelu_f(z) : z;
      if (OUT_F32) static_cast<float*>(out)[(b * Cout + o) * (int64_t)m + x] = y;
      else static_cast<__hip_bfloat16*>(out)[(b * m + x) * (int64_t)Cout + o] = __float2bfloat16(y);
    }
  }
}

// Weight gradient of one layer: gW[o, c, k] = sum_{b, x} g[b, o, x] a[b, c, x + k - K/2] and
// gb[o] = sum_{b, x} g[b, o, x].  Block (o, c-group of 8): threads stride over (b, x) and keep
// 8 K partial sums; then a fixed-order reduction (wave shuffles, then the four waves).
__global__ __launch_bounds__(256) void k_conv_wgrad(const float* __restrict__ a, int Cin, const float* __restrict__ g,
                                                    int Cout, int K, int m, int64_t B, float* __restrict__ gW,
                                                    float* __restrict__ gb) {
  constexpr int CG = 8;
  constexpr int KMAX = 15;
  __shared__ float red[4][CG * KMAX + 1];
  const int o = blockIdx.x;
  const int c0 = blockIdx.y * CG;
  const int h = K / 2;
  float acc[CG * KMAX + 1];
#pragma unroll
  for (int j = 0; j < CG * KMAX + 1; ++j) acc[j] = 0.f;
  const int64_t total = B * (int64_t)m;
  for (int64_t p = threadIdx.x; p < total; p += 256) {
    const int64_t b = p / m;
    const int x = (int)(p % m);
    const float gv = g[(b * Cout + o) * (int64_t)m + x];
    acc[CG * KMAX] += gv;
#pragma unroll
    for (int cj = 0; cj < CG; ++cj) {
      const int c = c0 + cj;
      if (c >= Cin) break;
      const float* ar = a + (b * Cin + c) * (int64_t)m;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k >= K) break;
        const int xs = x + k - h;
        if (xs >= 0 && xs < m) acc[cj * KMAX + k] = fmaf(gv, ar[xs], acc[cj * KMAX + k]);
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < CG * KMAX + 1; ++j) {
    float v = acc[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave][j] = v;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < CG * KMAX + 1; j += 256) {
    const float v = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
    if (j == CG * KMAX) {
      if (blockIdx.y == 0) gb[o] = v;
    } else {
      const int cj = j / KMAX, k = j % KMAX;
      if (c0 + cj < Cin && k < K) gW[((int64_t)o * Cin + c0 + cj) * K + k] = v;
    }
  }
}

// W' (Cin, Cout, K) with W'[c, o, k] = W[o, c, K - 1 - k]: the input gradient of a "same"
// correlation is the correlation of the output gradient with W'.
__global__ void k_flip_transpose(const float* __restrict__ W, int Cout, int Cin, int K, float* __restrict__ Wt) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)Cout * Cin * K;
  if (t >= n) return;
  const int k = (int)(t % K);
  const int64_t oc = t / K;
  const int o = (int)(oc / Cin), c = (int)(oc % Cin);
  Wt[((int64_t)c * Cout + o) * K + (K - 1 - k)] = W[t];
}

// g *= GELU'(z) elementwise.
__global__ void k_gelu_bwd(float* __restrict__ g, const float* __restrict__ z, int64_t n) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) g[t] *= gelu_grad_f(z[t]);
}

// mean of B values in one block (fixed order)
__global__ void k_mean(const float* __restrict__ v, int64_t B, float* __restrict__ out) {
  __shared__ float s[256];
  float a = 0.f;
  for (int64_t i = threadIdx.x; i < B; i += 256) a += v[i];
  s[threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    float tot = 0.f;
    for (int i = 0; i < 256; ++i) tot += s[i];
    *out = tot / (float)B;
  }
}

// Adam (Kingma & Ba, Algorithm 1); c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ mo,
                       float* __restrict__ ve, int64_t n, float lr, float beta1, float beta2, float eps, float c1,
                       float c2) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gi = g[t];
  const float m1 = beta1 * mo[t] + (1.f - beta1) * gi;
  const float v1 = beta2 * ve[t] + (1.f - beta2) * gi * gi;
  mo[t] = m1;
  ve[t] = v1;
  p[t] -= lr * (m1 * c1) / (sqrtf(v1 * c2) + eps);
}

// The shift head (per system (b, q) of a batch of B members x Q shifts, c_q = 1 / (1 + s_q)):
// y_{b,q} = sum_d c_q^(d+1) Y[b, d] over the trunk output Y (B, D, m).
__device__ inline float head_value(const float* __restrict__ Y, int64_t b, int D, int m, int x, float c) {
  float y = 0.f, p = c;
  for (int d = 0; d < D; ++d) {
    y = fmaf(p, Y[(b * D + d) * (int64_t)m + x], y);
    p *= c;
  }
  return y;
}

// Relative L2 loss of each system against its target T (B, Q, m): per[b Q + q] = ||y - t|| / ||t||
// and scale[b Q + q] = 1 / (||y - t|| ||t|| B Q), the factor of its gradient.  One block per system.
__global__ __launch_bounds__(256) void k_head_rel_l2(const float* __restrict__ Y, int D, const float* __restrict__ cq,
                                                     int Q, const float* __restrict__ T, int m, int64_t B,
                                                     float* __restrict__ per, float* __restrict__ scale) {
  __shared__ float sd[4], st[4];
  const int64_t sys = blockIdx.x, b = sys / Q;
  const float c = cq[sys % Q];
  float dd = 0.f, tt = 0.f;
  for (int x = threadIdx.x; x < m; x += 256) {
    const float tv = T[sys * m + x];
    const float d = head_value(Y, b, D, m, x, c) - tv;
    dd = fmaf(d, d, dd);
    tt = fmaf(tv, tv, tt);
  }
  for (int off = 32; off > 0; off >>= 1) {
    dd += __shfl_xor(dd, off, 64);
    tt += __shfl_xor(tt, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sd[wave] = dd;
    st[wave] = tt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float dn = sqrtf(((sd[0] + sd[1]) + sd[2]) + sd[3]);
    const float tn = sqrtf(((st[0] + st[1]) + st[2]) + st[3]);
    scale[sys] = (dn > 0.f && tn > 0.f) ? 1.0f / (dn * tn * (float)(B * Q)) : 0.f;
    per[sys] = tn > 0.f ? dn / tn : 0.f;
  }
}

// Gradient of the mean loss w.r.t. the trunk output: gY[b, d, x] = sum_q c_q^(d+1) scale_{b,q}
// (y_{b,q}[x] - T_{b,q}[x]).  One thread per (b, x).
__global__ void k_head_grad(const float* __restrict__ Y, int D, const float* __restrict__ cq, int Q,
                            const float* __restrict__ T, const float* __restrict__ scale, int m, int64_t B,
                            float* __restrict__ gY) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= B * m) return;
  const int64_t b = t / m;
  const int x = (int)(t % m);
  float g[16];
  for (int d = 0; d < D; ++d) g[d] = 0.f;
  for (int q = 0; q < Q; ++q) {
    const float c = cq[q];
    const float r = scale[b * Q + q] * (head_value(Y, b, D, m, x, c) - T[(b * Q + q) * (int64_t)m + x]);
    float p = c;
    for (int d = 0; d < D; ++d) {
      g[d] = fmaf(p, r, g[d]);
      p *= c;
    }
  }
  for (int d = 0; d < D; ++d) gY[(b * D + d) * (int64_t)m + x] = g[d];
}

}  // namespace

static unsigned nb1(int64_t n) { return (unsigned)((n + 255) / 256); }

size_t net_conv_smem(int K, int CPW) { return sizeof(float) * ((size_t)kCIC * (kTX + K - 1) + 4 * CPW * kCIC * K); }

hipError_t launch_conv_fwd(const float* in, int Cin, const float* W, const float* bias, int Cout, int K, int m,
                           int64_t B, float* pre, float* act, int gelu, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  if (!in || !W || !act || K < 1 || K > 15 || (K % 2) == 0) return hipErrorInvalidValue;
  const unsigned gx = (unsigned)((m + kTX - 1) / kTX);
  if (Cout >= 16) {
    constexpr int CPW = 4;
    dim3 grid(gx, (unsigned)((Cout + 4 * CPW - 1) / (4 * CPW)), (unsigned)B);
    hipLaunchKernelGGL((k_conv_fwd<CPW>), grid, dim3(256), net_conv_smem(K, CPW), st, in, Cin, W, bias, Cout, K, m,
                       pre, act, gelu);
  } else {
    constexpr int CPW = 1;
    dim3 grid(gx, (unsigned)((Cout + 3) / 4), (unsigned)B);
    hipLaunchKernelGGL((k_conv_fwd<CPW>), grid, dim3(256), net_conv_smem(K, CPW), st, in, Cin, W, bias, Cout, K, m,
                       pre, act, gelu);
  }
  return hipGetLastError();
}

int bf16_cp(int Cin) { return (Cin + 7) / 8 * 8; }
int bf16_kd(int Cin, int K) { return (K * bf16_cp(Cin) + 31) / 32 * 32; }
int bf16_opad(int Cout) { return (Cout + 15) / 16 * 16; }

hipError_t launch_pack_weights_bf16(const float* W, int Cout, int Cin, int K, __hip_bfloat16* out, hipStream_t st) {
  const int Cp = bf16_cp(Cin), KD = bf16_kd(Cin, K), Op = bf16_opad(Cout);
  const int64_t cnt = (int64_t)Op * KD;
  hipLaunchKernelGGL(k_pack_weights_bf16, dim3(nb1(cnt)), dim3(256), 0, st, W, Cout, Cin, K, Cp, KD, Op, out);
  return hipGetLastError();
}

hipError_t launch_conv_bf16(const void* in, bool in_f32, int Cin, const __hip_bfloat16* Wp, const float* bias, int Cout,
                            int K, int m, int64_t B, void* out, bool out_f32, int gelu, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  if (!in || !Wp || !out || K < 1 || K > 15 || (K % 2) == 0 || Cin > 64 || Cout > 64) return hipErrorInvalidValue;

  if (!in_f32 && bf16_cp(Cin) != Cin) return hipErrorInvalidValue;  // BF16 inputs carry Cp channels
  const int Cp = bf16_cp(Cin), KD = bf16_kd(Cin, K);
  const size_t smem = sizeof(__hip_bfloat16) * (size_t)(64 + K - 1) * (Cp + 8);
  const dim3 grid((unsigned)((m + 63) / 64), (unsigned)((Cout + 63) / 64), (unsigned)B);
#define IE_CB(I, O)                                                                                             \
  hipLaunchKernelGGL((k_conv_bf16<I, O>), grid, dim3(256), smem, st, in, Cin, Cp, Wp, KD, bias, Cout, K, m, out, \
                     gelu)
  if (in_f32 && out_f32) IE_CB(true, true);
  else if (in_f32) IE_CB(true, false);
  else if (out_f32) IE_CB(false, true);
  else IE_CB(false, false);
#undef IE_CB
  return hipGetLastError();
}

hipError_t launch_conv_wgrad(const float* a, int Cin, const float* g, int Cout, int K, int m, int64_t B, float* gW,
                             float* gb, hipStream_t st) {
  if (K < 1 || K > 15) return hipErrorInvalidValue;
  dim3 grid((unsigned)Cout, (unsigned)((Cin + 7) / 8));
  hipLaunchKernelGGL(k_conv_wgrad, grid, dim3(256), 0, st, a, Cin, g, Cout, K, m, B, gW, gb);
  return hipGetLastError();
}

hipError_t launch_flip_transpose(const float* W, int Cout, int Cin, int K, float* Wt, hipStream_t st) {
  const int64_t n = (int64_t)Cout * Cin * K;
  hipLaunchKernelGGL(k_flip_transpose, dim3(nb1(n)), dim3(256), 0, st, W, Cout, Cin, K, Wt);
  return hipGetLastError();
}

hipError_t launch_gelu_bwd(float* g, const float* z, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_gelu_bwd, dim3(nb1(n)), dim3(256), 0, st, g, z, n);
  return hipGetLastError();
}

hipError_t launch_head_loss_grad(const float* Y, int D, const float* cq, int Q, const float* T, int m, int64_t B,
                                 float* per, float* scale, float* mean, float* gY, hipStream_t st) {
  if (D < 1 || D > 16 || Q < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_head_rel_l2, dim3((unsigned)(B * Q)), dim3(256), 0, st, Y, D, cq, Q, T, m, B, per, scale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, st, per, B * Q, mean);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_head_grad, dim3(nb1(B * m)), dim3(256), 0, st, Y, D, cq, Q, T, scale, m, B, gY);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* mo, float* ve, int64_t n, float lr, int64_t t,
                       hipStream_t st) {
  const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)t)));
  hipLaunchKernelGGL(k_adam, dim3(nb1(n)), dim3(256), 0, st, p, g, mo, ve, n, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace infoesrf
