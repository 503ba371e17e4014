// Pieces of a cycled assimilation around the update: the multi-layer Lorenz-96 forecast
// (Sec. 5.1, eq. 5.1) integrated with classical RK4, synthetic observations y = H x + noise,
// and the analysis ensemble with relaxation to prior spread (the posterior inflation of
// Sec. 5.3).
#include <atomic>
#include <cmath>

#include "internal.hpp"

namespace infoesrf {

namespace {

constexpr int kFcThreads = 512;
constexpr int kFcPer = 16;  // state entries per thread: n <= 8192

// One block integrates one ensemble column for `steps` RK4 steps.  The column stays on chip:
// each thread keeps its entries' state and RK sum in registers, and stage inputs (which
// neighbours read) go through two LDS buffers used in turn.
__global__ __launch_bounds__(kFcThreads) void k_l96_forecast(double* __restrict__ X, int64_t ld, int nz, int nx,
                                                             const double* __restrict__ forcing, double gamma,
                                                             double dt, int steps) {
  extern __shared__ double fs[];  // 2 x n
  const int n = nz * nx;
  double* col = X + (int64_t)blockIdx.x * ld;
  double* buf[2] = {fs, fs + n};
  double x[kFcPer], acc[kFcPer], kk[kFcPer], F[kFcPer];
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < kFcPer; ++e) {
    const int i = t + e * kFcThreads;
    x[e] = i < n ? col[i] : 0.0;
    F[e] = i < n ? forcing[i / nx] : 0.0;
  }
  auto tendency = [&](const double* s, int e) {
    const int i = t + e * kFcThreads;
    const int j = i / nx, c = i - j * nx;
    const int row = j * nx;
    const int cm1 = c == 0 ? nx - 1 : c - 1;
    const int cp1 = c == nx - 1 ? 0 : c + 1;
    const int cm2 = c >= 2 ? c - 2 : c - 2 + nx;
    const double xi = s[i];
    double v = s[row + cm1] * (s[row + cp1] - s[row + cm2]) - xi + F[e];
    if (j > 0) v += gamma * (s[i - nx] - xi);
    if (j < nz - 1) v += gamma * (s[i + nx] - xi);
    return v;
  };
  int cur = 0;
#pragma unroll
  for (int e = 0; e < kFcPer; ++e) {
    const int i = t + e * kFcThreads;
    if (i < n) buf[cur][i] = x[e];
  }
  __syncthreads();
  for (int st = 0; st < steps; ++st) {
    // stages: k1 = f(x), k2 = f(x + dt/2 k1), k3 = f(x + dt/2 k2), k4 = f(x + dt k3)
    for (int stage = 0; stage < 4; ++stage) {
      const double* s = buf[cur];
      double* nxt = buf[cur ^ 1];
      const double wsum = (stage == 0 || stage == 3) ? 1.0 : 2.0;
      const double cin = (stage < 2) ? 0.5 * dt : dt;  // coefficient of k for the next stage input
#pragma unroll
      for (int e = 0; e < kFcPer; ++e) {
        const int i = t + e * kFcThreads;
        if (i < n) {
          kk[e] = tendency(s, e);
          acc[e] = (stage == 0 ? 0.0 : acc[e]) + wsum * kk[e];
          if (stage < 3) nxt[i] = x[e] + cin * kk[e];
          else {
            x[e] += dt / 6.0 * acc[e];
            nxt[i] = x[e];
          }
        }
      }
      __syncthreads();
      cur ^= 1;
    }
  }
#pragma unroll
  for (int e = 0; e < kFcPer; ++e) {
    const int i = t + e * kFcThreads;
    if (i < n) col[i] = x[e];
  }
}

// y[r] = sum_e h_w[e] x[h_idx[e]] + noise[r] (indices outside [0, n) are skipped).
__global__ void k_observe(const int32_t* __restrict__ h_ptr, const int32_t* __restrict__ h_idx,
                          const double* __restrict__ h_w, const double* __restrict__ x, int64_t n,
                          const double* __restrict__ noise, int64_t m, double* __restrict__ y) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= m) return;
  double a = 0.0;
  for (int32_t e = h_ptr[r]; e < h_ptr[r + 1]; ++e) {
    const int32_t j = h_idx[e];
    if (j >= 0 && j < n) a += h_w[e] * x[j];
  }
  y[r] = a + (noise ? noise[r] : 0.0);
}

// Analysis members X[k, i] = mean_a[k] + f_k Xa'[k, i] with the relaxation-to-prior-spread factor
// f_k = 1 + alpha (sigma_f - sigma_a) / sigma_a of row k (sigma from the forecast members Xf and
// the analysis deviations; f_k = 1 where sigma_a = 0).  One thread per state variable.
// Xout may alias Xf: each thread reads its row completely before writing it.
__global__ void k_rtps_assemble(const double* Xf, int64_t ldf, const double* __restrict__ mean_a,
                                const double* __restrict__ Xa, int64_t lda, int64_t n, int N, double alpha,
                                double* Xout, int64_t ldo) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  double mf = 0.0;
  for (int i = 0; i < N; ++i) mf += Xf[(int64_t)i * ldf + k];
  mf /= N;
  double vf = 0.0, va = 0.0;
  for (int i = 0; i < N; ++i) {
    const double df = Xf[(int64_t)i * ldf + k] - mf;
    const double da = Xa[(int64_t)i * lda + k];
    vf += df * df;
    va += da * da;
  }
  const double sf = sqrt(vf / (N - 1)), sa = sqrt(va / (N - 1));
  const double f = sa > 0.0 ? 1.0 + alpha * (sf - sa) / sa : 1.0;
  const double mu = mean_a[k];
  for (int i = 0; i < N; ++i) Xout[(int64_t)i * ldo + k] = mu + f * Xa[(int64_t)i * lda + k];
}

}  // namespace

}  // namespace infoesrf

using namespace infoesrf;

extern "C" int infoesrf_l96_forecast(double* X, int64_t ld, int64_t k, int32_t nz, int32_t nx,
                                     const double* forcing, double gamma, double dt, int32_t steps, void* stream) {
  clear_error();
  IE_CHECK(X && forcing, INFOESRF_ERR_INVALID_ARG, "X and forcing must be non-NULL");
  IE_CHECK(nz >= 1 && nx >= 4, INFOESRF_ERR_INVALID_ARG, "need nz >= 1 and nx >= 4");
  const int64_t n = (int64_t)nz * nx;
  IE_CHECK(n <= (int64_t)kFcThreads * kFcPer, INFOESRF_ERR_INVALID_ARG, "the forecast kernel holds n <= 8192");
  IE_CHECK(ld >= n && k >= 0 && steps >= 0, INFOESRF_ERR_INVALID_ARG, "need ld >= n, k >= 0, steps >= 0");
  IE_CHECK(std::isfinite(dt) && std::isfinite(gamma), INFOESRF_ERR_INVALID_ARG, "dt and gamma must be finite");
  if (k == 0 || steps == 0) return INFOESRF_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t smem = 2 * sizeof(double) * (size_t)n;
  static std::atomic<bool> attr{false};  // set once (before any graph capture that follows)
  if (smem > 64 * 1024 && !attr.load(std::memory_order_acquire)) {
    IE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_l96_forecast),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
    attr.store(true, std::memory_order_release);
  }
  hipLaunchKernelGGL(k_l96_forecast, dim3((unsigned)k), dim3(kFcThreads), smem, st, X, ld, (int)nz, (int)nx, forcing,
                     gamma, dt, (int)steps);
  IE_HIP(hipGetLastError());
  return INFOESRF_OK;
}

extern "C" int infoesrf_observe(const infoesrf_problem* prob, const double* x, const double* noise, double* y,
                                void* stream) {
  clear_error();
  IE_CHECK(prob && prob->h_ptr && prob->h_idx && prob->h_w && x && y, INFOESRF_ERR_INVALID_ARG,
           "problem, H, x and y must be non-NULL");
  IE_CHECK(prob->m >= 1 && prob->n >= 1, INFOESRF_ERR_INVALID_ARG, "need n, m >= 1");
  hipLaunchKernelGGL(k_observe, dim3((unsigned)((prob->m + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), prob->h_ptr, prob->h_idx, prob->h_w, x, prob->n, noise, prob->m,
                     y);
  IE_HIP(hipGetLastError());
  return INFOESRF_OK;
}

extern "C" int infoesrf_rtps_assemble(const double* Xf, int64_t ldf, const double* mean_a, const double* Xa_pert,
                                      int64_t lda, int64_t n, int64_t N, double alpha, double* Xout, int64_t ldo,
                                      void* stream) {
  clear_error();
  IE_CHECK(Xf && mean_a && Xa_pert && Xout, INFOESRF_ERR_INVALID_ARG, "arrays must be non-NULL");
  IE_CHECK(n >= 1 && N >= 2 && ldf >= n && lda >= n && ldo >= n, INFOESRF_ERR_INVALID_ARG,
           "need n >= 1, N >= 2 and leading dimensions >= n");
  IE_CHECK(std::isfinite(alpha) && alpha >= 0.0 && alpha <= 1.0, INFOESRF_ERR_INVALID_ARG, "alpha must be in [0, 1]");
  hipLaunchKernelGGL(k_rtps_assemble, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), Xf, ldf, mean_a, Xa_pert, lda, n, (int)N, alpha, Xout, ldo);
  IE_HIP(hipGetLastError());
  return INFOESRF_OK;
}
