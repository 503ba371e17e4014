// The normalized observation covariance S = R^{-1/2} H P H^T R^{-1/2} (the matrix of Theorem 3,
// applied in every shifted system of Appendix E) assembled once per call as a dense m x m
// matrix.  When m is small next to the covariance's band (few observations of a large state, as
// in the experiments of Sec. 4 and Sec. 5), an m x m product per PCG iteration costs far less
// than a pass over the band of P, and the band is then used only m times, to form S.
#include "internal.hpp"

namespace infoesrf {

namespace {

template <typename T>
__device__ inline T cast_to(double v);
template <>
__device__ inline double cast_to<double>(double v) {
  return v;
}
template <>
__device__ inline float cast_to<float>(double v) {
  return (float)v;
}

// V[c * ldv + r] = (r == j0 + c), r < rows, c < bc: unit columns of the observation space.
__global__ void k_unit_cols(int64_t rows, int64_t j0, int64_t bc, double* __restrict__ V, int64_t ldv) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= rows * bc) return;
  const int64_t c = t / rows, r = t - c * rows;
  V[c * ldv + r] = (r == j0 + c) ? 1.0 : 0.0;
}

// V[:, c] = H^T R^{-1/2} e_{j0 + c}: row j0 + c of H, scaled by r^{-1/2}, on a zeroed state
// column.  One thread per column adds the row's entries in order (repeated indices sum).
__global__ void k_scatter_unit_obs(const int32_t* __restrict__ h_ptr, const int32_t* __restrict__ h_idx,
                                   const double* __restrict__ h_w, const double* __restrict__ r_var, int64_t n,
                                   int64_t j0, int64_t bc, double* __restrict__ V, int64_t ldv) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= bc) return;
  const int64_t k = j0 + c;
  const double sc = 1.0 / sqrt(r_var[k]);
  double* col = V + c * ldv;
  for (int32_t e = h_ptr[k]; e < h_ptr[k + 1]; ++e) {
    const int32_t j = h_idx[e];
    if (j >= 0 && j < n) col[j] += sc * h_w[e];
  }
}

// S[(j0 + c) * lds + r] = (S e_{j0+c})_r from the apply output T: the observation-domain
// output itself, or R^{-1/2} H T for a state-domain output.
__global__ void k_gather_s_cols(int obs_domain, const double* __restrict__ T, int64_t ldt,
                                const int32_t* __restrict__ h_ptr, const int32_t* __restrict__ h_idx,
                                const double* __restrict__ h_w, const double* __restrict__ r_var, int64_t n,
                                int64_t m, int64_t j0, int64_t bc, double* __restrict__ S, int64_t lds) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m * bc) return;
  const int64_t c = t / m, r = t - c * m;
  const double* col = T + c * ldt;
  double v;
  if (obs_domain) {
    v = col[r];
  } else {
    double a = 0.0;
    for (int32_t e = h_ptr[r]; e < h_ptr[r + 1]; ++e) {
      const int32_t j = h_idx[e];
      if (j >= 0 && j < n) a += h_w[e] * col[j];
    }
    v = a / sqrt(r_var[r]);
  }
  S[(j0 + c) * lds + r] = v;
}

// S <- (S + S^T) / 2 (S is symmetric in exact arithmetic; its columns come from separate
// applies), and the FP32 copy when one is kept.
__global__ void k_symmetrize(double* __restrict__ S, int64_t m, int64_t lds, float* __restrict__ S32) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m * m) return;
  const int64_t c = t / m, r = t - c * m;
  if (r > c) return;  // each pair once, by its upper-triangle thread
  const double v = 0.5 * (S[c * lds + r] + S[r * lds + c]);
  S[c * lds + r] = v;
  S[r * lds + c] = v;
  if (S32) {
    S32[c * lds + r] = (float)v;
    S32[r * lds + c] = (float)v;
  }
}

// T[c * ldt + r] = sum_k S[k * lds + r] V[c * ldv + k] for r < m and slots c < *nact.
// A block computes 64 rows x 16 slots: thread t owns row t % 64 and slots 4 (t / 64) .. +3.
// Tiles of 32 along k of S (64 rows) and of V (16 slots) are staged in LDS: the S reads are
// unit-stride across a wave, the V reads are one broadcast word per wave.
constexpr int kDsRows = 64, kDsSlots = 16, kDsK = 32;

template <typename TS, typename TV, typename TT>
__global__ __launch_bounds__(256) void k_dense_s_apply(const TS* __restrict__ S, int64_t lds, int64_t m,
                                                       const TV* __restrict__ V, int64_t ldv,
                                                       const int32_t* __restrict__ nact, int64_t Bmax,
                                                       TT* __restrict__ T, int64_t ldt,
                                                       int32_t* __restrict__ zero_counter) {
  __shared__ double sS[kDsK][kDsRows];
  __shared__ double sV[kDsSlots][kDsK + 1];
  const int tid = threadIdx.x;
  const int64_t na = nact ? (int64_t)*nact : Bmax;
  if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0 && zero_counter) {
    zero_counter[0] = 0;  // list and live counters of the next PCG step (nobody reads them now)
    zero_counter[1] = 0;
  }
  const int64_t r0 = (int64_t)blockIdx.x * kDsRows, c0 = (int64_t)blockIdx.y * kDsSlots;
  if (c0 >= na) return;  // the whole block is past the active slots (uniform exit)
  const int rr = tid & (kDsRows - 1), sg = tid >> 6;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = 0; k0 < m; k0 += kDsK) {
    for (int o = tid; o < kDsK * kDsRows; o += 256) {
      const int kk = o / kDsRows, r = o - kk * kDsRows;
      const int64_t gk = k0 + kk, gr = r0 + r;
      sS[kk][r] = (gk < m && gr < m) ? (double)S[gk * lds + gr] : 0.0;
    }
    for (int o = tid; o < kDsSlots * kDsK; o += 256) {
      const int cc = o / kDsK, kk = o - cc * kDsK;
      const int64_t gk = k0 + kk, gc = c0 + cc;
      sV[cc][kk] = (gk < m && gc < na) ? (double)V[gc * ldv + gk] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kDsK; ++kk) {
      const double s = sS[kk][rr];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] += s * sV[sg * 4 + j][kk];
    }
    __syncthreads();
  }
  const int64_t gr = r0 + rr;
  if (gr >= m) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t gc = c0 + sg * 4 + j;
    if (gc < na) T[gc * ldt + gr] = cast_to<TT>(acc[j]);
  }
}

inline unsigned nblocks(int64_t count) { return (unsigned)((count + 255) / 256); }

}  // namespace

hipError_t launch_unit_cols(int64_t rows, int64_t j0, int64_t bc, double* V, int64_t ldv, hipStream_t st) {
  if (rows <= 0 || bc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unit_cols, dim3(nblocks(rows * bc)), dim3(256), 0, st, rows, j0, bc, V, ldv);
  return hipGetLastError();
}

hipError_t launch_scatter_unit_obs(const int32_t* h_ptr, const int32_t* h_idx, const double* h_w,
                                   const double* r_var, int64_t n, int64_t j0, int64_t bc, double* V, int64_t ldv,
                                   hipStream_t st) {
  if (bc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_unit_obs, dim3(nblocks(bc)), dim3(256), 0, st, h_ptr, h_idx, h_w, r_var, n, j0, bc,
                     V, ldv);
  return hipGetLastError();
}

hipError_t launch_gather_s_cols(int obs_domain, const double* T, int64_t ldt, const int32_t* h_ptr,
                                const int32_t* h_idx, const double* h_w, const double* r_var, int64_t n, int64_t m,
                                int64_t j0, int64_t bc, double* S, int64_t lds, hipStream_t st) {
  if (m <= 0 || bc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_s_cols, dim3(nblocks(m * bc)), dim3(256), 0, st, obs_domain, T, ldt, h_ptr, h_idx,
                     h_w, r_var, n, m, j0, bc, S, lds);
  return hipGetLastError();
}

hipError_t launch_symmetrize(double* S, int64_t m, int64_t lds, float* S32, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_symmetrize, dim3(nblocks(m * m)), dim3(256), 0, st, S, m, lds, S32);
  return hipGetLastError();
}

hipError_t launch_dense_s_apply(Prec prec, const void* S, int64_t lds, int64_t m, const void* V, int64_t ldv,
                                const int32_t* nact, int64_t Bmax, void* T, int64_t ldt, int32_t* zero_counter,
                                hipStream_t st) {
  if (!S || !V || !T) return hipErrorInvalidValue;
  const int64_t cb = std::max<int64_t>(1, (Bmax + kDsSlots - 1) / kDsSlots);
  const dim3 grid((unsigned)((m + kDsRows - 1) / kDsRows), (unsigned)cb);
  if (m <= 0) return hipSuccess;
  if (prec == Prec::F64) {
    hipLaunchKernelGGL((k_dense_s_apply<double, double, double>), grid, dim3(256), 0, st, (const double*)S, lds, m,
                       (const double*)V, ldv, nact, Bmax, (double*)T, ldt, zero_counter);
  } else if (prec == Prec::F32) {
    hipLaunchKernelGGL((k_dense_s_apply<float, float, float>), grid, dim3(256), 0, st, (const float*)S, lds, m,
                       (const float*)V, ldv, nact, Bmax, (float*)T, ldt, zero_counter);
  } else {
    return hipErrorInvalidValue;  // no BF16 dense form
  }
  return hipGetLastError();
}

}  // namespace infoesrf
