// Ensemble statistics and observation-operator kernels (gfx950).
//
//  * ensemble mean and normalized perturbations (Sec. 2.2, eq. 2.9)
//  * R^{-1/2}-scaled observed perturbations b_i = R^{-1/2} H z_i and the
//    innovation R^{-1/2}(y - H mu) (Appendix E, eq. E.1; Sec. 3.2, eq. 3.4)
//  * diag(S), used by the preconditioner's beta (Appendix E)
//  * CSR -> CSC transpose of H for the scatter H^T R^{-1/2} u
#include "internal.hpp"

namespace infoesrf {

namespace {

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t count, int per = kBlock) { return (unsigned)((count + per - 1) / per); }

__global__ void k_ens_stats(const double* __restrict__ X, int64_t n, int64_t N, double* __restrict__ mu,
                            double* __restrict__ Z, float* __restrict__ Z32) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  // the members eight at a time: their loads in flight together, the sum in member order
  constexpr int U = 8;
  double s = 0.0;
  int64_t i = 0;
  for (; i + U <= N; i += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = X[k + (i + u) * n];
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  for (; i < N; ++i) s += X[k + i * n];
  const double m = s / (double)N;
  mu[k] = m;
  const double sc = 1.0 / sqrt((double)(N - 1));
  for (i = 0; i < N; i += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = i + u < N ? X[k + (i + u) * n] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i + u < N) {
        const double z = (v[u] - m) * sc;
        Z[k + (i + u) * n] = z;
        if (Z32) Z32[k + (i + u) * n] = (float)z;
      }
    }
  }
}

// Column counts of H (one thread per CSR row); also validates indices and that the entry count
// fits the cap entries the CSC copy has room for.
__global__ void k_csc_count(const int32_t* __restrict__ h_ptr, const int32_t* __restrict__ h_idx, int64_t m,
                            int64_t n, int64_t cap, int32_t* __restrict__ cnt, int32_t* __restrict__ flags) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= m) return;
  const int32_t e0 = h_ptr[r], e1 = h_ptr[r + 1];
  if (e1 < e0 || e0 < 0 || e1 > h_ptr[m] || (int64_t)h_ptr[m] > cap || (r == 0 && e0 != 0)) {
    atomicOr(flags, kFlagBadInput);
    return;
  }
  int32_t prev = -1;
  for (int32_t e = e0; e < e1; ++e) {
    const int32_t c = h_idx[e];
    if (c < 0 || c >= n || c <= prev) {
      atomicOr(flags, kFlagBadInput);
      return;
    }
    prev = c;
    atomicAdd(&cnt[c], 1);
  }
}

// Exclusive scan of n counts in one block (n may be large: serial chunks per thread).
__global__ void k_scan_one_block(const int32_t* __restrict__ cnt, int64_t n, int32_t* __restrict__ out_ptr) {
  __shared__ int32_t part[kBlock];
  const int t = threadIdx.x;
  const int64_t per = (n + kBlock - 1) / kBlock;
  const int64_t a = t * per, b = min<int64_t>(n, a + per);
  int32_t s = 0;
  for (int64_t k = a; k < b; ++k) s += cnt[k];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int32_t run = 0;
    for (int i = 0; i < kBlock; ++i) {
      const int32_t v = part[i];
      part[i] = run;
      run += v;
    }
    out_ptr[n] = run;
  }
  __syncthreads();
  int32_t run = part[t];
  for (int64_t k = a; k < b; ++k) {
    out_ptr[k] = run;
    run += cnt[k];
  }
}

__global__ void k_csc_fill(const int32_t* __restrict__ h_ptr, const int32_t* __restrict__ h_idx,
                           const double* __restrict__ h_w, int64_t m, const int32_t* __restrict__ col_ptr,
                           int32_t* __restrict__ cursor, int32_t* __restrict__ row_of, double* __restrict__ w_of,
                           const int32_t* __restrict__ flags) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= m || *flags) return;
  for (int32_t e = h_ptr[r]; e < h_ptr[r + 1]; ++e) {
    const int32_t c = h_idx[e];
    const int32_t pos = col_ptr[c] + atomicAdd(&cursor[c], 1);
    row_of[pos] = (int32_t)r;
    w_of[pos] = h_w[e];
  }
}

// Sort each column's entries by row so the scatter sums in a fixed order.
__global__ void k_csc_sort(const int32_t* __restrict__ col_ptr, int64_t n, int32_t* __restrict__ row_of,
                           double* __restrict__ w_of, const int32_t* __restrict__ flags) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= n || *flags) return;
  const int32_t a = col_ptr[c], b = col_ptr[c + 1];
  for (int32_t i = a + 1; i < b; ++i) {
    const int32_t rk = row_of[i];
    const double wk = w_of[i];
    int32_t j = i - 1;
    while (j >= a && row_of[j] > rk) {
      row_of[j + 1] = row_of[j];
      w_of[j + 1] = w_of[j];
      --j;
    }
    row_of[j + 1] = rk;
    w_of[j + 1] = wk;
  }
}

// dinv_r * sum_e w_e Z[idx_e, i]: observation r of member i
__device__ inline double obs_rhs_entry(const int32_t* __restrict__ h_ptr, const int32_t* __restrict__ h_idx,
                                       const double* __restrict__ h_w, const double* __restrict__ r_var,
                                       const double* __restrict__ Z, int64_t n, int64_t r, int64_t i) {
  double acc = 0.0;
  for (int32_t e = h_ptr[r]; e < h_ptr[r + 1]; ++e) {
    const int32_t j = h_idx[e];
    if (j >= 0 && j < n) acc += h_w[e] * Z[j + i * n];  // invalid indices are flagged elsewhere
  }
  return acc / sqrt(r_var[r]);
}

// rhs[s * ld + r] = dinv_r * sum_e w_e Z[idx_e, i], i = (s - s0) % N
__global__ void k_obs_rhs(const int32_t* __restrict__ h_ptr, const int32_t* __restrict__ h_idx,
                          const double* __restrict__ h_w, const double* __restrict__ r_var,
                          const double* __restrict__ Z, int64_t n, int64_t N, int64_t m, double* __restrict__ rhs,
                          int64_t ld, int64_t s0, int64_t cnt) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m * cnt) return;
  const int64_t c = t / m, r = t % m;
  rhs[(s0 + c) * ld + r] = obs_rhs_entry(h_ptr, h_idx, h_w, r_var, Z, n, r, c % N);
}

// The same for systems 0 .. cnt-1 over the whole ld x spad block: zeros in the padding rows
// (r >= m) and padding systems (s >= cnt).
__global__ void k_obs_rhs_padded(const int32_t* __restrict__ h_ptr, const int32_t* __restrict__ h_idx,
                                 const double* __restrict__ h_w, const double* __restrict__ r_var,
                                 const double* __restrict__ Z, int64_t n, int64_t N, int64_t m,
                                 double* __restrict__ rhs, int64_t ld, int64_t cnt, int64_t spad) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ld * spad) return;
  const int64_t c = t / ld, r = t % ld;
  rhs[t] = (c < cnt && r < m) ? obs_rhs_entry(h_ptr, h_idx, h_w, r_var, Z, n, r, c % N) : 0.0;
}

__global__ void k_innovation(const int32_t* __restrict__ h_ptr, const int32_t* __restrict__ h_idx,
                             const double* __restrict__ h_w, const double* __restrict__ r_var,
                             const double* __restrict__ y, const double* __restrict__ mu, int64_t m, int64_t n,
                             double* __restrict__ out, int64_t ld, int64_t s) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= m) return;
  double hm = 0.0;
  for (int32_t e = h_ptr[r]; e < h_ptr[r + 1]; ++e) {
    const int32_t j = h_idx[e];
    if (j >= 0 && j < n) hm += h_w[e] * mu[j];
  }
  out[s * ld + r] = (y[r] - hm) / sqrt(r_var[r]);
}

__device__ inline int32_t wrap_offset(int32_t d, int32_t len, int32_t periodic) {
  if (periodic) {
    d = ((d + len / 2) % len + len) % len - len / 2;
  }
  return d;
}

__device__ inline double stencil_value(const Grid& g, int64_t a, int64_t b) {
  const int32_t za = (int32_t)(a / g.nx), xa = (int32_t)(a % g.nx);
  const int32_t zb = (int32_t)(b / g.nx), xb = (int32_t)(b % g.nx);
  const int32_t dz = wrap_offset(zb - za, g.nz, g.pz);
  const int32_t dx = wrap_offset(xb - xa, g.nx, g.px);
  if (dz < -g.bz || dz > g.bz || dx < -g.bx || dx > g.bx) return 0.0;
  return g.table[(dz + g.bz) * (2 * g.bx + 1) + (dx + g.bx)];
}

// diag(S)_r = (1 / r_r) sum_{e,f in row r} h_e h_f L(a_e, a_f) sum_i z_i[a_e] z_i[a_f], the scalar
// beta of the limited-memory preconditioner (Appendix E).  One block per observation: its
// threads share the row's (e, f) pairs, and the row's entries of Z are staged in LDS a chunk
// of members at a time (member-major, so a wave's pairs with consecutive f read consecutive
// words).  Rows longer than the staging buffer read Z from global memory.  Entry indices
// outside [0, n) are skipped (the CSC build flags them).
constexpr int kDiagThreads = 256;
constexpr int kDiagStage = 4096;  // doubles

__global__ __launch_bounds__(kDiagThreads) void k_diag_S(const int32_t* __restrict__ h_ptr,
                                                         const int32_t* __restrict__ h_idx,
                                                         const double* __restrict__ h_w,
                                                         const double* __restrict__ r_var,
                                                         const double* __restrict__ Z, int64_t n, int64_t N,
                                                         Grid g, const double* __restrict__ dense_L,
                                                         double* __restrict__ diagS) {
  __shared__ double zs[kDiagStage];
  __shared__ double part[kDiagThreads / 64];
  const int64_t r = blockIdx.x;
  const int tid = threadIdx.x;
  const int32_t e0 = h_ptr[r];
  const int64_t cnt = h_ptr[r + 1] - e0;
  const bool staged = cnt <= kDiagStage;
  const int64_t nc = staged ? max<int64_t>(1, min<int64_t>(N, kDiagStage / max<int64_t>(cnt, 1))) : N;
  double acc = 0.0;
  for (int64_t i0 = 0; i0 < N; i0 += nc) {
    const int64_t ni = min<int64_t>(nc, N - i0);
    if (staged) {
      __syncthreads();  // the previous chunk's reads are done
      for (int64_t t = tid; t < cnt * ni; t += kDiagThreads) {
        const int64_t i = t / cnt, e = t - i * cnt;
        const int64_t a = h_idx[e0 + e];
        zs[t] = (a >= 0 && a < n) ? Z[a + (i0 + i) * n] : 0.0;
      }
      __syncthreads();
    }
    for (int64_t q = tid; q < cnt * cnt; q += kDiagThreads) {
      const int64_t e = q / cnt, f = q - e * cnt;
      const int64_t a = h_idx[e0 + e], b = h_idx[e0 + f];
      if (a < 0 || a >= n || b < 0 || b >= n) continue;
      const double l = dense_L ? dense_L[a + b * n] : stencil_value(g, a, b);
      if (l == 0.0) continue;
      double zz = 0.0;
      if (staged) {
        for (int64_t i = 0; i < ni; ++i) zz += zs[i * cnt + e] * zs[i * cnt + f];
      } else {
        for (int64_t i = 0; i < N; ++i) zz += Z[a + i * n] * Z[b + i * n];
      }
      acc += h_w[e0 + e] * h_w[e0 + f] * l * zz;
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((tid & 63) == 0) part[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int w = 0; w < kDiagThreads / 64; ++w) tot += part[w];
    diagS[r] = tot / r_var[r];
  }
}

__global__ void k_lattice_members(const int32_t* __restrict__ h_idx, const double* __restrict__ h_w,
                                  const double* __restrict__ r_var, const double* __restrict__ Z, int64_t n,
                                  int64_t N, int64_t m, double* __restrict__ Zt, float* __restrict__ Zt32,
                                  SubTable sub) {
  // one thread per (observation k, member i); the first threads also form the sub-sampled stencil
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (sub.out) {
    const int w = 2 * sub.bxs + 1;
    if (t < (2 * sub.bzs + 1) * w) {
      const int dz = (int)(t / w) - sub.bzs, dx = (int)(t % w) - sub.bxs;
      sub.out[t] = sub.table[(dz * sub.sz + sub.bz) * (2 * sub.bx + 1) + (dx * sub.sx + sub.bx)];
    }
  }
  if (t >= m * N) return;
  const int64_t k = t % m, i = t / m;
  const double sc = h_w[k] / sqrt(r_var[k]);
  int64_t j = h_idx[k];
  if (j < 0 || j >= n) j = 0;  // a wrong lattice claim is flagged by the lattice check
  const double v = sc * Z[j + i * n];
  Zt[k + i * m] = v;
  if (Zt32) Zt32[k + i * m] = (float)v;
}

__global__ void k_subsample_table(const double* __restrict__ table, int32_t bz, int32_t bx, int32_t sz, int32_t sx,
                                  int32_t bzs, int32_t bxs, double* __restrict__ sub) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int w = 2 * bxs + 1;
  if (t >= (2 * bzs + 1) * w) return;
  const int dz = t / w - bzs, dx = t % w - bxs;
  sub[t] = table[(dz * sz + bz) * (2 * bx + 1) + (dx * sx + bx)];
}

__global__ void k_convert_f32(const double* __restrict__ in, float* __restrict__ out, int64_t count) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count) out[t] = (float)in[t];
}

__global__ void k_convert_bf16(const double* __restrict__ in, __hip_bfloat16* __restrict__ out, int64_t count) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count) out[t] = __float2bfloat16((float)in[t]);
}

}  // namespace

hipError_t launch_ens_stats(const double* X, int64_t n, int64_t N, double* mu, double* Z, float* Z32,
                            hipStream_t st) {
  // 64-thread blocks: a 4096-point grid spreads over 64 CUs
  hipLaunchKernelGGL(k_ens_stats, dim3(blocks_for(n, 64)), dim3(64), 0, st, X, n, N, mu, Z, Z32);
  return hipGetLastError();
}

hipError_t launch_csc_count(const int32_t* h_ptr, const int32_t* h_idx, int64_t m, int64_t n, int64_t cap,
                            int32_t* col_cnt, int32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_csc_count, dim3(blocks_for(m)), dim3(kBlock), 0, st, h_ptr, h_idx, m, n, cap, col_cnt,
                     flags);
  return hipGetLastError();
}

hipError_t launch_csc_finish(const int32_t* h_ptr, const int32_t* h_idx, const double* h_w, int64_t m, int64_t n,
                             int32_t* col_cnt, int32_t* col_ptr, int32_t* row_of, double* w_of, int32_t* flags,
                             hipStream_t st) {
  hipError_t e;
  hipLaunchKernelGGL(k_scan_one_block, dim3(1), dim3(kBlock), 0, st, col_cnt, n, col_ptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_fill_i32(col_cnt, 0, n, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_csc_fill, dim3(blocks_for(m)), dim3(kBlock), 0, st, h_ptr, h_idx, h_w, m, col_ptr, col_cnt,
                     row_of, w_of, flags);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_csc_sort, dim3(blocks_for(n)), dim3(kBlock), 0, st, col_ptr, n, row_of, w_of, flags);
  return hipGetLastError();
}

hipError_t launch_obs_rhs_padded(const int32_t* h_ptr, const int32_t* h_idx, const double* h_w, const double* r_var,
                                 const double* Z, int64_t n, int64_t N, int64_t m, double* rhs, int64_t ld,
                                 int64_t cnt, int64_t spad, hipStream_t st) {
  if (ld < m || spad < cnt || N < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_obs_rhs_padded, dim3(blocks_for(ld * spad)), dim3(kBlock), 0, st, h_ptr, h_idx, h_w, r_var, Z,
                     n, N, m, rhs, ld, cnt, spad);
  return hipGetLastError();
}

hipError_t launch_obs_rhs(const int32_t* h_ptr, const int32_t* h_idx, const double* h_w, const double* r_var,
                          const double* Z, int64_t n, int64_t N, int64_t m, double* rhs, int64_t ld, int64_t s0,
                          int64_t cnt, hipStream_t st) {
  hipLaunchKernelGGL(k_obs_rhs, dim3(blocks_for(m * cnt)), dim3(kBlock), 0, st, h_ptr, h_idx, h_w, r_var, Z, n, N,
                     m, rhs, ld, s0, cnt);
  return hipGetLastError();
}

hipError_t launch_innovation(const int32_t* h_ptr, const int32_t* h_idx, const double* h_w, const double* r_var,
                             const double* y, const double* mu, int64_t m, int64_t n, double* out, int64_t ld,
                             int64_t s, hipStream_t st) {
  hipLaunchKernelGGL(k_innovation, dim3(blocks_for(m)), dim3(kBlock), 0, st, h_ptr, h_idx, h_w, r_var, y, mu, m, n,
                     out, ld, s);
  return hipGetLastError();
}

hipError_t launch_diag_S(const int32_t* h_ptr, const int32_t* h_idx, const double* h_w, const double* r_var,
                         const double* Z, int64_t n, int64_t N, int64_t m, const Grid& g, const double* dense_L,
                         double* diagS, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_S, dim3((unsigned)m), dim3(kDiagThreads), 0, st, h_ptr, h_idx, h_w, r_var, Z, n, N, g,
                     dense_L, diagS);
  return hipGetLastError();
}

hipError_t launch_lattice_members(const int32_t* h_idx, const double* h_w, const double* r_var, const double* Z,
                                  int64_t n, int64_t N, int64_t m, double* Zt, float* Zt32, hipStream_t st,
                                  const SubTable& sub) {
  const int64_t cnt = sub.out ? (int64_t)(2 * sub.bzs + 1) * (2 * sub.bxs + 1) : 0;
  hipLaunchKernelGGL(k_lattice_members, dim3(blocks_for(std::max<int64_t>(m * N, cnt))), dim3(kBlock), 0, st, h_idx,
                     h_w, r_var, Z, n, N, m, Zt, Zt32, sub);
  return hipGetLastError();
}

hipError_t launch_subsample_table(const double* table, int32_t bz, int32_t bx, int32_t sz, int32_t sx, int32_t bzs,
                                  int32_t bxs, double* sub, hipStream_t st) {
  const int cnt = (2 * bzs + 1) * (2 * bxs + 1);
  hipLaunchKernelGGL(k_subsample_table, dim3(blocks_for(cnt)), dim3(kBlock), 0, st, table, bz, bx, sz, sx, bzs, bxs,
                     sub);
  return hipGetLastError();
}

hipError_t launch_convert_f32(const double* in, float* out, int64_t count, hipStream_t st) {
  if (count > 0 && (!in || !out)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_convert_f32, dim3(blocks_for(count)), dim3(kBlock), 0, st, in, out, count);
  return hipGetLastError();
}

hipError_t launch_convert_bf16(const double* in, __hip_bfloat16* out, int64_t count, hipStream_t st) {
  if (count > 0 && (!in || !out)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_convert_bf16, dim3(blocks_for(count)), dim3(kBlock), 0, st, in, out, count);
  return hipGetLastError();
}

}  // namespace infoesrf
