// Batched preconditioned conjugate gradients (Golub & Van Loan Alg. 11.5.1) with the
// limited-memory Ritz preconditioner of Appendix E, plus the observation-space glue
// around the covariance apply.
//
// Layout: every observation-space vector family (x, r, p, q, b) is an m x S
// matrix stored "system-fastest": element (row r, system s) at r*ld + s, so a
// wavefront touches 64 consecutive systems of one row.  Reductions over rows
// are split into chunks of `chunk_rows`; each (chunk, system) partial is
// written once and every consumer re-reduces the partials of a system in the
// same fixed order, so results are bit-reproducible run to run.
//
// Per iteration (systems listed in `act`, count `*nact`):
//   apply:      q = C p = (1+sigma) p + S p, partials of p^T q
//   step:       alpha = r^T z / p^T q; x += alpha p; r -= alpha q; partials of
//               r^T r, Phi^T r, (S Phi)^T r
//   direction:  convergence test, z = P^{-1} r from those dots alone
//               (no further pass over r), r^T z, p = z + beta p.
#include "internal.hpp"

namespace infoesrf {

namespace {

constexpr int kSys = 64;    // systems per block
constexpr int kLanes = 4;   // row lanes per block (256 threads)

__device__ inline int32_t load_nact(const int32_t* nact, int64_t fallback) {
  return nact ? *nact : (int32_t)fallback;
}

// --------------------------------------------------------------- apply glue

template <typename TV>
__device__ inline TV to_prec(double v);
template <>
__device__ inline double to_prec<double>(double v) { return v; }
template <>
__device__ inline float to_prec<float>(double v) { return (float)v; }

template <typename TV>
__global__ void k_gather_active(const double* __restrict__ P, int64_t ldp, const int32_t* __restrict__ act,
                                const int32_t* __restrict__ nact, int64_t rows, int64_t Bpad,
                                TV* __restrict__ V, int64_t ldv) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= rows * Bpad) return;
  const int64_t r = t / Bpad, c = t % Bpad;
  const int32_t na = load_nact(nact, Bpad);
  V[r * ldv + c] = (c < na) ? to_prec<TV>(P[r * ldp + act[c]]) : TV(0);
}

template <typename TV>
__global__ void k_scatter_state(const double* __restrict__ P, int64_t ldp, const int32_t* __restrict__ act,
                                const int32_t* __restrict__ nact, const int32_t* __restrict__ col_ptr,
                                const int32_t* __restrict__ row_of, const double* __restrict__ w_of,
                                const double* __restrict__ r_var, int64_t n, int64_t m, int64_t Bpad,
                                TV* __restrict__ V, int64_t ldv) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * Bpad) return;
  const int64_t k = t / Bpad, c = t % Bpad;
  const int32_t na = load_nact(nact, Bpad);
  double acc = 0.0;
  if (c < na) {
    const int32_t s = act[c];
    for (int32_t e = col_ptr[k]; e < col_ptr[k + 1]; ++e) {
      const int32_t r = row_of[e];
      if (r >= 0 && r < m) acc += w_of[e] / sqrt(r_var[r]) * P[r * ldp + s];
    }
  }
  V[k * ldv + c] = to_prec<TV>(acc);
}

// q = (1 + sigma_s) p + S p, with S p = T (obs domain) or R^{-1/2} H T (state domain); partial p^T q.
template <typename TT>
__global__ __launch_bounds__(256) void k_apply_finish(int obs_domain, const double* __restrict__ P, int64_t ldp,
                                                      const TT* __restrict__ T, int64_t ldt,
                                                      const int32_t* __restrict__ act,
                                                      const int32_t* __restrict__ nact,
                                                      const double* __restrict__ sigma,
                                                      const int32_t* __restrict__ h_ptr,
                                                      const int32_t* __restrict__ h_idx,
                                                      const double* __restrict__ h_w,
                                                      const double* __restrict__ r_var, int64_t m,
                                                      int64_t n_state, int64_t Bpad, double* __restrict__ Qv,
                                                      double* __restrict__ part, int chunk_rows) {
  __shared__ double red[kLanes][kSys];
  const int cl = threadIdx.x % kSys, lane_r = threadIdx.x / kSys;
  const int64_t c = blockIdx.y * (int64_t)kSys + cl;
  const int32_t na = load_nact(nact, Bpad);
  const int64_t r0 = blockIdx.x * (int64_t)chunk_rows;
  const int64_t r1 = min<int64_t>(m, r0 + chunk_rows);
  double dot = 0.0;
  if (c < na) {
    const int32_t s = act[c];
    const double coef = 1.0 + sigma[s];
    for (int64_t r = r0 + lane_r; r < r1; r += kLanes) {
      double sp;
      if (obs_domain) {
        sp = (double)T[r * ldt + c];
      } else {
        double a = 0.0;
        for (int32_t e = h_ptr[r]; e < h_ptr[r + 1]; ++e) {
          const int32_t j = h_idx[e];
          if (j >= 0 && j < n_state) a += h_w[e] * (double)T[(int64_t)j * ldt + c];
        }
        sp = a / sqrt(r_var[r]);
      }
      const double pv = P[r * ldp + s];
      const double qv = coef * pv + sp;
      Qv[r * ldp + s] = qv;
      dot += pv * qv;
    }
  }
  red[lane_r][cl] = dot;
  __syncthreads();
  if (lane_r == 0 && c < na) {
    double s = red[0][cl];
    for (int j = 1; j < kLanes; ++j) s += red[j][cl];
    part[blockIdx.x * Bpad + c] = s;
  }
}

// --------------------------------------------------------------- PCG kernels

// Accumulate r^T r, Phi^T r, (S Phi)^T r of the rows of this block's chunk for system s.
template <int P>
__device__ inline void chunk_dots(const PCGState& st, const LMP& lmp, int32_t s, int64_t r0, int64_t r1, int lane_r,
                                  double* acc) {
#pragma unroll
  for (int j = 0; j < 2 * P + 1; ++j) acc[j] = 0.0;
  for (int64_t r = r0 + lane_r; r < r1; r += kLanes) {
    const double rv = st.r[r * st.ld + s];
    acc[0] += rv * rv;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      acc[1 + j] += lmp.Phi[r * P + j] * rv;
      acc[1 + P + j] += lmp.SPhi[r * P + j] * rv;
    }
  }
}

template <int P>
__device__ inline void reduce_store(double* acc, double (*red)[kSys], int cl, int lane_r, bool ok, double* part2,
                                    int64_t base) {
  // red: [kLanes][kSys] reused per component (fixed order)
  for (int j = 0; j < 2 * P + 1; ++j) {
    red[lane_r][cl] = acc[j];
    __syncthreads();
    if (lane_r == 0 && ok) {
      double s = red[0][cl];
      for (int t = 1; t < kLanes; ++t) s += red[t][cl];
      part2[base * (2 * P + 1) + j] = s;
    }
    __syncthreads();
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_pcg_dots(PCGState st, LMP lmp, const int32_t* __restrict__ act,
                                                  const int32_t* __restrict__ nact, int64_t Bpad,
                                                  double* __restrict__ part2) {
  __shared__ double red[kLanes][kSys];
  const int cl = threadIdx.x % kSys, lane_r = threadIdx.x / kSys;
  const int64_t c = blockIdx.y * (int64_t)kSys + cl;
  const int32_t na = load_nact(nact, Bpad);
  const int64_t r0 = blockIdx.x * (int64_t)st.chunk_rows;
  const int64_t r1 = min<int64_t>(st.m, r0 + st.chunk_rows);
  double acc[2 * P + 1];
  bool ok = false;
  if (c < na) {
    const int32_t s = act[c];
    ok = (st.done[s] == 0);
    if (ok) {
      chunk_dots<P>(st, lmp, s, r0, r1, lane_r, acc);
    }
  }
  if (!ok) {
#pragma unroll
    for (int j = 0; j < 2 * P + 1; ++j) acc[j] = 0.0;
  }
  reduce_store<P>(acc, red, cl, lane_r, ok, part2, blockIdx.x * Bpad + c);
}

template <int P>
__global__ __launch_bounds__(256) void k_pcg_step(PCGState st, LMP lmp, const int32_t* __restrict__ act,
                                                  const int32_t* __restrict__ nact, int64_t Bpad,
                                                  const double* __restrict__ part_pq, double* __restrict__ part2) {
  __shared__ double red[kLanes][kSys];
  const int cl = threadIdx.x % kSys, lane_r = threadIdx.x / kSys;
  const int64_t c = blockIdx.y * (int64_t)kSys + cl;
  const int32_t na = load_nact(nact, Bpad);
  const int64_t r0 = blockIdx.x * (int64_t)st.chunk_rows;
  const int64_t r1 = min<int64_t>(st.m, r0 + st.chunk_rows);
  double acc[2 * P + 1];
  bool ok = false;
  if (c < na) {
    const int32_t s = act[c];
    ok = (st.done[s] == 0);
    if (ok) {
      double pq = 0.0;
      for (int k = 0; k < st.nchunks; ++k) pq += part_pq[k * Bpad + c];
      const double rz = st.rz[s];
      if (!(pq > 0.0) || !isfinite(pq)) {
        // curvature breakdown: every chunk of this system sees the same pq and stops; the
        // first chunk retires the system and raises the flag
        if (blockIdx.x == 0 && lane_r == 0) {
          atomicOr(st.flags, isfinite(pq) ? kFlagNotSPD : kFlagNumeric);
          st.done[s] = 2;
        }
        ok = false;
      } else {
        const double alpha = rz / pq;
        for (int64_t r = r0 + lane_r; r < r1; r += kLanes) {
          const int64_t e = r * st.ld + s;
          st.x[e] += alpha * st.p[e];
          st.r[e] -= alpha * st.q[e];
        }
        chunk_dots<P>(st, lmp, s, r0, r1, lane_r, acc);
      }
    }
  }
  if (!ok) {
#pragma unroll
    for (int j = 0; j < 2 * P + 1; ++j) acc[j] = 0.0;
  }
  reduce_store<P>(acc, red, cl, lane_r, ok, part2, blockIdx.x * Bpad + c);
}

template <int P>
__global__ __launch_bounds__(256) void k_pcg_direction(PCGState st, LMP lmp, const int32_t* __restrict__ act,
                                                       const int32_t* __restrict__ nact, int64_t Bpad,
                                                       const double* __restrict__ part2, double tol_rel, int first,
                                                       int max_iter, const double* __restrict__ rz_cur,
                                                       double* __restrict__ rz_next) {
  const int cl = threadIdx.x % kSys, lane_r = threadIdx.x / kSys;
  const int64_t c = blockIdx.y * (int64_t)kSys + cl;
  const int32_t na = load_nact(nact, Bpad);
  if (c >= na) return;
  const int32_t s = act[c];
  if (st.done[s] != 0) return;
  const bool writer = (blockIdx.x == 0 && lane_r == 0);
  // reduce the dots of r over chunks (fixed order)
  double d[2 * P + 1];
#pragma unroll
  for (int j = 0; j < 2 * P + 1; ++j) d[j] = 0.0;
  for (int k = 0; k < st.nchunks; ++k) {
    const double* src = part2 + (k * Bpad + c) * (2 * P + 1);
#pragma unroll
    for (int j = 0; j < 2 * P + 1; ++j) d[j] += src[j];
  }
  const double rr = d[0];
  const double rn = sqrt(rr);
  const double bn = st.bnorm[s];
  const int it = st.iters[s] + (first ? 0 : 1);
  if (!isfinite(rr)) {
    if (writer) {
      atomicOr(st.flags, kFlagNumeric);
      st.done[s] = 2;
      st.iters[s] = it;
    }
    return;
  }
  if (rn <= tol_rel * bn) {
    if (writer) {
      st.done[s] = 1;
      st.iters[s] = it;
      st.relres[s] = bn > 0.0 ? rn / bn : 0.0;
    }
    return;
  }
  const double sig1 = 1.0 + st.sigma[s];
  double c1[P > 0 ? P : 1], gam[P > 0 ? P : 1];
  double rz = rr;
  if (P > 0) {
    const double beta_l = sig1 + *lmp.dmin;
    const double* Gpp = lmp.G;
    const double* Gps = lmp.G + P * P;
    const double* Gss = lmp.G + 2 * P * P;
#pragma unroll
    for (int j = 0; j < P; ++j) c1[j] = d[1 + j] / (sig1 + lmp.theta[j]);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      // (C Phi)^T (C Phi) = Gss + sig1 (Gps + Gps^T) + sig1^2 Gpp
      double mc = 0.0;
#pragma unroll
      for (int l = 0; l < P; ++l)
        mc += (Gss[j * P + l] + sig1 * (Gps[j * P + l] + Gps[l * P + j]) + sig1 * sig1 * Gpp[j * P + l]) * c1[l];
      const double c2 = (d[1 + P + j] + sig1 * d[1 + j] - mc) / (sig1 + lmp.theta[j]);
      gam[j] = (sig1 - beta_l) * c1[j] + c2;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) rz -= d[1 + P + j] * c1[j] + d[1 + j] * gam[j];
  }
  const double beta = first ? 0.0 : rz / rz_cur[s];
  const int64_t r0 = blockIdx.x * (int64_t)st.chunk_rows;
  const int64_t r1 = min<int64_t>(st.m, r0 + st.chunk_rows);
  for (int64_t r = r0 + lane_r; r < r1; r += kLanes) {
    const int64_t e = r * st.ld + s;
    double z = st.r[e];
#pragma unroll
    for (int j = 0; j < P; ++j) z -= lmp.SPhi[r * P + j] * c1[j] + lmp.Phi[r * P + j] * gam[j];
    st.p[e] = first ? z : z + beta * st.p[e];
  }
  if (writer) {
    rz_next[s] = rz;
    st.iters[s] = it;
    st.relres[s] = bn > 0.0 ? rn / bn : 0.0;
    if (!(rz > 0.0)) atomicOr(st.flags, isfinite(rz) ? kFlagNotSPD : kFlagNumeric);
    if (it >= max_iter) st.done[s] = 2;
  }
}

__global__ void k_compact(const int32_t* __restrict__ done, int64_t S, int32_t* __restrict__ act,
                          int32_t* __restrict__ nact) {
  __shared__ int32_t cnt[256];
  const int t = threadIdx.x;
  const int64_t per = (S + 255) / 256;
  const int64_t a = t * per, b = min<int64_t>(S, a + per);
  int32_t c = 0;
  for (int64_t s = a; s < b; ++s) c += (done[s] == 0);
  cnt[t] = c;
  __syncthreads();
  if (t == 0) {
    int32_t run = 0;
    for (int i = 0; i < 256; ++i) {
      const int32_t v = cnt[i];
      cnt[i] = run;
      run += v;
    }
    *nact = run;
  }
  __syncthreads();
  int32_t pos = cnt[t];
  for (int64_t s = a; s < b; ++s)
    if (done[s] == 0) act[pos++] = (int32_t)s;
}

__global__ void k_iota(int32_t* __restrict__ act, int32_t* __restrict__ nact, int64_t S) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < S) act[t] = (int32_t)t;
  if (t == 0) *nact = (int32_t)S;
}

// --------------------------------------------------------------- misc
__global__ void k_fill_f64(double* p, double v, int64_t count) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count) p[t] = v;
}
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t count) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count) p[t] = v;
}
__global__ void k_sub(const double* a, const double* b, double* out, int64_t m, int64_t S, int64_t ld) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m * S) return;
  const int64_t e = (t / S) * ld + t % S;
  out[e] = a[e] - b[e];
}
__global__ void k_axpy(double* x, const double* d, int64_t m, int64_t S, int64_t ld) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m * S) return;
  const int64_t e = (t / S) * ld + t % S;
  x[e] += d[e];
}
// per-system 2-norm, one block of 256 per 64 systems; fixed order
__global__ void k_col_norms(const double* __restrict__ v, int64_t m, int64_t S, int64_t ld, double* __restrict__ out) {
  __shared__ double red[kLanes][kSys];
  const int cl = threadIdx.x % kSys, lane_r = threadIdx.x / kSys;
  const int64_t s = blockIdx.x * (int64_t)kSys + cl;
  double acc = 0.0;
  if (s < S)
    for (int64_t r = lane_r; r < m; r += kLanes) {
      const double x = v[r * ld + s];
      acc += x * x;
    }
  red[lane_r][cl] = acc;
  __syncthreads();
  if (lane_r == 0 && s < S) {
    double t = red[0][cl];
    for (int j = 1; j < kLanes; ++j) t += red[j][cl];
    out[s] = sqrt(t);
  }
}
__global__ void k_residual_status(const double* rn, const double* bn, double tol, double* relres, int32_t* done,
                                  int64_t S, int32_t* flags) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= S) return;
  const double rr = bn[s] > 0.0 ? rn[s] / bn[s] : 0.0;
  relres[s] = rr;
  if (!isfinite(rr)) {
    atomicOr(flags, kFlagNumeric);
    done[s] = 2;
    return;
  }
  done[s] = (rr <= tol) ? 1 : 0;
}
__global__ void k_quad_combine(const double* __restrict__ u, int64_t ldu, int64_t m, int64_t N, int32_t Q,
                               const double* __restrict__ pw, double* __restrict__ ubar, int64_t ldb, int64_t s0) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m * N) return;
  const int64_t r = t / N, i = t % N;
  double acc = 0.0;
  for (int32_t q = 0; q < Q; ++q) acc += pw[q] * u[r * ldu + s0 + q * N + i];
  ubar[r * ldb + i] = acc;
}
__global__ void k_final_pert(const double* __restrict__ Z, const double* __restrict__ T, int64_t ldt, int64_t n,
                             int64_t N, double scale, double* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * N) return;
  const int64_t k = t % n, i = t / n;
  out[k + i * n] = scale * (Z[k + i * n] - T[k * ldt + i]);
}
__global__ void k_final_mean(const double* __restrict__ mu, const double* __restrict__ T, int64_t ldt, int64_t n,
                             int64_t col, double* __restrict__ out) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) out[k] = mu[k] + T[k * ldt + col];
}
__global__ void k_to_sysfast(const double* __restrict__ V, int64_t ldv, int64_t n, int64_t B,
                             double* __restrict__ out, int64_t ldo) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * ldo) return;
  const int64_t k = t / ldo, b = t % ldo;
  out[k * ldo + b] = (b < B) ? V[k + b * ldv] : 0.0;
}
__global__ void k_from_sysfast(const double* __restrict__ in, int64_t ldi, int64_t n, int64_t B,
                               double* __restrict__ out, int64_t ldo) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * B) return;
  const int64_t k = t % n, b = t / n;
  out[k + b * ldo] = in[k * ldi + b];
}
__global__ void k_export_stats(const int32_t* iters, const double* relres, const int32_t* done, int64_t S,
                               int32_t* oi, double* orr, uint8_t* oc, double tol) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= S) return;
  if (oi) oi[s] = iters[s];
  if (orr) orr[s] = relres[s];
  if (oc) oc[s] = (done[s] == 1 && relres[s] <= tol) ? 1 : 0;
}
__global__ void k_nan_check(const double* v, int64_t count, int32_t* flags) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count && !isfinite(v[t])) atomicOr(flags, kFlagNumeric);
}

inline unsigned nb(int64_t count) { return (unsigned)((count + 255) / 256); }

template <int P>
hipError_t dispatch_dots(const PCGState& s, const LMP& lmp, const int32_t* act, const int32_t* nact, int64_t Bpad,
                         double* part2, hipStream_t st) {
  dim3 grid(s.nchunks, (unsigned)((Bpad + kSys - 1) / kSys));
  hipLaunchKernelGGL(k_pcg_dots<P>, grid, dim3(256), 0, st, s, lmp, act, nact, Bpad, part2);
  return hipGetLastError();
}
template <int P>
hipError_t dispatch_step(const PCGState& s, const LMP& lmp, const int32_t* act, const int32_t* nact, int64_t Bpad,
                         const double* part_pq, double* part2, hipStream_t st) {
  dim3 grid(s.nchunks, (unsigned)((Bpad + kSys - 1) / kSys));
  hipLaunchKernelGGL(k_pcg_step<P>, grid, dim3(256), 0, st, s, lmp, act, nact, Bpad, part_pq, part2);
  return hipGetLastError();
}
template <int P>
hipError_t dispatch_dir(const PCGState& s, const LMP& lmp, const int32_t* act, const int32_t* nact, int64_t Bpad,
                        const double* part2, double tol, int first, int max_iter, const double* rz_cur,
                        double* rz_next, hipStream_t st) {
  dim3 grid(s.nchunks, (unsigned)((Bpad + kSys - 1) / kSys));
  hipLaunchKernelGGL(k_pcg_direction<P>, grid, dim3(256), 0, st, s, lmp, act, nact, Bpad, part2, tol, first,
                     max_iter, rz_cur, rz_next);
  return hipGetLastError();
}

#define IE_P_SWITCH(p, CALL)         \
  switch (p) {                       \
    case 0: return CALL(0);          \
    case 4: return CALL(4);          \
    case 8: return CALL(8);          \
    case 10: return CALL(10);        \
    case 12: return CALL(12);        \
    case 16: return CALL(16);        \
    default: return hipErrorInvalidValue; \
  }

}  // namespace

hipError_t launch_gather_active(Prec prec, const double* P, int64_t ldp, const int32_t* act, const int32_t* nact,
                                int64_t rows, int64_t Bpad, void* V, int64_t ldv, hipStream_t st) {
  if (prec == Prec::F64)
    hipLaunchKernelGGL(k_gather_active<double>, dim3(nb(rows * Bpad)), dim3(256), 0, st, P, ldp, act, nact, rows,
                       Bpad, (double*)V, ldv);
  else
    hipLaunchKernelGGL(k_gather_active<float>, dim3(nb(rows * Bpad)), dim3(256), 0, st, P, ldp, act, nact, rows,
                       Bpad, (float*)V, ldv);
  return hipGetLastError();
}

hipError_t launch_scatter_state(Prec prec, const double* P, int64_t ldp, const int32_t* act, const int32_t* nact,
                                const int32_t* col_ptr, const int32_t* row_of, const double* w_of,
                                const double* r_var, int64_t n, int64_t m, int64_t Bpad, void* V, int64_t ldv,
                                hipStream_t st) {
  if (prec == Prec::F64)
    hipLaunchKernelGGL(k_scatter_state<double>, dim3(nb(n * Bpad)), dim3(256), 0, st, P, ldp, act, nact, col_ptr,
                       row_of, w_of, r_var, n, m, Bpad, (double*)V, ldv);
  else
    hipLaunchKernelGGL(k_scatter_state<float>, dim3(nb(n * Bpad)), dim3(256), 0, st, P, ldp, act, nact, col_ptr,
                       row_of, w_of, r_var, n, m, Bpad, (float*)V, ldv);
  return hipGetLastError();
}

hipError_t launch_apply_finish(Prec prec, int obs_domain, const double* P, int64_t ldp, const void* T, int64_t ldt,
                               const int32_t* act, const int32_t* nact, const double* sigma, const int32_t* h_ptr,
                               const int32_t* h_idx, const double* h_w, const double* r_var, int64_t m,
                               int64_t n_state, int64_t Bpad, double* Qv, double* part, int chunk_rows,
                               hipStream_t st) {
  const int nchunks = (int)((m + chunk_rows - 1) / chunk_rows);
  dim3 grid(nchunks, (unsigned)((Bpad + kSys - 1) / kSys));
  if (prec == Prec::F64)
    hipLaunchKernelGGL(k_apply_finish<double>, grid, dim3(256), 0, st, obs_domain, P, ldp, (const double*)T, ldt,
                       act, nact, sigma, h_ptr, h_idx, h_w, r_var, m, n_state, Bpad, Qv, part, chunk_rows);
  else
    hipLaunchKernelGGL(k_apply_finish<float>, grid, dim3(256), 0, st, obs_domain, P, ldp, (const float*)T, ldt, act,
                       nact, sigma, h_ptr, h_idx, h_w, r_var, m, n_state, Bpad, Qv, part, chunk_rows);
  return hipGetLastError();
}

hipError_t launch_pcg_dots(const PCGState& s, const LMP& lmp, const int32_t* act, const int32_t* nact, int64_t Bpad,
                           double* part2, hipStream_t st) {
#define IE_CALL(P) dispatch_dots<P>(s, lmp, act, nact, Bpad, part2, st)
  IE_P_SWITCH(lmp.p, IE_CALL)
#undef IE_CALL
}

hipError_t launch_pcg_step(const PCGState& s, const LMP& lmp, const int32_t* act, const int32_t* nact, int64_t Bpad,
                           const double* part_pq, double* part2, hipStream_t st) {
#define IE_CALL(P) dispatch_step<P>(s, lmp, act, nact, Bpad, part_pq, part2, st)
  IE_P_SWITCH(lmp.p, IE_CALL)
#undef IE_CALL
}

hipError_t launch_pcg_direction(const PCGState& s, const LMP& lmp, const int32_t* act, const int32_t* nact,
                                int64_t Bpad, const double* part2, double tol_rel, int first, int max_iter,
                                const double* rz_cur, double* rz_next, hipStream_t st) {
#define IE_CALL(P) dispatch_dir<P>(s, lmp, act, nact, Bpad, part2, tol_rel, first, max_iter, rz_cur, rz_next, st)
  IE_P_SWITCH(lmp.p, IE_CALL)
#undef IE_CALL
}

hipError_t launch_compact(const int32_t* done, int64_t S, int32_t* act, int32_t* nact, hipStream_t st) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(256), 0, st, done, S, act, nact);
  return hipGetLastError();
}
hipError_t launch_iota(int32_t* act, int32_t* nact, int64_t S, hipStream_t st) {
  hipLaunchKernelGGL(k_iota, dim3(nb(S > 0 ? S : 1)), dim3(256), 0, st, act, nact, S);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3(nb(count)), dim3(256), 0, st, p, v, count);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(nb(count)), dim3(256), 0, st, p, v, count);
  return hipGetLastError();
}
hipError_t launch_sub(const double* a, const double* b, double* out, int64_t m, int64_t S, int64_t ld,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_sub, dim3(nb(m * S)), dim3(256), 0, st, a, b, out, m, S, ld);
  return hipGetLastError();
}
hipError_t launch_axpy_masked(double* x, const double* d, int64_t m, int64_t S, int64_t ld, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(nb(m * S)), dim3(256), 0, st, x, d, m, S, ld);
  return hipGetLastError();
}
hipError_t launch_col_norms(const double* v, int64_t m, int64_t S, int64_t ld, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_col_norms, dim3((unsigned)((S + kSys - 1) / kSys)), dim3(256), 0, st, v, m, S, ld, out);
  return hipGetLastError();
}
hipError_t launch_residual_status(const double* rn, const double* bn, double tol, double* relres, int32_t* done,
                                  int64_t S, int32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_residual_status, dim3(nb(S)), dim3(256), 0, st, rn, bn, tol, relres, done, S, flags);
  return hipGetLastError();
}
hipError_t launch_quad_combine(const double* u, int64_t ldu, int64_t m, int64_t N, int32_t Q, const double* pw,
                               double* ubar, int64_t ldb, int64_t s0, hipStream_t st) {
  hipLaunchKernelGGL(k_quad_combine, dim3(nb(m * N)), dim3(256), 0, st, u, ldu, m, N, Q, pw, ubar, ldb, s0);
  return hipGetLastError();
}
hipError_t launch_final_pert(const double* Z, const double* T, int64_t ldt, int64_t n, int64_t N, double scale,
                             double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_final_pert, dim3(nb(n * N)), dim3(256), 0, st, Z, T, ldt, n, N, scale, out);
  return hipGetLastError();
}
hipError_t launch_final_mean(const double* mu, const double* T, int64_t ldt, int64_t n, int64_t col, double* out,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_final_mean, dim3(nb(n)), dim3(256), 0, st, mu, T, ldt, n, col, out);
  return hipGetLastError();
}
hipError_t launch_to_sysfast(const double* V, int64_t ldv, int64_t n, int64_t B, double* out, int64_t ldo,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_to_sysfast, dim3(nb(n * ldo)), dim3(256), 0, st, V, ldv, n, B, out, ldo);
  return hipGetLastError();
}
hipError_t launch_from_sysfast(const double* in, int64_t ldi, int64_t n, int64_t B, double* out, int64_t ldo,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_from_sysfast, dim3(nb(n * B)), dim3(256), 0, st, in, ldi, n, B, out, ldo);
  return hipGetLastError();
}
hipError_t launch_export_stats(const int32_t* iters, const double* relres, const int32_t* done, int64_t S,
                               int32_t* out_iters, double* out_relres, uint8_t* out_conv, double tol,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_export_stats, dim3(nb(S)), dim3(256), 0, st, iters, relres, done, S, out_iters, out_relres,
                     out_conv, tol);
  return hipGetLastError();
}
hipError_t launch_nan_check(const double* v, int64_t count, int32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_nan_check, dim3(nb(count)), dim3(256), 0, st, v, count, flags);
  return hipGetLastError();
}

}  // namespace infoesrf
