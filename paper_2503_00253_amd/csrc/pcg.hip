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

// Block arrival count of a column tile; true in the last block to arrive (which resets the counter).
// One agent-scope release per block (thread 0, after the block's barrier) and one acquire in the
// last block: on gfx950 each agent-scope fence is an L2 writeback/invalidate, because the L2s of
// the eight XCDs are not coherent with each other, so fences are kept to one per block.
__device__ inline bool last_arrival_apply(int32_t* cnt, int total, int* s_flag) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const int prev = atomicAdd(cnt, 1);
    const int last = (prev == total - 1);
    if (last) {
      atomicExch(cnt, 0);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    *s_flag = last;
  }
  __syncthreads();
  return *s_flag != 0;
}

template <typename TV>
__device__ inline TV to_prec(double v);
template <>
__device__ inline double to_prec<double>(double v) { return v; }
template <>
__device__ inline float to_prec<float>(double v) { return (float)v; }
template <>
__device__ inline __hip_bfloat16 to_prec<__hip_bfloat16>(double v) { return __float2bfloat16((float)v); }

// Index of (row r, column c) in an apply buffer: system-fastest (FP64/FP32 applies) or
// system-major (BF16 applies, column c contiguous in r).
template <typename TV>
__device__ inline int64_t vidx(int64_t r, int64_t c, int64_t ld) {
  return r * ld + c;
}
template <>
__device__ inline int64_t vidx<__hip_bfloat16>(int64_t r, int64_t c, int64_t ld) {
  return c * ld + r;
}

template <typename TV>
__global__ void k_gather_active(const double* __restrict__ P, int64_t ldp, const int32_t* __restrict__ act,
                                const int32_t* __restrict__ nact, int64_t rows, int64_t Bpad,
                                TV* __restrict__ V, int64_t ldv) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= rows * Bpad) return;
  const int64_t r = t / Bpad, c = t % Bpad;
  const int32_t na = load_nact(nact, Bpad);
  V[vidx<TV>(r, c, ldv)] = to_prec<TV>((c < na) ? P[r * ldp + act[c]] : 0.0);
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
  V[vidx<TV>(k, c, ldv)] = to_prec<TV>(acc);
}

// q = (1 + sigma_s) p + S p, with S p = T (obs domain) or R^{-1/2} H T (state domain); partial p^T q.
// With an AlphaOut, the last block of each column tile also forms alpha_s = rz_s / p^T q
// (and retires systems whose curvature is not positive).
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
                                                      double* __restrict__ part, int chunk_rows, AlphaOut ao) {
  __shared__ double red[16][16];
  __shared__ int s_flag;
  const int cl = threadIdx.x % 16, lane_r = threadIdx.x / 16;
  const int64_t c = blockIdx.y * (int64_t)16 + cl;
  const int32_t na = load_nact(nact, Bpad);
  const int64_t r0 = blockIdx.x * (int64_t)chunk_rows;
  const int64_t r1 = min<int64_t>(m, r0 + chunk_rows);
  double dot = 0.0;
  if (c < na) {
    const int32_t s = act[c];
    const double coef = 1.0 + sigma[s];
    for (int64_t r = r0 + lane_r; r < r1; r += 16) {
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
    double t = red[0][cl];
    for (int j = 1; j < 16; ++j) t += red[j][cl];
    part[blockIdx.x * Bpad + c] = t;
  }
  if (!ao.alpha) return;
  if (!last_arrival_apply(ao.tile_cnt + blockIdx.y, gridDim.x, &s_flag)) return;
  if (threadIdx.x < 16 && c < na) {
    const int32_t s = act[c];
    if (ao.done[s] == 0) {
      double pq = 0.0;
      for (int k = 0; k < (int)gridDim.x; ++k) pq += part[k * Bpad + c];  // after the fence of last_arrival
      if (!(pq > 0.0) || !isfinite(pq)) {
        atomicOr(ao.flags, isfinite(pq) ? kFlagNotSPD : kFlagNumeric);
        ao.done[s] = 2;
        ao.alpha[s] = 0.0;
      } else {
        ao.alpha[s] = ao.rz[s] / pq;
      }
    }
  }
}

// --------------------------------------------------------------- PCG kernels
//
// Thread layout of the reduction kernels: a block holds 16 systems (columns of
// the active list) x 16 row lanes and covers `chunk_rows` rows.  Partial sums
// of a (chunk, system) are written once; the last block of each column tile to
// finish (counted with a device-scope atomic after a fence) reduces the
// partials of its 16 systems over all chunks in chunk order.  No block waits
// for another, and the summation order is fixed.

constexpr int kCS = 16;   // systems per block
constexpr int kRL = 16;   // row lanes per block

// Values written by other blocks of the same kernel are read only after last_arrival(), whose
// agent-scope acquire invalidates this CU's L1 and the XCD's L2 lines, so plain loads see them.
__device__ inline double vload(const double* p) { return *p; }
__device__ inline int32_t vload_i32(const int32_t* p) { return *p; }

__device__ inline bool last_arrival(int32_t* cnt, int total, int* s_flag) {
  return last_arrival_apply(cnt, total, s_flag);
}

// LMP coefficients of one system from the dots of r (Appendix E preconditioner):
//   c1 = Theta^{-1} Phi^T r, c2 = Theta^{-1} [(C Phi)^T r - (C Phi)^T (C Phi) c1],
//   z = r - S Phi c1 - Phi gamma, gamma = (1 + sigma - beta_L) c1 + c2, r^T z.
template <int P>
__device__ inline double lmp_coefficients(const LMP& lmp, double sig1, const double* d, double* c1, double* gam) {
  double rz = d[0];
  if (P == 0) return rz;
  const double beta_l = sig1 + *lmp.dmin;
  const double* Gpp = lmp.G;
  const double* Gps = lmp.G + P * P;
  const double* Gss = lmp.G + 2 * P * P;
  for (int j = 0; j < P; ++j) c1[j] = d[1 + j] / (sig1 + lmp.theta[j]);
  for (int j = 0; j < P; ++j) {
    double mc = 0.0;
    for (int l = 0; l < P; ++l)
      mc += (Gss[j * P + l] + sig1 * (Gps[j * P + l] + Gps[l * P + j]) + sig1 * sig1 * Gpp[j * P + l]) * c1[l];
    const double c2 = (d[1 + P + j] + sig1 * d[1 + j] - mc) / (sig1 + lmp.theta[j]);
    gam[j] = (sig1 - beta_l) * c1[j] + c2;
  }
  for (int j = 0; j < P; ++j) rz -= d[1 + P + j] * c1[j] + d[1 + j] * gam[j];
  return rz;
}

// mode 0: dots of r only (start of a solve); mode 1: alpha step on x and r, then dots.
// The last block per column tile turns the dots into per-system coefficients
// (coef[s*W + 0..P) = c1, [P..2P) = gamma, [2P] = beta), the convergence status and
// r^T z; the last of those blocks writes the next active list (act_out, nact_out).
template <int P>
__global__ __launch_bounds__(256) void k_pcg_step(PCGState st, LMP lmp, int mode, const int32_t* __restrict__ act,
                                                  const int32_t* __restrict__ nact, int32_t* __restrict__ act_out,
                                                  int32_t* __restrict__ nact_out, int64_t Bpad, double tol_rel) {
  constexpr int W = 2 * P + 1;
  extern __shared__ double sm[];  // kRL * kCS * W doubles, reused for the final sums
  __shared__ int s_flag;
  __shared__ int32_t s_cnt[256];
  const int cl = threadIdx.x % kCS, lr = threadIdx.x / kCS;
  const int64_t c = blockIdx.y * (int64_t)kCS + cl;
  const int32_t na = *nact;
  const int64_t r0 = blockIdx.x * (int64_t)st.chunk_rows;
  const int64_t r1 = min<int64_t>(st.m, r0 + st.chunk_rows);
  double acc[W];
#pragma unroll
  for (int j = 0; j < W; ++j) acc[j] = 0.0;
  int32_t s = -1;
  bool ok = false;
  if (c < na) {
    s = act[c];
    ok = (st.done[s] == 0);
  }
  // Ritz-basis rows of this chunk, shared by the block's 16 systems
  double* sphi = sm;                        // chunk_rows x 2P (Phi row, then S Phi row)
  for (int o = threadIdx.x; o < (int)(r1 - r0) * 2 * P; o += blockDim.x) {
    const int rl = o / (2 * P), j = o % (2 * P);
    sphi[o] = (j < P) ? lmp.Phi[(r0 + rl) * P + j] : lmp.SPhi[(r0 + rl) * P + (j - P)];
  }
  __syncthreads();
  if (ok) {
    const double alpha = mode ? st.alpha[s] : 0.0;
    for (int64_t r = r0 + lr; r < r1; r += kRL) {
      const int64_t e = r * st.ld + s;
      double rv = st.r[e];
      if (mode) {
        st.x[e] += alpha * st.p[e];
        rv -= alpha * st.q[e];
        st.r[e] = rv;
      }
      acc[0] += rv * rv;
      const double* row = sphi + (r - r0) * 2 * P;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        acc[1 + j] += row[j] * rv;
        acc[1 + P + j] += row[P + j] * rv;
      }
    }
  }
  __syncthreads();  // sphi is reused below
  // block reduction over the 16 row lanes (fixed order)
#pragma unroll
  for (int j = 0; j < W; ++j) sm[(j * kRL + lr) * kCS + cl] = acc[j];
  __syncthreads();
  for (int o = threadIdx.x; o < W * kCS; o += blockDim.x) {
    const int j = o / kCS, cc = o % kCS;
    const int64_t col = blockIdx.y * (int64_t)kCS + cc;
    double t = 0.0;
    for (int l = 0; l < kRL; ++l) t += sm[(j * kRL + l) * kCS + cc];
    if (col < na) st.part[(blockIdx.x * Bpad + col) * W + j] = t;
  }
  if (!last_arrival(st.tile_cnt + blockIdx.y, gridDim.x, &s_flag)) return;

  // ---- last block of this column tile: reduce over chunks, per-system scalars
  __shared__ double sG[3 * 16 * 16 + 16];
  __shared__ double sc1[kCS][16];
  for (int o = threadIdx.x; o < 3 * P * P; o += blockDim.x) sG[o] = lmp.G[o];
  if (threadIdx.x < P) sG[3 * P * P + threadIdx.x] = lmp.theta[threadIdx.x];
  for (int o = threadIdx.x; o < W * kCS; o += blockDim.x) {
    const int j = o / kCS, cc = o % kCS;
    const int64_t col = blockIdx.y * (int64_t)kCS + cc;
    double t = 0.0;
    if (col < na)
      for (int k = 0; k < (int)gridDim.x; ++k) t += vload(&st.part[(k * Bpad + col) * W + j]);
    sm[j * kCS + cc] = t;
  }
  __syncthreads();
  // one system per column (cc), its P coefficient indices spread over the 16 lanes (jj)
  const int cc = threadIdx.x % kCS, jj = threadIdx.x / kCS;
  const int64_t col = blockIdx.y * (int64_t)kCS + cc;
  int32_t sy = -1;
  int state = 0;  // 0 skip, 1 converged, 2 non-finite, 3 continue
  double sig1 = 1.0;
  if (col < na) {
    sy = act[col];
    if (st.done[sy] == 0) {
      const double rr = sm[cc];
      sig1 = 1.0 + st.sigma[sy];
      state = !isfinite(rr) ? 2 : (sqrt(rr) <= tol_rel * st.thresh[sy] ? 1 : 3);
    }
  }
  const double* sth = sG + 3 * P * P;
  if (state == 3 && jj < P) sc1[cc][jj] = sm[(1 + jj) * kCS + cc] / (sig1 + sth[jj]);
  __syncthreads();
  double* cf = (sy >= 0) ? st.coef + (int64_t)sy * W : nullptr;
  if (state == 3 && jj < P) {
    // (C Phi)^T (C Phi) = Gss + sig1 (Gps + Gps^T) + sig1^2 Gpp, applied to c1
    const double* Gpp = sG;
    const double* Gps = sG + P * P;
    const double* Gss = sG + 2 * P * P;
    double mc = 0.0;
    for (int l = 0; l < P; ++l)
      mc += (Gss[jj * P + l] + sig1 * (Gps[jj * P + l] + Gps[l * P + jj]) + sig1 * sig1 * Gpp[jj * P + l]) *
            sc1[cc][l];
    const double c2 = (sm[(1 + P + jj) * kCS + cc] + sig1 * sm[(1 + jj) * kCS + cc] - mc) / (sig1 + sth[jj]);
    const double beta_l = sig1 + *lmp.dmin;
    const double g = (sig1 - beta_l) * sc1[cc][jj] + c2;
    cf[jj] = sc1[cc][jj];
    cf[P + jj] = g;
    // the products of r^T z, summed below in index order
    sm[(W + jj) * kCS + cc] = sm[(1 + P + jj) * kCS + cc] * sc1[cc][jj] + sm[(1 + jj) * kCS + cc] * g;
  }
  __syncthreads();
  if (state != 0 && jj == 0) {
    const double rr = sm[cc];
    const double bn = st.bnorm[sy];
    const int it = st.iters[sy] + mode;
    st.iters[sy] = it;
    st.relres[sy] = bn > 0.0 ? sqrt(rr) / bn : 0.0;
    if (state == 2) {
      atomicOr(st.flags, kFlagNumeric);
      st.done[sy] = 2;
    } else if (state == 1) {
      st.done[sy] = 1;
    } else {
      double rz = rr;
      for (int j = 0; j < P; ++j) rz -= sm[(W + j) * kCS + cc];
      cf[2 * P] = mode ? rz / st.rz[sy] : 0.0;
      st.rz[sy] = rz;
      if (!(rz > 0.0)) {
        atomicOr(st.flags, isfinite(rz) ? kFlagNotSPD : kFlagNumeric);
        st.done[sy] = 2;
      } else if (it >= st.max_iter) {
        st.done[sy] = 2;
      }
    }
  }
  if (!last_arrival(st.glob_cnt, gridDim.y, &s_flag)) return;

  // ---- last block overall: next active list, in the order of the current one
  const int per = (na + 255) / 256;
  const int a = threadIdx.x * per, b = min(na, a + per);
  int32_t keep = 0;
  for (int i = a; i < b; ++i) keep += (vload_i32(&st.done[act[i]]) == 0);
  s_cnt[threadIdx.x] = keep;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int i = 0; i < 256; ++i) {
      const int32_t v = s_cnt[i];
      s_cnt[i] = run;
      run += v;
    }
    *nact_out = run;
  }
  __syncthreads();
  int32_t pos = s_cnt[threadIdx.x];
  for (int i = a; i < b; ++i) {
    const int32_t sy = act[i];
    if (vload_i32(&st.done[sy]) == 0) act_out[pos++] = sy;
  }
}

// p = z + beta p with z = r - S Phi c1 - Phi gamma for the systems of the (new) active list;
// optionally also writes p into the apply buffer V (column c of the list, apply precision).
template <int P, typename TV>
__global__ __launch_bounds__(256) void k_pcg_direction(PCGState st, LMP lmp, int first,
                                                       const int32_t* __restrict__ act,
                                                       const int32_t* __restrict__ nact, TV* __restrict__ V,
                                                       int64_t ldv) {
  constexpr int W = 2 * P + 1;
  __shared__ double cf[kCS][W];
  const int cl = threadIdx.x % kCS, lr = threadIdx.x / kCS;
  const int64_t c = blockIdx.y * (int64_t)kCS + cl;
  const int32_t na = *nact;
  if (blockIdx.y * (int64_t)kCS >= na) return;
  for (int o = threadIdx.x; o < kCS * W; o += blockDim.x) {
    const int cc = o / W, j = o % W;
    const int64_t col = blockIdx.y * (int64_t)kCS + cc;
    cf[cc][j] = (col < na) ? st.coef[(int64_t)act[col] * W + j] : 0.0;
  }
  __syncthreads();
  if (c >= na) return;
  const int32_t s = act[c];
  const double beta = cf[cl][2 * P];
  const int64_t r0 = blockIdx.x * (int64_t)st.chunk_rows;
  const int64_t r1 = min<int64_t>(st.m, r0 + st.chunk_rows);
  for (int64_t r = r0 + lr; r < r1; r += kRL) {
    const int64_t e = r * st.ld + s;
    double z = st.r[e];
#pragma unroll
    for (int j = 0; j < P; ++j) z -= lmp.SPhi[r * P + j] * cf[cl][j] + lmp.Phi[r * P + j] * cf[cl][P + j];
    const double pn = first ? z : z + beta * st.p[e];
    st.p[e] = pn;
    if (V) V[vidx<TV>(r, c, ldv)] = to_prec<TV>(pn);
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
// per-system 2-norm in two passes: partial sums of row chunks (16 systems x 16 row lanes per
// block), then one thread per system adds the chunks in order.
__global__ void k_col_norms_part(const double* __restrict__ v, int64_t m, int64_t S, int64_t ld, int chunk_rows,
                                 double* __restrict__ part) {
  __shared__ double red[16][16];
  const int cl = threadIdx.x % 16, lr = threadIdx.x / 16;
  const int64_t s = blockIdx.y * (int64_t)16 + cl;
  const int64_t r0 = blockIdx.x * (int64_t)chunk_rows, r1 = min<int64_t>(m, r0 + chunk_rows);
  double acc = 0.0;
  if (s < S)
    for (int64_t r = r0 + lr; r < r1; r += 16) {
      const double x = v[r * ld + s];
      acc += x * x;
    }
  red[lr][cl] = acc;
  __syncthreads();
  if (lr == 0 && s < S) {
    double t = red[0][cl];
    for (int j = 1; j < 16; ++j) t += red[j][cl];
    part[blockIdx.x * S + s] = t;
  }
}
__global__ void k_col_norms_fin(const double* __restrict__ part, int nchunks, int64_t S, double* __restrict__ out) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= S) return;
  double t = 0.0;
  for (int k = 0; k < nchunks; ++k) t += part[k * S + s];
  out[s] = sqrt(t);
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
hipError_t dispatch_step(const PCGState& s, const LMP& lmp, int mode, const int32_t* act, const int32_t* nact,
                         int32_t* act_out, int32_t* nact_out, int64_t Bpad, double tol, hipStream_t st) {
  constexpr int W = 2 * P + 1;
  size_t smem = sizeof(double) * (size_t)kCS * (kRL * W > W + P ? kRL * W : W + P);
  const size_t stage = sizeof(double) * (size_t)s.chunk_rows * 2 * P;  // Ritz rows of one chunk
  if (stage > smem) smem = stage;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pcg_step<P>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    attr = true;
  }
  dim3 grid(s.nchunks, (unsigned)((Bpad + kCS - 1) / kCS));
  hipLaunchKernelGGL(k_pcg_step<P>, grid, dim3(256), smem, st, s, lmp, mode, act, nact, act_out, nact_out, Bpad, tol);
  return hipGetLastError();
}
template <int P>
hipError_t dispatch_dir(Prec vp, const PCGState& s, const LMP& lmp, int first, const int32_t* act,
                        const int32_t* nact, int64_t Bpad, void* V, int64_t ldv, hipStream_t st) {
  dim3 grid(s.nchunks, (unsigned)((Bpad + kCS - 1) / kCS));
  if (vp == Prec::F64)
    hipLaunchKernelGGL((k_pcg_direction<P, double>), grid, dim3(256), 0, st, s, lmp, first, act, nact, (double*)V,
                       ldv);
  else if (vp == Prec::F32)
    hipLaunchKernelGGL((k_pcg_direction<P, float>), grid, dim3(256), 0, st, s, lmp, first, act, nact, (float*)V, ldv);
  else
    hipLaunchKernelGGL((k_pcg_direction<P, __hip_bfloat16>), grid, dim3(256), 0, st, s, lmp, first, act, nact,
                       (__hip_bfloat16*)V, ldv);
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
  else if (prec == Prec::F32)
    hipLaunchKernelGGL(k_gather_active<float>, dim3(nb(rows * Bpad)), dim3(256), 0, st, P, ldp, act, nact, rows,
                       Bpad, (float*)V, ldv);
  else
    hipLaunchKernelGGL(k_gather_active<__hip_bfloat16>, dim3(nb(rows * Bpad)), dim3(256), 0, st, P, ldp, act, nact,
                       rows, Bpad, (__hip_bfloat16*)V, ldv);
  return hipGetLastError();
}

hipError_t launch_scatter_state(Prec prec, const double* P, int64_t ldp, const int32_t* act, const int32_t* nact,
                                const int32_t* col_ptr, const int32_t* row_of, const double* w_of,
                                const double* r_var, int64_t n, int64_t m, int64_t Bpad, void* V, int64_t ldv,
                                hipStream_t st) {
  if (prec == Prec::F64)
    hipLaunchKernelGGL(k_scatter_state<double>, dim3(nb(n * Bpad)), dim3(256), 0, st, P, ldp, act, nact, col_ptr,
                       row_of, w_of, r_var, n, m, Bpad, (double*)V, ldv);
  else if (prec == Prec::F32)
    hipLaunchKernelGGL(k_scatter_state<float>, dim3(nb(n * Bpad)), dim3(256), 0, st, P, ldp, act, nact, col_ptr,
                       row_of, w_of, r_var, n, m, Bpad, (float*)V, ldv);
  else
    hipLaunchKernelGGL(k_scatter_state<__hip_bfloat16>, dim3(nb(n * Bpad)), dim3(256), 0, st, P, ldp, act, nact,
                       col_ptr, row_of, w_of, r_var, n, m, Bpad, (__hip_bfloat16*)V, ldv);
  return hipGetLastError();
}

hipError_t launch_apply_finish(Prec prec, int obs_domain, const double* P, int64_t ldp, const void* T, int64_t ldt,
                               const int32_t* act, const int32_t* nact, const double* sigma, const int32_t* h_ptr,
                               const int32_t* h_idx, const double* h_w, const double* r_var, int64_t m,
                               int64_t n_state, int64_t Bpad, double* Qv, double* part, int chunk_rows,
                               const AlphaOut* alpha, hipStream_t st) {
  const int nchunks = (int)((m + chunk_rows - 1) / chunk_rows);
  dim3 grid(nchunks, (unsigned)((Bpad + 15) / 16));
  const AlphaOut ao = alpha ? *alpha : AlphaOut{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (prec == Prec::F64)
    hipLaunchKernelGGL(k_apply_finish<double>, grid, dim3(256), 0, st, obs_domain, P, ldp, (const double*)T, ldt,
                       act, nact, sigma, h_ptr, h_idx, h_w, r_var, m, n_state, Bpad, Qv, part, chunk_rows, ao);
  else
    hipLaunchKernelGGL(k_apply_finish<float>, grid, dim3(256), 0, st, obs_domain, P, ldp, (const float*)T, ldt, act,
                       nact, sigma, h_ptr, h_idx, h_w, r_var, m, n_state, Bpad, Qv, part, chunk_rows, ao);
  return hipGetLastError();
}

hipError_t launch_pcg_step(const PCGState& s, const LMP& lmp, int mode, const int32_t* act, const int32_t* nact,
                           int32_t* act_out, int32_t* nact_out, int64_t Bpad, double tol_rel, hipStream_t st) {
#define IE_CALL(P) dispatch_step<P>(s, lmp, mode, act, nact, act_out, nact_out, Bpad, tol_rel, st)
  IE_P_SWITCH(lmp.p, IE_CALL)
#undef IE_CALL
}

hipError_t launch_pcg_direction(Prec vprec, const PCGState& s, const LMP& lmp, int first, const int32_t* act,
                                const int32_t* nact, int64_t Bpad, void* V, int64_t ldv, hipStream_t st) {
#define IE_CALL(P) dispatch_dir<P>(vprec, s, lmp, first, act, nact, Bpad, V, ldv, st)
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
hipError_t launch_col_norms(const double* v, int64_t m, int64_t S, int64_t ld, double* out, double* scratch,
                            hipStream_t st) {
  const int chunk = 64;
  const int nchunks = (int)((m + chunk - 1) / chunk);
  hipLaunchKernelGGL(k_col_norms_part, dim3(nchunks, (unsigned)((S + 15) / 16)), dim3(256), 0, st, v, m, S, ld, chunk,
                     scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_norms_fin, dim3(nb(S)), dim3(256), 0, st, scratch, nchunks, S, out);
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
