// Batched preconditioned conjugate gradients (Golub & Van Loan Alg. 11.5.1) with the
// limited-memory Ritz preconditioner of Appendix E, plus the observation-space glue
// around the covariance apply.
//
// Layout: every family of observation-space vectors (x, r, p, b, u) and the apply
// buffers are system-major: element (row r, system s) at s * ld + r.  One
// workgroup owns one system in the fused PCG kernel, so every reduction of an
// iteration is local to a workgroup (fixed shuffle/LDS tree: bit-reproducible)
// and the whole iteration after the covariance apply is one launch:
//
//   q = (1 + sigma) p + S p  (S p from the apply output),  alpha = r^T z / p^T q,
//   x += alpha p, r -= alpha q, dots of r with itself and the Ritz bases,
//   convergence test, z = P^{-1} r from those dots, p = z + beta p,
//   and p written into the next apply buffer at a slot claimed with an atomic.
//
// Apply columns are independent, so the order in which systems claim slots does
// not change any value.
#include "internal.hpp"

namespace infoesrf {

namespace {

inline unsigned nb(int64_t count) { return (unsigned)((count + 255) / 256); }

__device__ inline int32_t load_nact(const int32_t* nact, int64_t fallback) {
  return nact ? *nact : (int32_t)fallback;
}

template <typename TV>
__device__ inline TV to_prec(double v);
template <>
__device__ inline double to_prec<double>(double v) { return v; }
template <>
__device__ inline float to_prec<float>(double v) { return (float)v; }
template <>
__device__ inline __hip_bfloat16 to_prec<__hip_bfloat16>(double v) { return __float2bfloat16((float)v); }

// --------------------------------------------------------------- apply glue

// V[c * ldv + r] = P[act[c] * ldp + r] for c < nact (zero for nact <= c < Bmax), r < rows.
template <typename TV>
__global__ void k_gather_active(const double* __restrict__ P, int64_t ldp, const int32_t* __restrict__ act,
                                const int32_t* __restrict__ nact, int64_t rows, int64_t Bmax, TV* __restrict__ V,
                                int64_t ldv) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= rows * Bmax) return;
  const int64_t c = t / rows, r = t % rows;
  const int32_t na = load_nact(nact, Bmax);
  V[c * ldv + r] = to_prec<TV>((c < na) ? P[(int64_t)act[c] * ldp + r] : 0.0);
}

// V[c * ldv + k] = sum_{e in column k of H} w_e r_{row}^{-1/2} P[act[c] * ldp + row_e]
template <typename TV>
__global__ void k_scatter_state(const double* __restrict__ P, int64_t ldp, const int32_t* __restrict__ act,
                                const int32_t* __restrict__ nact, const int32_t* __restrict__ col_ptr,
                                const int32_t* __restrict__ row_of, const double* __restrict__ w_of,
                                const double* __restrict__ r_var, int64_t n, int64_t m, int64_t Bmax,
                                TV* __restrict__ V, int64_t ldv) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * Bmax) return;
  const int64_t c = t / n, k = t % n;
  const int32_t na = load_nact(nact, Bmax);
  double acc = 0.0;
  if (c < na) {
    const int64_t s = act[c];
    for (int32_t e = col_ptr[k]; e < col_ptr[k + 1]; ++e) {
      const int32_t r = row_of[e];
      if (r >= 0 && r < m) acc += w_of[e] / sqrt(r_var[r]) * P[s * ldp + r];
    }
  }
  V[c * ldv + k] = to_prec<TV>(acc);
}

// S p at row r of apply column c: obs domain T itself, state domain R^{-1/2} H T.
template <typename TT>
__device__ inline double s_times(int obs_domain, const TT* T, int64_t ldt, int64_t c, int64_t r,
                                 const int32_t* h_ptr, const int32_t* h_idx, const double* h_w,
                                 const double* r_var, int64_t n_state) {
  const TT* col = T + c * ldt;
  if (obs_domain) return (double)col[r];
  double a = 0.0;
  for (int32_t e = h_ptr[r]; e < h_ptr[r + 1]; ++e) {
    const int32_t j = h_idx[e];
    if (j >= 0 && j < n_state) a += h_w[e] * (double)col[j];
  }
  return a / sqrt(r_var[r]);
}

// Q[s * ldp + r] = (1 + sigma_s) P[s * ldp + r] + (S P)[r, s], s = act[c].
template <typename TT>
__global__ void k_apply_finish(int obs_domain, const double* __restrict__ P, int64_t ldp, const TT* __restrict__ T,
                               int64_t ldt, const int32_t* __restrict__ act, const int32_t* __restrict__ nact,
                               const double* __restrict__ sigma, const int32_t* __restrict__ h_ptr,
                               const int32_t* __restrict__ h_idx, const double* __restrict__ h_w,
                               const double* __restrict__ r_var, int64_t m, int64_t n_state, int64_t Bmax,
                               double* __restrict__ Qv) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m * Bmax) return;
  const int64_t c = t / m, r = t % m;
  if (c >= load_nact(nact, Bmax)) return;
  const int64_t s = act[c];
  const double sp = s_times<TT>(obs_domain, T, ldt, c, r, h_ptr, h_idx, h_w, r_var, n_state);
  Qv[s * ldp + r] = (1.0 + sigma[s]) * P[s * ldp + r] + sp;
}

// --------------------------------------------------------------- fused PCG iteration

// Sum over the workgroup (256 threads) of W values per thread; fixed tree (DPP sums within a
// wavefront, then the four wavefronts in order).  Result broadcast to every thread in out[].
template <int W>
__device__ inline void block_sum(const double* v, double (*sred)[4], double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const double x = wave_sum_dpp(v[j]);
    if (lane == 63) sred[j][wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < W; ++j) out[j] = ((sred[j][0] + sred[j][1]) + sred[j][2]) + sred[j][3];
  __syncthreads();
}

// The same sums (same order) written once to LDS: out_lds[j] for j < W, read back by every lane.
template <int W>
__device__ inline void block_sum_lds(const double* v, double (*sred)[4], double* out_lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const double x = wave_sum_dpp(v[j]);
    if (lane == 63) sred[j][wave] = x;
  }
  __syncthreads();
  if ((int)threadIdx.x < W) {
    const int j = threadIdx.x;
    out_lds[j] = ((sred[j][0] + sred[j][1]) + sred[j][2]) + sred[j][3];
  }
  __syncthreads();
}

template <int P, int RPT, typename TT, typename TV>
__global__ __launch_bounds__(256) void k_pcg_fused(PCGState st, LMP lmp, int mode, int obs_domain, int plain,
                                                   const TT* __restrict__ T, int64_t ldt,
                                                   const int32_t* __restrict__ act, const int32_t* __restrict__ nact,
                                                   int32_t* __restrict__ act_out, int32_t* __restrict__ nact_out,
                                                   TV* __restrict__ V, int64_t ldv, const int32_t* __restrict__ h_ptr,
                                                   const int32_t* __restrict__ h_idx, const double* __restrict__ h_w,
                                                   const double* __restrict__ r_var, int64_t n_state) {
  constexpr int W = 2 * P + 1;
  __shared__ double sred[W][4];
  __shared__ double sG[3 * P * P + P + 1];
  __shared__ double scoef[2 * P + 2];
  __shared__ double sdot[W];  // the reduced dots (broadcast reads; lanes index them by thread id)
  __shared__ int s_slot;
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  // The kernel is a chain of dependent steps per system, so every load that does not depend on
  // an earlier result is issued in the same round trip: (1) the list entry with the list length
  // (c < grid <= list capacity); (2) everything the system needs; (3) Phi, S Phi for the dots;
  // (4) Phi, S Phi again for the preconditioned residual.
  const int na = *nact;
  const int32_t s = act[c];
  if (st.prof.vectors && c == 0 && tid == 0) {
    atomicAdd(st.prof.vectors, (unsigned long long)na);
    atomicAdd(st.prof.flops, (double)na * st.prof.flops_per_vector);
    atomicAdd(st.prof.bytes, (double)na * st.prof.bytes_per_vector);
  }
  if (c >= na) return;
  const int64_t m = st.m;
  const int64_t base = (int64_t)s * st.ld;

  // Next list: a system claims a slot (appended in any order) and writes its next apply input
  // there.  nact_out[0] counts the list; in the masked solver, where retired systems stay in the
  // list, nact_out[1] counts the systems still iterating.  In the masked solver a system claims
  // its slot once it knows it continues (the atomic overlaps the preconditioner arithmetic); in
  // the compacted one it claims at the start (see below).
  int slot_reg = -1;  // thread 0: a slot claimed early whose number is consumed in write_v
  auto claim = [&](bool live) {
    if (tid == 0) {
      const int slot = atomicAdd(nact_out, 1);
      if (live && plain) atomicAdd(nact_out + 1, 1);
      act_out[slot] = s;
      s_slot = slot;
    }
  };
  auto claim_early = [&]() {
    if (tid == 0) slot_reg = atomicAdd(nact_out, 1);
  };
  auto write_v = [&](const double* pv) {
    if (tid == 0 && slot_reg >= 0) {  // the early claim's result is needed only now
      act_out[slot_reg] = s;
      s_slot = slot_reg;
    }
    __syncthreads();
    if (V) {
      TV* col = V + (int64_t)s_slot * ldv;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int64_t r = tid + 256 * j;
        if (r < m) col[r] = to_prec<TV>(pv ? pv[j] : 0.0);
      }
    }
  };
  auto append = [&](const double* pv) {
    claim(pv != nullptr);
    write_v(pv);
  };

  // (2) per-system scalars and vectors, and the preconditioner's small matrices into LDS
  const int32_t dn = st.done[s];
  const double sig1 = 1.0 + st.sigma[s];
  const double rz_old = st.rz[s];
  const int it = st.iters[s] + mode;
  const double bn = st.bnorm[s];
  const double thresh = st.thresh[s];
  double rv[RPT], pv[RPT], xv[RPT], sv[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int64_t r = tid + 256 * j;
    const bool ok = r < m;
    rv[j] = ok ? st.r[base + r] : 0.0;
    pv[j] = ok ? st.p[base + r] : 0.0;
    xv[j] = (ok && mode == 1) ? st.x[base + r] : 0.0;
    sv[j] = (ok && mode == 1 && obs_domain) ? (double)T[(int64_t)c * ldt + r] : 0.0;
  }
  // The Ritz vectors are read for the dots of r and, when they fit in registers, kept for the
  // preconditioned residual, so each system reads them once per iteration.  (They are not loaded
  // with the system's data: that many loads in flight would stall the first round trip.)
  constexpr bool kCache = (RPT * P <= 24);
  constexpr int kC = (kCache && P > 0) ? RPT * P : 1;
  double ph[kC], sph[kC];
  if (P > 0) {
    for (int o = tid; o < 3 * P * P; o += blockDim.x) sG[o] = lmp.G[o];
    if (tid < P) sG[3 * P * P + tid] = lmp.theta[tid];
  }
  const double dmin = (P > 0) ? *lmp.dmin : 0.0;

  if (dn != 0) {  // only reachable in the masked solver, or for a slot that broke down
    if (plain) append(nullptr);
    return;
  }
  // Compacted lists: a live system claims its next slot now, so the atomic's round trip overlaps
  // the step.  A system that then converges or breaks down leaves a zero direction in the slot
  // and drops out of the next step, where done != 0.
  if (!plain) claim_early();
  if (mode == 1) {
    double qv[RPT];
    double pq = 0.0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int64_t r = tid + 256 * j;
      qv[j] = 0.0;
      if (r < m) {
        const double sp =
            obs_domain ? sv[j] : s_times<TT>(obs_domain, T, ldt, c, r, h_ptr, h_idx, h_w, r_var, n_state);
        qv[j] = sig1 * pv[j] + sp;
        pq += pv[j] * qv[j];
      }
    }
    double tot;
    block_sum<1>(&pq, sred, &tot);
    if (!(tot > 0.0) || !isfinite(tot)) {
      if (tid == 0) {
        atomicOr(st.flags, isfinite(tot) ? kFlagNotSPD : kFlagNumeric);
        st.done[s] = 2;
      }
      if (plain) append(nullptr);
      else write_v(nullptr);
      return;
    }
    const double alpha = rz_old / tot;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int64_t r = tid + 256 * j;
      if (r < m) {
        st.x[base + r] = xv[j] + alpha * pv[j];
        rv[j] -= alpha * qv[j];
        st.r[base + r] = rv[j];
      }
    }
  }
  // (3) dots of r: r^T r, Phi^T r, (S Phi)^T r.
  double acc[W];
  const double* d = sdot;
#pragma unroll
  for (int j = 0; j < W; ++j) acc[j] = 0.0;
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int64_t r = tid + 256 * j;
    if (r < m) {
      acc[0] += rv[j] * rv[j];
#pragma unroll
      for (int l = 0; l < P; ++l) {
        const double a = lmp.Phi[l * lmp.ld + r], b = lmp.SPhi[l * lmp.ld + r];
        if (kCache) {
          ph[j * P + l] = a;
          sph[j * P + l] = b;
        }
        acc[1 + l] += a * rv[j];
        acc[1 + P + l] += b * rv[j];
      }
    }
  }
  block_sum_lds<W>(acc, sred, sdot);  // also orders the LDS writes of sG above
  const double rn = sqrt(d[0]);
  if (tid == 0) {
    st.iters[s] = it;
    st.relres[s] = bn > 0.0 ? rn / bn : 0.0;
  }
  if (!isfinite(d[0])) {
    if (tid == 0) {
      atomicOr(st.flags, kFlagNumeric);
      st.done[s] = 2;
    }
    if (plain) append(nullptr);
    else write_v(nullptr);
    return;
  }
  if (rn <= thresh) {
    if (tid == 0) st.done[s] = 1;
    if (plain) append(nullptr);
    else write_v(nullptr);
    return;
  }
  if (it >= st.max_iter) {
    if (tid == 0) st.done[s] = 2;
    if (plain) append(nullptr);
    else write_v(nullptr);
    return;
  }
  if (plain) claim(true);
  // limited-memory preconditioner coefficients (Appendix E), with Theta = diag(1 + sigma + theta_j):
  //   c1 = Theta^{-1} Phi^T r,  c2 = Theta^{-1} [(C Phi)^T r - (C Phi)^T (C Phi) c1],
  //   gamma = (1 + sigma - beta_L) c1 + c2,  z = r - S Phi c1 - Phi gamma,
  //   r^T z = r^T r - ((S Phi)^T r) . c1 - (Phi^T r) . gamma.
  double rz = d[0];
  if (P > 0) {
    const double* sth = sG + 3 * P * P;
    if (tid < P) scoef[tid] = sdot[1 + tid] / (sig1 + sth[tid]);
    __syncthreads();
    if (tid < P) {
      const double* Gpp = sG;
      const double* Gps = sG + P * P;
      const double* Gss = sG + 2 * P * P;
      double mc = 0.0;
      for (int l = 0; l < P; ++l)
        mc += (Gss[tid * P + l] + sig1 * (Gps[tid * P + l] + Gps[l * P + tid]) + sig1 * sig1 * Gpp[tid * P + l]) *
              scoef[l];
      const double c2 = (sdot[1 + P + tid] + sig1 * sdot[1 + tid] - mc) / (sig1 + sth[tid]);
      const double beta_l = sig1 + dmin;
      scoef[P + tid] = (sig1 - beta_l) * scoef[tid] + c2;
    }
    __syncthreads();
    for (int l = 0; l < P; ++l) rz -= d[1 + P + l] * scoef[l] + d[1 + l] * scoef[P + l];
  }
  const double beta = mode ? rz / rz_old : 0.0;
  if (!(rz > 0.0) || !isfinite(rz)) {
    if (tid == 0) {
      atomicOr(st.flags, isfinite(rz) ? kFlagNotSPD : kFlagNumeric);
      st.done[s] = 2;
    }
    write_v(nullptr);  // the slot is claimed: a zero direction, skipped next step (done != 0)
    return;
  }
  if (tid == 0) st.rz[s] = rz;  // rz_old was read into registers at the start
  // (4) the preconditioned residual and the next direction
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int64_t r = tid + 256 * j;
    if (r < m) {
      double z = rv[j];
#pragma unroll
      for (int l = 0; l < P; ++l) {
        const double a = kCache ? ph[j * P + l] : lmp.Phi[l * lmp.ld + r];
        const double b = kCache ? sph[j * P + l] : lmp.SPhi[l * lmp.ld + r];
        z -= b * scoef[l] + a * scoef[P + l];
      }
      pv[j] = mode ? z + beta * pv[j] : z;
      st.p[base + r] = pv[j];
    }
  }
  write_v(pv);
}

// --------------------------------------------------------------- list and vector kernels

__global__ __launch_bounds__(256) void k_compact(const int32_t* __restrict__ done, int64_t S,
                                                 int32_t* __restrict__ act, int32_t* __restrict__ nact) {
  __shared__ int swave[4];
  __shared__ int total;
  const int t = threadIdx.x;
  const int64_t per = (S + 255) / 256;
  const int64_t a = t * per, b = min<int64_t>(S, a + per);
  int32_t c = 0;
  for (int64_t s = a; s < b; ++s) c += (done[s] == 0);
  int32_t pos = block_exclusive_scan<256>(c, swave, &total);
  if (t == 0) *nact = total;
  for (int64_t s = a; s < b; ++s)
    if (done[s] == 0) act[pos++] = (int32_t)s;
}

__global__ void k_iota(int32_t* __restrict__ act, int32_t* __restrict__ nact, int64_t S) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < S) act[t] = (int32_t)t;
  if (t == 0) *nact = (int32_t)S;
}

__global__ void k_fill_f64(double* p, double v, int64_t count) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count) p[t] = v;
}
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t count) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count) p[t] = v;
}
__global__ void k_sub(const double* a, const double* b, double* out, int64_t count) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count) out[t] = a[t] - b[t];
}
__global__ void k_axpy(double* x, const double* d, int64_t count) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count) x[t] += d[t];
}
// per-system 2-norm: one workgroup per system, fixed tree
__global__ __launch_bounds__(256) void k_col_norms(const double* __restrict__ v, int64_t m, int64_t ld,
                                                   double* __restrict__ out) {
  __shared__ double sred[1][4];
  const int64_t s = blockIdx.x;
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < m; r += 256) {
    const double x = v[s * ld + r];
    acc += x * x;
  }
  double tot;
  block_sum<1>(&acc, sred, &tot);
  if (threadIdx.x == 0) out[s] = sqrt(tot);
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
// ubar[i * ldb + r] = sum_q p_q u[(s0 + q N + i) * ldu + r]
__global__ void k_quad_combine(const double* __restrict__ u, int64_t ldu, int64_t m, int64_t N, int32_t Q,
                               const double* __restrict__ pw, double* __restrict__ ubar, int64_t ldb, int64_t s0,
                               int32_t* __restrict__ act, int32_t* __restrict__ nact) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (act && t < N) act[t] = (int32_t)t;
  if (act && t == 0) *nact = (int32_t)N;
  if (t >= m * N) return;
  const int64_t i = t / m, r = t % m;
  // eight loads in flight, then the terms in order of q
  constexpr int U = 8;
  double acc = 0.0;
  for (int32_t q0 = 0; q0 < Q; q0 += U) {
    double v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) v[k] = q0 + k < Q ? u[(s0 + (int64_t)(q0 + k) * N + i) * ldu + r] : 0.0;
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (q0 + k < Q) acc += pw[q0 + k] * v[k];
  }
  ubar[i * ldb + r] = acc;
}
__global__ void k_final_pert(const double* __restrict__ Z, const double* __restrict__ T, int64_t ldt, int64_t n,
                             int64_t N, double scale, double* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * N) return;
  const int64_t k = t % n, i = t / n;
  out[k + i * n] = scale * (Z[k + i * n] - T[i * ldt + k]);
}
__global__ void k_final_mean(const double* __restrict__ mu, const double* __restrict__ T, int64_t ldt, int64_t n,
                             int64_t col, double* __restrict__ out) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) out[k] = mu[k] + T[col * ldt + k];
}
// dst[c * ldd + r] = src[c * lds + r] (r < rows), zero for rows <= r < ldd
__global__ void k_copy_cols(const double* __restrict__ src, int64_t lds, int64_t rows, int64_t cols,
                            double* __restrict__ dst, int64_t ldd) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ldd * cols) return;
  const int64_t c = t / ldd, r = t % ldd;
  dst[t] = (r < rows) ? src[c * lds + r] : 0.0;
}
template <int P, int RPT, typename TT, typename TV>
hipError_t fused_typed(const PCGState& s, const LMP& lmp, int mode, int obs, int plain, const void* T, int64_t ldt,
                       const int32_t* act, const int32_t* nact, int32_t* act_out, int32_t* nact_out, int64_t Bmax,
                       void* V, int64_t ldv, const int32_t* h_ptr, const int32_t* h_idx, const double* h_w,
                       const double* r_var, int64_t n_state, hipStream_t st) {
  if (Bmax <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_pcg_fused<P, RPT, TT, TV>), dim3((unsigned)Bmax), dim3(256), 0, st, s, lmp, mode, obs, plain,
                     (const TT*)T, ldt, act, nact, act_out, nact_out, (TV*)V, ldv, h_ptr, h_idx, h_w, r_var, n_state);
  return hipGetLastError();
}

template <int P, int RPT>
hipError_t fused_prec(Prec prec, const PCGState& s, const LMP& lmp, int mode, int obs, int plain, const void* T,
                      int64_t ldt, const int32_t* act, const int32_t* nact, int32_t* act_out, int32_t* nact_out,
                      int64_t Bmax, void* V, int64_t ldv, const int32_t* h_ptr, const int32_t* h_idx,
                      const double* h_w, const double* r_var, int64_t n_state, hipStream_t st) {
  // T is FP64 for FP64 applies and FP32 otherwise; V (written only in the observation domain) has the
  // apply precision.
  switch (prec) {
    case Prec::F64:
      return fused_typed<P, RPT, double, double>(s, lmp, mode, obs, plain, T, ldt, act, nact, act_out, nact_out, Bmax,
                                                 V, ldv, h_ptr, h_idx, h_w, r_var, n_state, st);
    case Prec::F32:
      return fused_typed<P, RPT, float, float>(s, lmp, mode, obs, plain, T, ldt, act, nact, act_out, nact_out, Bmax,
                                               V, ldv, h_ptr, h_idx, h_w, r_var, n_state, st);
    default:
      return fused_typed<P, RPT, float, __hip_bfloat16>(s, lmp, mode, obs, plain, T, ldt, act, nact, act_out,
                                                        nact_out, Bmax, V, ldv, h_ptr, h_idx, h_w, r_var, n_state,
                                                        st);
  }
}

template <int P>
hipError_t fused_rows(Prec prec, const PCGState& s, const LMP& lmp, int mode, int obs, int plain, const void* T,
                      int64_t ldt, const int32_t* act, const int32_t* nact, int32_t* act_out, int32_t* nact_out,
                      int64_t Bmax, void* V, int64_t ldv, const int32_t* h_ptr, const int32_t* h_idx,
                      const double* h_w, const double* r_var, int64_t n_state, hipStream_t st) {
  const int64_t rpt = (s.m + 255) / 256;
#define IE_F(R)                                                                                                     \
  return fused_prec<P, R>(prec, s, lmp, mode, obs, plain, T, ldt, act, nact, act_out, nact_out, Bmax, V, ldv, h_ptr, \
                          h_idx, h_w, r_var, n_state, st)
  if (rpt <= 1) IE_F(1);
  if (rpt <= 2) IE_F(2);
  if (rpt <= 4) IE_F(4);
  if (rpt <= 8) IE_F(8);
  if (rpt <= 16) IE_F(16);
#undef IE_F
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_gather_active(Prec prec, const double* P, int64_t ldp, const int32_t* act, const int32_t* nact,
                                int64_t rows, int64_t Bmax, void* V, int64_t ldv, hipStream_t st) {
  if (Bmax <= 0) return hipSuccess;
  if (prec == Prec::F64)
    hipLaunchKernelGGL(k_gather_active<double>, dim3(nb(rows * Bmax)), dim3(256), 0, st, P, ldp, act, nact, rows, Bmax,
                       (double*)V, ldv);
  else if (prec == Prec::F32)
    hipLaunchKernelGGL(k_gather_active<float>, dim3(nb(rows * Bmax)), dim3(256), 0, st, P, ldp, act, nact, rows, Bmax,
                       (float*)V, ldv);
  else
    hipLaunchKernelGGL(k_gather_active<__hip_bfloat16>, dim3(nb(rows * Bmax)), dim3(256), 0, st, P, ldp, act, nact,
                       rows, Bmax, (__hip_bfloat16*)V, ldv);
  return hipGetLastError();
}

hipError_t launch_scatter_state(Prec prec, const double* P, int64_t ldp, const int32_t* act, const int32_t* nact,
                                const int32_t* col_ptr, const int32_t* row_of, const double* w_of,
                                const double* r_var, int64_t n, int64_t m, int64_t Bmax, void* V, int64_t ldv,
                                hipStream_t st) {
  if (Bmax <= 0) return hipSuccess;
  if (prec == Prec::F64)
    hipLaunchKernelGGL(k_scatter_state<double>, dim3(nb(n * Bmax)), dim3(256), 0, st, P, ldp, act, nact, col_ptr,
                       row_of, w_of, r_var, n, m, Bmax, (double*)V, ldv);
  else if (prec == Prec::F32)
    hipLaunchKernelGGL(k_scatter_state<float>, dim3(nb(n * Bmax)), dim3(256), 0, st, P, ldp, act, nact, col_ptr,
                       row_of, w_of, r_var, n, m, Bmax, (float*)V, ldv);
  else
    hipLaunchKernelGGL(k_scatter_state<__hip_bfloat16>, dim3(nb(n * Bmax)), dim3(256), 0, st, P, ldp, act, nact,
                       col_ptr, row_of, w_of, r_var, n, m, Bmax, (__hip_bfloat16*)V, ldv);
  return hipGetLastError();
}

hipError_t launch_apply_finish(Prec prec, int obs_domain, const double* P, int64_t ldp, const void* T, int64_t ldt,
                               const int32_t* act, const int32_t* nact, const double* sigma, const int32_t* h_ptr,
                               const int32_t* h_idx, const double* h_w, const double* r_var, int64_t m,
                               int64_t n_state, int64_t Bmax, double* Qv, hipStream_t st) {
  if (Bmax <= 0) return hipSuccess;
  if (prec == Prec::F64)
    hipLaunchKernelGGL(k_apply_finish<double>, dim3(nb(m * Bmax)), dim3(256), 0, st, obs_domain, P, ldp,
                       (const double*)T, ldt, act, nact, sigma, h_ptr, h_idx, h_w, r_var, m, n_state, Bmax, Qv);
  else
    hipLaunchKernelGGL(k_apply_finish<float>, dim3(nb(m * Bmax)), dim3(256), 0, st, obs_domain, P, ldp,
                       (const float*)T, ldt, act, nact, sigma, h_ptr, h_idx, h_w, r_var, m, n_state, Bmax, Qv);
  return hipGetLastError();
}

#define IE_P_SWITCH(p, CALL)              \
  switch (p) {                            \
    case 0: return CALL(0);               \
    case 4: return CALL(4);               \
    case 8: return CALL(8);               \
    case 10: return CALL(10);             \
    case 12: return CALL(12);             \
    case 16: return CALL(16);             \
    case 20: return CALL(20);             \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_pcg_fused(Prec prec, const PCGState& s, const LMP& lmp, int mode, int obs_domain, int plain,
                            const void* T, int64_t ldt, const int32_t* act, const int32_t* nact, int32_t* act_out,
                            int32_t* nact_out, int64_t Bmax, void* V, int64_t ldv, const int32_t* h_ptr,
                            const int32_t* h_idx, const double* h_w, const double* r_var, int64_t n_state,
                            hipStream_t st) {
#define IE_CALL(P)                                                                                                   \
  fused_rows<P>(prec, s, lmp, mode, obs_domain, plain, T, ldt, act, nact, act_out, nact_out, Bmax, V, ldv, h_ptr, \
                h_idx, h_w, r_var, n_state, st)
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
hipError_t launch_sub(const double* a, const double* b, double* out, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_sub, dim3(nb(count)), dim3(256), 0, st, a, b, out, count);
  return hipGetLastError();
}
hipError_t launch_axpy(double* x, const double* d, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(nb(count)), dim3(256), 0, st, x, d, count);
  return hipGetLastError();
}
hipError_t launch_col_norms(const double* v, int64_t m, int64_t S, int64_t ld, double* out, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_col_norms, dim3((unsigned)S), dim3(256), 0, st, v, m, ld, out);
  return hipGetLastError();
}
hipError_t launch_residual_status(const double* rn, const double* bn, double tol, double* relres, int32_t* done,
                                  int64_t S, int32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_residual_status, dim3(nb(S)), dim3(256), 0, st, rn, bn, tol, relres, done, S, flags);
  return hipGetLastError();
}
hipError_t launch_quad_combine(const double* u, int64_t ldu, int64_t m, int64_t N, int32_t Q, const double* pw,
                               double* ubar, int64_t ldb, int64_t s0, int32_t* act, int32_t* nact, hipStream_t st) {
  if ((act == nullptr) != (nact == nullptr) || m < 1 || N < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_quad_combine, dim3(nb(m * N)), dim3(256), 0, st, u, ldu, m, N, Q, pw, ubar, ldb, s0, act,
                     nact);
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
hipError_t launch_copy_cols(const double* src, int64_t lds, int64_t rows, int64_t cols, double* dst, int64_t ldd,
                            hipStream_t st) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_cols, dim3(nb(ldd * cols)), dim3(256), 0, st, src, lds, rows, cols, dst, ldd);
  return hipGetLastError();
}

}  // namespace infoesrf
