// Multi-shift CG (the first alternative named in Sec. 3.2): the Q shifted systems
// ((1 + s_q) I + S) u = b_i of one member share their Krylov spaces, so one CG process on the
// smallest shift serves them all.  The shifted residuals stay parallel to the base residual,
// r_q = zeta_q r, and each shift's iterate follows from the base CG scalars through a
// three-term recurrence for zeta_q; every iteration takes one apply of S per member instead of
// one per (member, node).  No preconditioner: the limited-memory preconditioner of Appendix E
// depends on the shift and would break the shared Krylov space.
#include "internal.hpp"

namespace infoesrf {

namespace {

constexpr int kMscThreads = 256;

// Workgroup sum of two values per thread (fixed order: shuffles in a wavefront, then the four
// wavefronts in order); every thread gets both totals.
__device__ inline void sum2(double a, double b, double (*sred)[4], double* ta, double* tb) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  if (lane == 0) {
    sred[0][wave] = a;
    sred[1][wave] = b;
  }
  __syncthreads();
  *ta = ((sred[0][0] + sred[0][1]) + sred[0][2]) + sred[0][3];
  *tb = ((sred[1][0] + sred[1][1]) + sred[1][2]) + sred[1][3];
  __syncthreads();
}

// (S p)_r from the apply output column: the observation-domain output itself, or R^{-1/2} H T for
// a state-domain output.
__device__ inline double s_row(int obs_domain, const double* col, int64_t r, const int32_t* h_ptr,
                               const int32_t* h_idx, const double* h_w, const double* r_var, int64_t n_state) {
  if (obs_domain) return col[r];
  double a = 0.0;
  for (int32_t e = h_ptr[r]; e < h_ptr[r + 1]; ++e) {
    const int32_t j = h_idx[e];
    if (j >= 0 && j < n_state) a += h_w[e] * col[j];
  }
  return a / sqrt(r_var[r]);
}

// One multi-shift CG iteration per member of the list (one workgroup each).  The list holds the
// members' base systems q0 N + i.  mode 0 starts (p_q = b for every shift, zeta = 1); mode 1
// takes the base step from T = S p_base and updates every live shift.  A member with a live
// shift is appended to act_out (*nact_out zeroed beforehand) with its next base direction in V
// (observation domain; nullable).
template <int RPT>
__global__ __launch_bounds__(kMscThreads) void k_msc_step(MscState st, int mode, int obs_domain,
                                                          const double* __restrict__ T, int64_t ldt,
                                                          const int32_t* __restrict__ act,
                                                          const int32_t* __restrict__ nact,
                                                          int32_t* __restrict__ act_out,
                                                          int32_t* __restrict__ nact_out, double* __restrict__ V,
                                                          int64_t ldv, const int32_t* __restrict__ h_ptr,
                                                          const int32_t* __restrict__ h_idx,
                                                          const double* __restrict__ h_w,
                                                          const double* __restrict__ r_var, int64_t n_state) {
  __shared__ double sred[2][4];
  __shared__ double sz[kMaxQ], szp[kMaxQ], sig[kMaxQ], thr[kMaxQ], bnv[kMaxQ];
  __shared__ int32_t sdone[kMaxQ];
  __shared__ int s_slot;
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  if (c >= *nact) return;
  const int32_t sb = act[c];
  const int64_t N = st.N, m = st.m, ld = st.ld;
  const int64_t i = sb - (int64_t)st.q0 * N;
  const int Q = st.Q;
  // snapshot of the per-shift state: later writes in this launch go to global memory only
  if (tid < Q) {
    const int64_t s = (int64_t)tid * N + i;
    sz[tid] = st.zeta[s];
    szp[tid] = st.zeta_prev[s];
    sig[tid] = st.sigma[s];
    thr[tid] = st.thresh[s];
    bnv[tid] = st.bnorm[s];
    sdone[tid] = st.done[s];
  }
  const double* rcol = st.r + (int64_t)sb * ld;
  double rv[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int64_t r = tid + kMscThreads * j;
    rv[j] = r < m ? rcol[r] : 0.0;
  }
  __syncthreads();

  auto append = [&](const double* pv) {
    if (tid == 0) {
      const int slot = atomicAdd(nact_out, 1);
      act_out[slot] = sb;
      s_slot = slot;
    }
    __syncthreads();
    if (V) {
      double* col = V + (int64_t)s_slot * ldv;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int64_t r = tid + kMscThreads * j;
        if (r < m) col[r] = pv[j];
      }
    }
  };

  if (mode == 0) {
    double rr, unused;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) acc += rv[j] * rv[j];
    sum2(acc, 0.0, sred, &rr, &unused);
    bool live = false;
    for (int q = 0; q < Q; ++q) {
      const int64_t s = (int64_t)q * N + i;
      double* pc = st.p + s * ld;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int64_t r = tid + kMscThreads * j;
        if (r < m) pc[r] = rv[j];
      }
      if (tid == 0) {
        st.zeta[s] = 1.0;
        st.zeta_prev[s] = 1.0;
      }
      live = live || sdone[q] == 0;
    }
    if (tid == 0) {
      st.rr[i] = rr;
      st.alpha_prev[i] = 1.0;
      st.beta_prev[i] = 0.0;
      st.mit[i] = 0;
    }
    if (live) append(rv);
    return;
  }

  // base step: Ap = (1 + s_q0) p + S p on the base direction
  const double sig0 = sig[st.q0];
  const double* pcol = st.p + (int64_t)sb * ld;
  const double* tcol = T + (int64_t)c * ldt;
  double pv[RPT], apv[RPT];
  double pap = 0.0;
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int64_t r = tid + kMscThreads * j;
    pv[j] = 0.0;
    apv[j] = 0.0;
    if (r < m) {
      pv[j] = pcol[r];
      apv[j] = (1.0 + sig0) * pv[j] + s_row(obs_domain, tcol, r, h_ptr, h_idx, h_w, r_var, n_state);
      pap += pv[j] * apv[j];
    }
  }
  const double rr_old = st.rr[i];
  const double alpha_prev = st.alpha_prev[i], beta_prev = st.beta_prev[i];
  const int it = st.mit[i] + 1;
  double tot, unused;
  sum2(pap, 0.0, sred, &tot, &unused);
  if (!(tot > 0.0) || !isfinite(tot)) {
    if (tid == 0) {
      atomicOr(st.flags, isfinite(tot) ? kFlagNotSPD : kFlagNumeric);
      for (int q = 0; q < Q; ++q)
        if (sdone[q] == 0) st.done[(int64_t)q * N + i] = 2;
    }
    return;
  }
  const double alpha = rr_old / tot;
  double rr_acc = 0.0;
  double* rw = st.r + (int64_t)sb * ld;
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int64_t r = tid + kMscThreads * j;
    if (r < m) {
      rv[j] -= alpha * apv[j];
      rw[r] = rv[j];
      rr_acc += rv[j] * rv[j];
    }
  }
  double rr_new;
  sum2(rr_acc, 0.0, sred, &rr_new, &unused);
  const double beta = rr_new / rr_old;
  const double rnorm = sqrt(rr_new);
  bool live = false;
  for (int q = 0; q < Q; ++q) {
    const int64_t s = (int64_t)q * N + i;
    const bool base = (q == st.q0);
    if (sdone[q] != 0 && !base) continue;
    const double z = sz[q], zp = szp[q], dsg = sig[q] - sig0;
    const double den = alpha * beta_prev * (zp - z) + zp * alpha_prev * (1.0 + dsg * alpha);
    const double zn = base ? 1.0 : z * zp * alpha_prev / den;
    const double ratio = zn / z;
    const double as = alpha * ratio, bs = ratio * ratio * beta;
    double* xc = st.x + s * ld;
    double* pc = st.p + s * ld;
    const bool upd_x = sdone[q] == 0;  // a finished base keeps only its direction moving
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int64_t r = tid + kMscThreads * j;
      if (r < m) {
        const double pold = base ? pv[j] : pc[r];
        if (upd_x) xc[r] += as * pold;
        const double pn = zn * rv[j] + bs * pold;
        pc[r] = pn;
        if (base) pv[j] = pn;
      }
    }
    if (!upd_x) continue;
    const double res = fabs(zn) * rnorm;
    const bool fin = isfinite(zn);
    int ndone = 0;
    if (!fin) ndone = 2;
    else if (res <= thr[q]) ndone = 1;
    else if (it >= st.max_iter) ndone = 2;
    if (tid == 0) {
      st.zeta_prev[s] = z;
      st.zeta[s] = zn;
      st.iters[s] += 1;
      st.relres[s] = bnv[q] > 0.0 ? res / bnv[q] : 0.0;
      if (ndone) st.done[s] = ndone;
      if (!fin) atomicOr(st.flags, kFlagNumeric);
    }
    live = live || ndone == 0;
  }
  if (tid == 0) {
    st.rr[i] = rr_new;
    st.alpha_prev[i] = alpha;
    st.beta_prev[i] = beta;
    st.mit[i] = it;
  }
  if (live) append(pv);
}

// act[i] = q0 N + i, *nact = N: the members' base systems.
__global__ void k_msc_list(int32_t* act, int32_t* nact, int64_t q0, int64_t N) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < N) act[t] = (int32_t)(q0 * N + t);
  if (t == 0) *nact = (int32_t)N;
}

template <int RPT>
hipError_t msc_launch(const MscState& s, int mode, int obs, const double* T, int64_t ldt, const int32_t* act,
                      const int32_t* nact, int32_t* act_out, int32_t* nact_out, int64_t Bmax, double* V, int64_t ldv,
                      const int32_t* h_ptr, const int32_t* h_idx, const double* h_w, const double* r_var,
                      int64_t n_state, hipStream_t st) {
  hipLaunchKernelGGL(k_msc_step<RPT>, dim3((unsigned)std::max<int64_t>(Bmax, 1)), dim3(kMscThreads), 0, st, s, mode,
                     obs, T, ldt, act, nact, act_out, nact_out, V, ldv, h_ptr, h_idx, h_w, r_var, n_state);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_msc_list(int32_t* act, int32_t* nact, int64_t q0, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_msc_list, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, act, nact, q0, N);
  return hipGetLastError();
}

hipError_t launch_msc_step(const MscState& s, int mode, int obs_domain, const double* T, int64_t ldt,
                           const int32_t* act, const int32_t* nact, int32_t* act_out, int32_t* nact_out, int64_t Bmax,
                           double* V, int64_t ldv, const int32_t* h_ptr, const int32_t* h_idx, const double* h_w,
                           const double* r_var, int64_t n_state, hipStream_t st) {
  if (s.Q < 1 || s.Q > kMaxQ || s.q0 < 0 || s.q0 >= s.Q) return hipErrorInvalidValue;
  if (mode == 1 && !T) return hipErrorInvalidValue;
  const int64_t rpt = (s.m + kMscThreads - 1) / kMscThreads;
#define IE_M(R)                                                                                                     \
  return msc_launch<R>(s, mode, obs_domain, T, ldt, act, nact, act_out, nact_out, Bmax, V, ldv, h_ptr, h_idx, h_w, \
                       r_var, n_state, st)
  if (rpt <= 1) IE_M(1);
  if (rpt <= 2) IE_M(2);
  if (rpt <= 4) IE_M(4);
  if (rpt <= 8) IE_M(8);
  if (rpt <= 16) IE_M(16);
#undef IE_M
  return hipErrorInvalidValue;
}

}  // namespace infoesrf
