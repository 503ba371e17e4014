// Persistent finish of the batched PCG: once few systems are left, one launch finishes them.
//
// After most of the Q N systems have converged, the last ones (the smallest shifts) still need
// tens of iterations, and every iteration costs two launches (the batched apply of S and the
// fused PCG step) whose fixed latency no longer shrinks with the work.  Here each workgroup takes
// a system from a work queue and iterates it to convergence on its own: its direction lives in
// LDS, its iterate and residual in registers, and the apply of S is done in place, from the
// explicit band of the localized covariance on the observed lattice or from the dense m x m S.
// The PCG step and the limited-memory preconditioner (Appendix E) are the same arithmetic as the
// fused step.  Every workgroup leaves when the queue is empty, and every system's loop ends at
// convergence, breakdown or the iteration cap.
#include "internal.hpp"

namespace infoesrf {

namespace {

constexpr int kTailThreads = 256;
constexpr int kTailMaxM = 4096;

__device__ inline int tail_wrap(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

// Workgroup sums of W values per thread (shuffles in a wavefront, the four wavefronts in order),
// written once to LDS.
template <int W>
__device__ inline void tail_sum(const double* v, double (*sred)[4], double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    double x = v[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) sred[j][wave] = x;
  }
  __syncthreads();
  if ((int)threadIdx.x < W) {
    const int j = threadIdx.x;
    out[j] = ((sred[j][0] + sred[j][1]) + sred[j][2]) + sred[j][3];
  }
  __syncthreads();
}

// (S p)_r with p in LDS: banded product on the observed lattice, or row r of the dense S.
__device__ inline double tail_apply_row(const TailApply& ap, const double* sp, int64_t r) {
  double acc = 0.0;
  if (ap.kind == 1) {
    for (int64_t k = 0; k < ap.m; ++k) acc += ap.S[k * ap.lds + r] * sp[k];
    return acc;
  }
  const Grid& g = ap.g;
  const int z = (int)(r / g.nx), x = (int)(r % g.nx);
  const int w = 2 * g.bx + 1;
  for (int li = 0; li < 2 * g.bz + 1; ++li) {
    int zz = z + li - g.bz;
    if (g.pz) zz = tail_wrap(zz, g.nz);
    else if (zz < 0 || zz >= g.nz) continue;
    const double* brow = ap.band + (int64_t)(li * w) * ap.ldb + r;
    const double* prow = sp + (int64_t)zz * g.nx;
    for (int d = 0; d < w; ++d) {
      int kx = x - g.bx + d;
      if (g.px) kx = tail_wrap(kx, g.nx);
      else if (kx < 0 || kx >= g.nx) continue;  // the band entry is 0 there
      acc += brow[(int64_t)d * ap.ldb] * prow[kx];
    }
  }
  return acc;
}

template <int P, int RPT>
__global__ __launch_bounds__(kTailThreads) void k_pcg_tail(PCGState st, LMP lmp, TailApply ap,
                                                           const int32_t* __restrict__ act,
                                                           const int32_t* __restrict__ nact,
                                                           int32_t* __restrict__ qctr) {
  constexpr int W = 2 * P + 1;
  __shared__ double sred[W][4];
  __shared__ double sG[3 * P * P + P + 1];
  __shared__ double scoef[2 * P + 2];
  __shared__ double sdot[W];
  __shared__ double sp[kTailMaxM];
  __shared__ int s_idx;
  const int tid = threadIdx.x;
  const int64_t m = st.m;
  if (P > 0) {
    for (int o = tid; o < 3 * P * P; o += kTailThreads) sG[o] = lmp.G[o];
    if (tid < P) sG[3 * P * P + tid] = lmp.theta[tid];
  }
  const double dmin = (P > 0) ? *lmp.dmin : 0.0;
  const int na = *nact;
  __syncthreads();
  for (;;) {
    if (tid == 0) s_idx = atomicAdd(qctr, 1);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();  // every thread has read s_idx before it is written again
    if (idx >= na) break;
    const int32_t s = act[idx];
    if (st.done[s] != 0) continue;
    const int64_t base = (int64_t)s * st.ld;
    const double sig1 = 1.0 + st.sigma[s];
    const double bn = st.bnorm[s];
    const double thresh = st.thresh[s];
    double rz = st.rz[s];
    int it = st.iters[s];
    double rv[RPT], pv[RPT], xv[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int64_t r = tid + kTailThreads * j;
      const bool ok = r < m;
      rv[j] = ok ? st.r[base + r] : 0.0;
      pv[j] = ok ? st.p[base + r] : 0.0;
      xv[j] = ok ? st.x[base + r] : 0.0;
    }
    int state = 0;
    double relres = 0.0;
    for (;;) {
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int64_t r = tid + kTailThreads * j;
        if (r < m) sp[r] = pv[j];
      }
      __syncthreads();
      double qv[RPT];
      double pq = 0.0;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int64_t r = tid + kTailThreads * j;
        qv[j] = 0.0;
        if (r < m) {
          qv[j] = sig1 * pv[j] + tail_apply_row(ap, sp, r);
          pq += pv[j] * qv[j];
        }
      }
      double tot[1];
      tail_sum<1>(&pq, sred, sdot);
      tot[0] = sdot[0];
      if (!(tot[0] > 0.0) || !isfinite(tot[0])) {
        if (tid == 0) atomicOr(st.flags, isfinite(tot[0]) ? kFlagNotSPD : kFlagNumeric);
        state = 2;
        break;
      }
      const double alpha = rz / tot[0];
      double acc[W];
#pragma unroll
      for (int j = 0; j < W; ++j) acc[j] = 0.0;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int64_t r = tid + kTailThreads * j;
        if (r < m) {
          xv[j] += alpha * pv[j];
          rv[j] -= alpha * qv[j];
          acc[0] += rv[j] * rv[j];
#pragma unroll
          for (int l = 0; l < P; ++l) {
            acc[1 + l] += (double)lmp.Phi32[l * lmp.ld + r] * rv[j];
            acc[1 + P + l] += (double)lmp.SPhi32[l * lmp.ld + r] * rv[j];
          }
        }
      }
      ++it;
      __syncthreads();  // sdot is rewritten below
      tail_sum<W>(acc, sred, sdot);
      const double rn = sqrt(sdot[0]);
      relres = bn > 0.0 ? rn / bn : 0.0;
      if (!isfinite(sdot[0])) {
        if (tid == 0) atomicOr(st.flags, kFlagNumeric);
        state = 2;
        break;
      }
      if (rn <= thresh) {
        state = 1;
        break;
      }
      if (it >= st.max_iter) {
        state = 2;
        break;
      }
      // limited-memory preconditioner coefficients, as in the fused step:
      //   c1 = Theta^{-1} Phi^T r,  c2 = Theta^{-1} [(C Phi)^T r - (C Phi)^T (C Phi) c1],
      //   gamma = (1 + sigma - beta_L) c1 + c2,  z = r - S Phi c1 - Phi gamma
      double rzn = sdot[0];
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
        for (int l = 0; l < P; ++l) rzn -= sdot[1 + P + l] * scoef[l] + sdot[1 + l] * scoef[P + l];
      }
      if (!(rzn > 0.0) || !isfinite(rzn)) {
        if (tid == 0) atomicOr(st.flags, isfinite(rzn) ? kFlagNotSPD : kFlagNumeric);
        state = 2;
        break;
      }
      const double beta = rzn / rz;
      rz = rzn;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int64_t r = tid + kTailThreads * j;
        if (r < m) {
          double z = rv[j];
#pragma unroll
          for (int l = 0; l < P; ++l)
            z -= (double)lmp.SPhi32[l * lmp.ld + r] * scoef[l] + (double)lmp.Phi32[l * lmp.ld + r] * scoef[P + l];
          pv[j] = z + beta * pv[j];
        }
      }
      __syncthreads();  // the LDS direction and scoef are rewritten in the next iteration
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int64_t r = tid + kTailThreads * j;
      if (r < m) {
        st.x[base + r] = xv[j];
        st.r[base + r] = rv[j];
        st.p[base + r] = pv[j];
      }
    }
    if (tid == 0) {
      st.rz[s] = rz;
      st.iters[s] = it;
      st.relres[s] = relres;
      st.done[s] = state;
    }
    __syncthreads();
  }
}

template <int P>
hipError_t tail_rows(const PCGState& s, const LMP& lmp, const TailApply& ap, const int32_t* act, const int32_t* nact,
                     int32_t* qctr, int64_t grid, hipStream_t st) {
  const int64_t rpt = (s.m + kTailThreads - 1) / kTailThreads;
  const dim3 g((unsigned)std::max<int64_t>(grid, 1)), b(kTailThreads);
#define IE_T(R)                                                                            \
  do {                                                                                      \
    hipLaunchKernelGGL((k_pcg_tail<P, R>), g, b, 0, st, s, lmp, ap, act, nact, qctr);        \
    return hipGetLastError();                                                               \
  } while (0)
  if (rpt <= 1) IE_T(1);
  if (rpt <= 2) IE_T(2);
  if (rpt <= 4) IE_T(4);
  if (rpt <= 8) IE_T(8);
  if (rpt <= 16) IE_T(16);
#undef IE_T
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_pcg_tail(const PCGState& s, const LMP& lmp, const TailApply& ap, const int32_t* act,
                           const int32_t* nact, int32_t* qctr, int64_t grid, hipStream_t st) {
  if (s.m < 1 || s.m > kTailMaxM || !act || !nact || !qctr) return hipErrorInvalidValue;
  if (ap.kind == 0 && (!ap.band || (int64_t)ap.g.nz * ap.g.nx != s.m)) return hipErrorInvalidValue;
  if (ap.kind == 1 && (!ap.S || ap.m != s.m)) return hipErrorInvalidValue;
  if (lmp.p > 0 && (!lmp.Phi32 || !lmp.SPhi32 || !lmp.G || !lmp.theta || !lmp.dmin)) return hipErrorInvalidValue;
  switch (lmp.p) {
    case 0: return tail_rows<0>(s, lmp, ap, act, nact, qctr, grid, st);
    case 4: return tail_rows<4>(s, lmp, ap, act, nact, qctr, grid, st);
    case 8: return tail_rows<8>(s, lmp, ap, act, nact, qctr, grid, st);
    case 10: return tail_rows<10>(s, lmp, ap, act, nact, qctr, grid, st);
    case 12: return tail_rows<12>(s, lmp, ap, act, nact, qctr, grid, st);
    case 16: return tail_rows<16>(s, lmp, ap, act, nact, qctr, grid, st);
    case 20: return tail_rows<20>(s, lmp, ap, act, nact, qctr, grid, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace infoesrf
