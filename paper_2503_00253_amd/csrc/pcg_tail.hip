// Persistent PCG: one launch iterates each listed system to the end.
//
// In the batched loop every PCG iteration costs two launches (the batched apply of S and the
// fused PCG step) and a round trip of x, r and p through HBM, whatever the number of live
// systems.  Here each workgroup takes a system from a work queue and iterates it to convergence
// on its own: the iterate, residual and direction stay in registers, the direction also in LDS,
// and the apply of S is done in place, from the explicit band of the localized covariance on the
// observed lattice or from the dense m x m S.  Each workgroup streams the band (or S) once per
// iteration from L2, so the apply trades L2 bandwidth for the launches and the HBM round trips;
// it pays when that matrix is small enough to stay in every XCD's L2.  The PCG step and the
// limited-memory preconditioner (Appendix E) are the same arithmetic as the fused step.  Every
// workgroup leaves when the queue is empty, and every system's loop ends at convergence,
// breakdown or the iteration cap.
//
// The band apply reads the direction from a padded copy of the observed lattice in LDS: bz rows
// above and below and bx columns left and right of the nz x nx lattice, holding the wrapped
// values along periodic axes (copied from the interior after each update) and zeros elsewhere,
// so the neighbour (z + li - bz, x + d - bx) of lattice point (z, x) sits at (z + li) Wp + x + d
// with no wrap or bounds test, and a thread walks a stencil row through consecutive LDS words.
// The band values are loaded a chunk at a time ahead of their use, to keep many loads in flight
// per wavefront.
#include <atomic>

#include "internal.hpp"

namespace infoesrf {

namespace {

constexpr int kTailMaxM = 4096;
// dynamic LDS for the (padded) direction, in doubles
constexpr int64_t kTailPadMax = 6144;

// Workgroup sums of Wn values per thread: DPP sums in a wavefront, then the NT / 64 wavefront
// partials in order (a fixed tree: bit-reproducible).  tail_sum1 returns its one sum to every
// thread; tail_sums writes sum j to out_lds[j] (thread j) and returns after a second barrier.
// sred must not be rewritten before every thread has passed a later barrier.
template <int Wn, int NT>
__device__ inline void tail_partials(const double* v, double (*sred)[NT / 64]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < Wn; ++j) {
    const double x = wave_sum_dpp(v[j]);
    if (lane == 63) sred[j][wave] = x;
  }
  __syncthreads();
}

template <int NT>
__device__ inline double tail_sum1(double v, double (*sred)[NT / 64]) {
  tail_partials<1, NT>(&v, sred);
  double t = sred[0][0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) t += sred[0][w];
  return t;
}

// The same sums through LDS when the workgroup's Wn x NT partials fit: every thread stores its
// Wn values, then 16 threads per value add NT / 16 partials each (a fixed order) and a row of 16
// lanes combines them by DPP.  Fewer cross-lane steps than Wn wavefront sums.
__host__ __device__ constexpr bool tail_lds_sums(int Wn, int NT) { return Wn > 1 && Wn * NT * 8 <= 96 * 1024; }

template <int Wn, int NT>
__device__ inline void tail_sums_lds(const double* v, double* part, double* out_lds) {
  constexpr int G = 16;
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < Wn; ++j) part[j * NT + tid] = v[j];
  __syncthreads();
  for (int u = tid; u < Wn * G; u += NT) {  // whole rows of 16 lanes stay active together
    const int j = u / G, c = u % G;
    const double* pj = part + j * NT + c;
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < NT / G; ++k) t += pj[G * k];
    t += dpp_f64<0xB1, 0xF>(t);   // quad_perm [1,0,3,2]
    t += dpp_f64<0x4E, 0xF>(t);   // quad_perm [2,3,0,1]
    t += dpp_f64<0x141, 0xF>(t);  // row_half_mirror
    t += dpp_f64<0x140, 0xF>(t);  // row_mirror
    if (c == 0) out_lds[j] = t;
  }
  __syncthreads();
}

template <int Wn, int NT>
__device__ inline void tail_sums(const double* v, double (*sred)[NT / 64], double* out_lds) {
  tail_partials<Wn, NT>(v, sred);
  if ((int)threadIdx.x < Wn) {
    const int j = threadIdx.x;
    double t = sred[j][0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) t += sred[j][w];
    out_lds[j] = t;
  }
  __syncthreads();
}

// Raw buffer loads: a descriptor over the whole array (reads past its end return zero), a
// per-lane byte offset in one vector register and a uniform byte offset in a scalar register, so
// holding a load's address across iterations costs no more than its row's offset.
__device__ inline __amdgpu_buffer_rsrc_t tail_rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ inline double tail_ld8(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
}

// Whether the kernel keeps the thread's rows of the Ritz bases in registers.
__host__ __device__ constexpr bool tail_caches_ritz(int P, int RPT, int NT) {
  return P > 0 && RPT * P <= 20 && NT < 1024;
}

// Rows of a thread: pairs of adjacent rows, 2 (tid + NT jj) + b for jj < RPT / 2, b in {0, 1}, so
// that one 16-byte load brings a band entry of both rows.
template <int NT>
__device__ inline int tail_row(int tid, int j) {
  return 2 * (tid + NT * (j >> 1)) + (j & 1);
}

__device__ inline double2 tail_ld16(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
}

// Lane l's value of a double, to every lane.
__device__ inline double tail_readlane(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Halo cell t (of the nh cells that hold wrapped values) of the padded lattice: sets its position
// and that of the interior cell it copies; false where the cell stays zero (a corner past an axis
// that is not periodic).  Cells first along periodic z (2 bz rows of Wp), then along periodic x
// (nz rows of 2 bx).  bz <= nz and bx <= nx along periodic axes (checked by the launcher).
__device__ inline bool tail_halo(const Grid& g, int Wp, int t, int& dst, int& src) {
  const int nzh = g.pz ? 2 * g.bz * Wp : 0;
  int zz, xx;
  if (t < nzh) {
    const int row = t / Wp;
    zz = row < g.bz ? row : row + g.nz;
    xx = t % Wp;
  } else {
    const int t2 = t - nzh, c = t2 % (2 * g.bx);
    zz = g.bz + t2 / (2 * g.bx);
    xx = c < g.bx ? c : c + g.nx;
  }
  int z = zz - g.bz, x = xx - g.bx;
  if (z < 0) z += g.nz;
  else if (z >= g.nz) z -= g.nz;
  if (x < 0 || x >= g.nx) {
    if (!g.px) return false;
    x = x < 0 ? x + g.nx : x - g.nx;
  }
  dst = zz * Wp + xx;
  src = (z + g.bz) * Wp + x + g.bx;
  return true;
}

template <int P, int RPT, int NT>
__global__ __launch_bounds__(NT) void k_pcg_tail(PCGState st, LMP lmp, TailApply ap,
                                                 const int32_t* __restrict__ act, const int32_t* __restrict__ nact,
                                                 int32_t* __restrict__ qctr, int phi_lds,
                                                 const double* __restrict__ r0, double* __restrict__ uacc,
                                                 TailCheck chk) {
  constexpr int W = 2 * P + 1;
  constexpr int NW = NT / 64;
  static_assert(RPT % 2 == 0, "rows come in pairs");
  // band (or S) entries per chunk: RPT / 2 * CH 16-byte loads in flight per thread
  constexpr int CH = RPT >= 4 ? 8 : 16;
  // the Ritz vectors of the thread's rows stay in registers when they fit
  constexpr bool kCache = tail_caches_ritz(P, RPT, NT);
  constexpr bool kLdsSums = tail_lds_sums(2 * P + 1, NT);
  constexpr int kC = kCache ? RPT * P : 1;
  __shared__ double sred1[1][NW];
  __shared__ double sredW[W][NW];
  __shared__ double sG[3 * P * P + P + 1];
  __shared__ double scoef[2 * P + 2];
  __shared__ double sM[P * P + 1];
  __shared__ double sdot[W];
  __shared__ int s_idx;
  // padded direction (band) or direction (dense S); then, when phi_lds, the Ritz bases
  extern __shared__ double sp[];
  const int tid = threadIdx.x;
  const int64_t m = st.m;
  const bool band = ap.kind == 0;
  const Grid g = ap.g;
  const int w = 2 * g.bx + 1, h = 2 * g.bz + 1;
  const int Wp = band ? g.nx + 2 * g.bx : 0;
  const int npad = band ? (g.nz + 2 * g.bz) * Wp : (int)m;
  // halo cells holding wrapped values
  const int nh = band ? (g.pz ? 2 * g.bz * Wp : 0) + (g.px ? g.nz * 2 * g.bx : 0) : 0;
  // stencil rows and entries per stencil row of the apply (the dense S: one row of m)
  const int hh = band ? h : 1, ww = band ? w : (int)m;
  if (P > 0) {
    for (int o = tid; o < 3 * P * P; o += NT) sG[o] = lmp.G[o];
    if (tid < P) sG[3 * P * P + tid] = lmp.theta[tid];
  }
  // zeros in the halo along axes that are not periodic (never rewritten)
  for (int o = tid; o < npad; o += NT) sp[o] = 0.0;
  const double dmin = (P > 0) ? *lmp.dmin : 0.0;
  const int na = *nact;
  // descriptors of the band (or S) and the Ritz bases; byte strides of their columns
  const __amdgpu_buffer_rsrc_t rsA =
      band ? tail_rsrc(ap.band, (int64_t)h * w * ap.ldb * 8) : tail_rsrc(ap.S, m * ap.lds * 8);
  const uint32_t colA = (uint32_t)((band ? ap.ldb : ap.lds) * 8);
  const __amdgpu_buffer_rsrc_t rsF = tail_rsrc(lmp.Phi, (int64_t)P * lmp.ld * 8);
  const __amdgpu_buffer_rsrc_t rsG = tail_rsrc(lmp.SPhi, (int64_t)P * lmp.ld * 8);
  const uint32_t colF = (uint32_t)(lmp.ld * 8);
  double* part = sp + npad;                           // W x NT partial sums
  double* sF = part + (kLdsSums ? W * NT : 0);        // Phi (P x m), when phi_lds
  double* sH = sF + (int64_t)P * m;                   // S Phi (P x m)
  if (phi_lds) {
    for (int o = tid; o < P * (int)m; o += NT) {
      const int l = o / (int)m, r = o % (int)m;
      sF[o] = tail_ld8(rsF, (uint32_t)r * 8, l * colF);
      sH[o] = tail_ld8(rsG, (uint32_t)r * 8, l * colF);
    }
  }
  // the corner of each row's stencil in the padded grid, and the row's byte offset in a column
  int corner[RPT];
  uint32_t roff[RPT / 2];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int r = tail_row<NT>(tid, j);
    corner[j] = (band && r < m) ? (r / g.nx) * Wp + r % g.nx : 0;
  }
  // byte offset of each pair in a column (pairs past m read the last pair and are discarded;
  // an odd m leaves its last pair one row into the column's padding, ld >= m + 1)
#pragma unroll
  for (int jj = 0; jj < RPT / 2; ++jj)
    roff[jj] = (uint32_t)min<int64_t>(tail_row<NT>(tid, 2 * jj), (m - 1) & ~(int64_t)1) * (uint32_t)sizeof(double);
  // q = (1 + sigma) v + S v for the thread's rows: v to LDS (and its wrapped copies), then the
  // band (or S) streamed from L2 against it
  auto apply_C = [&](const double* v, double sig1, double* qv) {
    // the direction into LDS, then its wrapped copies
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int r = tail_row<NT>(tid, j);
      if (r < m) sp[band ? corner[j] + g.bz * Wp + g.bx : r] = v[j];
    }
    __syncthreads();
    if (nh > 0) {
      for (int t = tid; t < nh; t += NT) {
        int dst, src;
        if (tail_halo(g, Wp, t, dst, src)) sp[dst] = sp[src];
      }
      __syncthreads();
    }
    // q = (1 + sigma) v + S v
    // A row of the band is h stencil rows of w consecutive entries, both in the band (columns
    // of colA bytes) and in the padded direction; the dense S is one stencil row of m entries.
    // Each stencil row goes in chunks of CH entries whose loads, for all the thread's row
    // pairs, are issued ahead of their multiply-adds (16 bytes a lane: the entry for both rows
    // of a pair; uniform column offsets in scalar registers, the pair a per-lane offset, the
    // direction at immediate LDS offsets), then one chunk for the rest of the row, whose
    // missing entries repeat the last one and are weighted by zero.
#pragma unroll
    for (int j = 0; j < RPT; ++j) qv[j] = 0.0;
    for (int li = 0; li < hh; ++li) {
      uint32_t so = (uint32_t)(li * ww) * colA;
      const int lrow = li * Wp;
      int d0 = 0;
      for (; d0 + CH <= ww; d0 += CH) {
        double2 bv[RPT / 2][CH];
#pragma unroll
        for (int jj = 0; jj < RPT / 2; ++jj)
#pragma unroll
          for (int k = 0; k < CH; ++k) bv[jj][k] = tail_ld16(rsA, roff[jj], so + (uint32_t)k * colA);
#pragma unroll
        for (int jj = 0; jj < RPT / 2; ++jj) {
          const double* p0 = sp + corner[2 * jj] + lrow + d0;
          const double* p1 = sp + corner[2 * jj + 1] + lrow + d0;
#pragma unroll
          for (int k = 0; k < CH; ++k) {
            qv[2 * jj] += bv[jj][k].x * p0[k];
            qv[2 * jj + 1] += bv[jj][k].y * p1[k];
          }
        }
        so += (uint32_t)CH * colA;
      }
      if (d0 < ww) {
        const int last = ww - d0 - 1;
        double2 bv[RPT / 2][CH];
#pragma unroll
        for (int jj = 0; jj < RPT / 2; ++jj)
#pragma unroll
          for (int k = 0; k < CH; ++k) bv[jj][k] = tail_ld16(rsA, roff[jj], so + (uint32_t)min(k, last) * colA);
#pragma unroll
        for (int jj = 0; jj < RPT / 2; ++jj) {
          const double* p0 = sp + corner[2 * jj] + lrow + d0;
          const double* p1 = sp + corner[2 * jj + 1] + lrow + d0;
#pragma unroll
          for (int k = 0; k < CH; ++k) {
            const int kk = min(k, last);
            qv[2 * jj] += (k <= last ? bv[jj][k].x : 0.0) * p0[kk];
            qv[2 * jj + 1] += (k <= last ? bv[jj][k].y : 0.0) * p1[kk];
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j) qv[j] += sig1 * v[j];
  };
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
    // a start (r0 given) takes x = 0 and the residual r0 and begins with the first step's
    // preconditioned residual; a continuation reads x, r, p and r^T z of the batched loop
    const bool start = r0 != nullptr;
    double rz = start ? 0.0 : st.rz[s];
    int it = st.iters[s];
    double rv[RPT], pv[RPT], xv[RPT];
    double ph[kC], sph[kC];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int64_t r = tail_row<NT>(tid, j);
      const bool ok = r < m;
      rv[j] = ok ? (start ? r0[base + r] : st.r[base + r]) : 0.0;
      pv[j] = (ok && !start) ? st.p[base + r] : 0.0;
      xv[j] = (ok && !start) ? st.x[base + r] : 0.0;
      if (kCache) {
#pragma unroll
        for (int l = 0; l < P; ++l) {
          ph[(j * P + l) % kC] = ok ? tail_ld8(rsF, (uint32_t)r * 8, l * colF) : 0.0;
          sph[(j * P + l) % kC] = ok ? tail_ld8(rsG, (uint32_t)r * 8, l * colF) : 0.0;
        }
      }
    }
    // M(sigma) = (C Phi)^T (C Phi) = Gss + sigma (Gps + Gps^T) + sigma^2 Gpp for this system's shift
    // (read after the first iteration's barriers)
    if (P > 0) {
      const double* Gpp = sG;
      const double* Gps = sG + P * P;
      const double* Gss = sG + 2 * P * P;
      for (int o = tid; o < P * P; o += NT) {
        const int a = o / P, l = o % P;
        sM[o] = Gss[a * P + l] + sig1 * (Gps[a * P + l] + Gps[l * P + a]) + sig1 * sig1 * Gpp[a * P + l];
      }
    }
    int state = 0;
    double relres = 0.0;
    bool first = start;
    for (;;) {
      if (!first) {  // the apply and the step (the first pass of a start only prepares p)
        double qv[RPT];
        apply_C(pv, sig1, qv);
        double pq = 0.0;
#pragma unroll
        for (int j = 0; j < RPT; ++j) pq += pv[j] * qv[j];
        const double tot = tail_sum1<NT>(pq, sred1);
        if (!(tot > 0.0) || !isfinite(tot)) {
          if (tid == 0) atomicOr(st.flags, isfinite(tot) ? kFlagNotSPD : kFlagNumeric);
          state = 2;
          break;
        }
        const double alpha = rz / tot;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          if (tail_row<NT>(tid, j) < m) {
            xv[j] += alpha * pv[j];
            rv[j] -= alpha * qv[j];
          }
        }
        ++it;
      }  // !first
      // dots of r: r^T r, Phi^T r, (S Phi)^T r
      double acc[W];
#pragma unroll
      for (int j = 0; j < W; ++j) acc[j] = 0.0;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int64_t r = tail_row<NT>(tid, j);
        if (r < m) {
          acc[0] += rv[j] * rv[j];
#pragma unroll
          for (int l = 0; l < P; ++l) {
            const double a = kCache ? ph[(j * P + l) % kC]
                                    : (phi_lds ? sF[l * m + r] : tail_ld8(rsF, (uint32_t)r * 8, l * colF));
            const double b = kCache ? sph[(j * P + l) % kC]
                                    : (phi_lds ? sH[l * m + r] : tail_ld8(rsG, (uint32_t)r * 8, l * colF));
            acc[1 + l] += a * rv[j];
            acc[1 + P + l] += b * rv[j];
          }
        }
      }
      if (kLdsSums) tail_sums_lds<W, NT>(acc, part, sdot);
      else tail_sums<W, NT>(acc, sredW, sdot);
      const double* dt = sdot;
      const double rn = sqrt(dt[0]);
      relres = bn > 0.0 ? rn / bn : 0.0;
      if (!isfinite(dt[0])) {
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
      // The first wavefront does it without a barrier: lane t < p holds c1_t, takes the others'
      // by readlane for (C Phi)^T (C Phi) c1 = M(sigma) c1 (M precomputed per system), and the
      // wavefront sums the p terms of r^T z's correction.
      double rzn = dt[0];
      if (P > 0) {
        if (tid < 64) {
          const double* sth = sG + 3 * P * P;
          double c1 = 0.0, term = 0.0;
          if (tid < P) c1 = dt[1 + tid] / (sig1 + sth[tid]);
          double mc = 0.0;
#pragma unroll
          for (int l = 0; l < P; ++l) {
            const double c1l = tail_readlane(c1, l);
            if (tid < P) mc += sM[tid * P + l] * c1l;
          }
          if (tid < P) {
            const double c2 = (dt[1 + P + tid] + sig1 * dt[1 + tid] - mc) / (sig1 + sth[tid]);
            const double beta_l = sig1 + dmin;
            const double gam = (sig1 - beta_l) * c1 + c2;
            scoef[tid] = c1;
            scoef[P + tid] = gam;
            term = dt[1 + P + tid] * c1 + dt[1 + tid] * gam;
          }
          const double tsum = wave_sum_dpp(term);
          if (tid == 63) scoef[2 * P] = tsum;
        }
        __syncthreads();
        rzn -= scoef[2 * P];
      }
      if (!(rzn > 0.0) || !isfinite(rzn)) {
        if (tid == 0) atomicOr(st.flags, isfinite(rzn) ? kFlagNotSPD : kFlagNumeric);
        state = 2;
        break;
      }
      const double beta = first ? 0.0 : rzn / rz;
      rz = rzn;
      first = false;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int64_t r = tail_row<NT>(tid, j);
        if (r < m) {
          double z = rv[j];
#pragma unroll
          for (int l = 0; l < P; ++l) {
            const double a = kCache ? ph[(j * P + l) % kC]
                                    : (phi_lds ? sF[l * m + r] : tail_ld8(rsF, (uint32_t)r * 8, l * colF));
            const double b = kCache ? sph[(j * P + l) % kC]
                                    : (phi_lds ? sH[l * m + r] : tail_ld8(rsG, (uint32_t)r * 8, l * colF));
            z -= b * scoef[l] + a * scoef[P + l];
          }
          pv[j] = z + beta * pv[j];
        }
      }
      // no barrier here: every thread read the LDS direction before the first reduction's
      // barrier, and sred1, sredW, sdot and scoef are rewritten only after the next direction's
    }
    // a start adds its correction to the solution; a continuation hands x, r, p back to the
    // batched loop, which adds x
    double un[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int64_t r = tail_row<NT>(tid, j);
      un[j] = 0.0;
      if (r < m) {
        if (start) {
          un[j] = uacc[base + r] + xv[j];
          uacc[base + r] = un[j];
        } else {
          st.x[base + r] = xv[j];
          st.r[base + r] = rv[j];
          st.p[base + r] = pv[j];
        }
      }
    }
    // the sweep's check of the new u: r = b - (1 + sigma) u - S u in FP64, kept for a further
    // sweep, and the status from ||r|| / ||b|| (every thread has left the loop's last LDS reads
    // behind the reductions' barriers)
    const bool check = start && chk.b != nullptr;
    double rr = 0.0;
    if (check) {
      double qv[RPT];
      apply_C(un, sig1, qv);
      double r2 = 0.0;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int64_t r = tail_row<NT>(tid, j);
        if (r < m) {
          const double rt = chk.b[base + r] - qv[j];
          st.r[base + r] = rt;
          r2 += rt * rt;
        }
      }
      const double rn = sqrt(tail_sum1<NT>(r2, sred1));
      rr = bn > 0.0 ? rn / bn : 0.0;
    }
    if (tid == 0) {
      if (st.prof.vectors) {
        const int done_its = it - st.iters[s];
        atomicAdd(st.prof.vectors, (unsigned long long)done_its);
        atomicAdd(st.prof.flops, (double)(done_its + (check ? 1 : 0)) * st.prof.flops_per_vector);
        atomicAdd(st.prof.bytes, st.prof.bytes_per_vector);
      }
      st.rz[s] = rz;
      st.iters[s] = it;
      if (!check) {
        st.relres[s] = relres;
        st.done[s] = state;
      } else {
        chk.sweeps[s] += 1;
        st.relres[s] = relres;
        chk.relres[s] = rr;
        if (!isfinite(rr)) {
          atomicOr(st.flags, kFlagNumeric);
          chk.fdone[s] = 2;
          st.done[s] = 1;
        } else if (rr <= chk.rtol) {
          chk.fdone[s] = 1;
          st.done[s] = 1;
        } else if (it >= st.max_iter) {
          chk.fdone[s] = chk.fixed ? 3 : 2;
          st.done[s] = 1;
        } else {
          st.done[s] = 0;
          st.thresh[s] = chk.fixed ? 0.0 : 0.5 * chk.rtol * bn;
        }
      }
    }
    __syncthreads();
  }
}

// The live systems (done == 0) node by node in order of increasing shift (the slowest first),
// members in order within a node: systems s = q G + i with one shift per group of G.  One
// workgroup: the Q = S / G node shifts are ranked in LDS (ties by node index), then the systems
// are compacted in that order (per-thread chunks and a workgroup scan of their counts).
constexpr int kOrderQ = 4096;
__global__ __launch_bounds__(1024) void k_order_live(const int32_t* __restrict__ done,
                                                     const double* __restrict__ sigma, int64_t S, int64_t G,
                                                     int32_t* __restrict__ act, int32_t* __restrict__ nact,
                                                     int32_t* __restrict__ qctr) {
  __shared__ int32_t perm[kOrderQ];
  __shared__ int swave[16];
  __shared__ int total;
  const int t = threadIdx.x;
  const int Q = (int)(S / G);
  for (int q = t; q < Q; q += 1024) {
    const double kq = sigma[(int64_t)q * G];
    int rank = 0;
    for (int j = 0; j < Q; ++j) {
      const double kj = sigma[(int64_t)j * G];
      rank += (kj < kq || (kj == kq && j < q)) ? 1 : 0;
    }
    perm[rank] = q;
  }
  __syncthreads();
  const int64_t per = (S + 1023) / 1024;
  const int64_t a = t * per, b = min<int64_t>(S, a + per);
  int32_t c = 0;
  for (int64_t u = a; u < b; ++u) c += (done[(int64_t)perm[u / G] * G + u % G] == 0);
  int32_t pos = block_exclusive_scan<1024>(c, swave, &total);
  if (t == 0) {
    *nact = total;
    if (qctr) *qctr = 0;
  }
  for (int64_t u = a; u < b; ++u) {
    const int64_t sys = (int64_t)perm[u / G] * G + u % G;
    if (done[sys] == 0) act[pos++] = (int32_t)sys;
  }
}

// two rows a thread (one pair) up to 1024 rows, on 128, 256 or 512 threads; four rows on 512 or
// 1024 threads beyond
int tail_threads(int64_t m) { return m > 2048 ? 1024 : (m > 512 ? 512 : (m > 256 ? 256 : 128)); }

size_t tail_lds_bytes(const TailApply& ap) {
  const int64_t npad = ap.kind == 0 ? (int64_t)(ap.g.nz + 2 * ap.g.bz) * (ap.g.nx + 2 * ap.g.bx) : ap.m;
  return (size_t)npad * sizeof(double);
}

// LDS (static and dynamic) the launcher lets one workgroup take: the kernel runs one workgroup
// per CU at the sizes where it needs this much
constexpr size_t kTailLdsBig = 150 * 1024;

template <int P, int RPT, int NT>
hipError_t tail_go(const PCGState& s, const LMP& lmp, const TailApply& ap, const int32_t* act, const int32_t* nact,
                   int32_t* qctr, int64_t grid, const double* r0, double* uacc, const TailCheck& chk,
                   hipStream_t st) {
  if ((int64_t)RPT * NT < s.m) return hipErrorInvalidValue;  // every row has a thread
  const void* fn = (const void*)k_pcg_tail<P, RPT, NT>;
  // the kernel's static LDS (read once per instantiation): static + dynamic stays within the CU's
  static std::atomic<size_t> stat_lds{~(size_t)0};
  size_t stat = stat_lds.load();
  if (stat == ~(size_t)0) {
    hipFuncAttributes fa{};
    const hipError_t e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess) return e;
    stat = fa.sharedSizeBytes;
    stat_lds.store(stat);
  }
  size_t lds = tail_lds_bytes(ap);
  if (tail_lds_sums(2 * P + 1, NT)) lds += (size_t)(2 * P + 1) * NT * sizeof(double);
  if (stat + lds > kTailLdsBig) return hipErrorInvalidValue;
  // the Ritz bases in LDS when the kernel does not keep them in registers and there is room
  const size_t phi = (size_t)16 * P * s.m;
  const int phi_lds = (P > 0 && !tail_caches_ritz(P, RPT, NT) && stat + lds + phi <= kTailLdsBig) ? 1 : 0;
  if (phi_lds) lds += phi;
  // dynamic LDS this instantiation may take (concurrent first calls raise it twice: harmless)
  static std::atomic<size_t> allowed{64 * 1024};
  if (lds > allowed.load()) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    allowed.store(lds);
  }
  // no more workgroups than can be resident at once: the others would only find the queue empty
  int dev = 0, per_cu = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, lds);
  if (e != hipSuccess) return e;
  const int64_t resident = std::max<int64_t>((int64_t)per_cu * cus, 1);
  const dim3 gdim((unsigned)std::max<int64_t>(std::min(grid, resident), 1)), b(NT);
  hipLaunchKernelGGL((k_pcg_tail<P, RPT, NT>), gdim, b, lds, st, s, lmp, ap, act, nact, qctr, phi_lds, r0, uacc,
                     chk);
  return hipGetLastError();
}

template <int P>
hipError_t tail_rows(const PCGState& s, const LMP& lmp, const TailApply& ap, const int32_t* act, const int32_t* nact,
                     int32_t* qctr, int64_t grid, const double* r0, double* uacc, const TailCheck& chk,
                     hipStream_t st) {
  const int nt = tail_threads(s.m);
  const int64_t rpt = (s.m + nt - 1) / nt;
  if (nt == 128) return tail_go<P, 2, 128>(s, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
  if (nt == 256) return tail_go<P, 2, 256>(s, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
  if (nt == 1024) return tail_go<P, 4, 1024>(s, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
  if (rpt <= 2) return tail_go<P, 2, 512>(s, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
  if (rpt <= 4) return tail_go<P, 4, 512>(s, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
  return hipErrorInvalidValue;
}

}  // namespace

bool tail_fits(const TailApply& ap) {
  if (ap.m < 1 || ap.m > kTailMaxM) return false;
  if (ap.kind == 0) {
    const Grid& g = ap.g;
    if (g.nz < 1 || g.nx < 1 || (int64_t)g.nz * g.nx != ap.m || g.bz < 0 || g.bx < 0) return false;
    // one wrapped copy per side along a periodic axis
    if ((g.pz && g.bz > g.nz) || (g.px && g.bx > g.nx)) return false;
  }
  return (int64_t)(tail_lds_bytes(ap) / sizeof(double)) <= kTailPadMax;
}

hipError_t launch_order_live(const int32_t* done, const double* sigma, int64_t S, int64_t G, int32_t* act,
                             int32_t* nact, int32_t* qctr, hipStream_t st) {
  if (!done || !sigma || !act || !nact || G < 1 || S < 1 || S % G != 0 || S / G > kOrderQ)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_order_live, dim3(1), dim3(1024), 0, st, done, sigma, S, G, act, nact, qctr);
  return hipGetLastError();
}

hipError_t launch_pcg_tail(const PCGState& s, const LMP& lmp, const TailApply& ap, const int32_t* act,
                           const int32_t* nact, int32_t* qctr, int64_t grid, const double* r0, double* uacc,
                           const TailCheck& chk, hipStream_t st) {
  if (s.m < 1 || s.m > kTailMaxM || s.m != ap.m || !act || !nact || !qctr || !tail_fits(ap) ||
      ((r0 == nullptr) != (uacc == nullptr)) || (chk.b && (!r0 || !chk.fdone || !chk.sweeps || !chk.relres)))
    return hipErrorInvalidValue;
  if (ap.kind == 0 && !ap.band) return hipErrorInvalidValue;
  if (ap.kind == 1 && !ap.S) return hipErrorInvalidValue;
  if (lmp.p > 0 && (!lmp.Phi || !lmp.SPhi || !lmp.G || !lmp.theta || !lmp.dmin)) return hipErrorInvalidValue;
  switch (lmp.p) {
    case 0: return tail_rows<0>(s, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
    case 4: return tail_rows<4>(s, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
    case 8: return tail_rows<8>(s, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
    case 10: return tail_rows<10>(s, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
    case 12: return tail_rows<12>(s, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
    case 16: return tail_rows<16>(s, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
    case 20: return tail_rows<20>(s, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace infoesrf
