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
#include <type_traits>

#include "internal.hpp"

namespace infoesrf {

namespace {

constexpr int kTailMaxM = 4096;
// dynamic LDS for the (padded) direction, in doubles
constexpr int64_t kTailPadMax = 6144;
// zeroed doubles after the padded direction: the packed FP32 band reads up to 3 entries past a
// stencil row's end
constexpr int kTailSlack = 4;

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

// Doubles between the partials of consecutive sums: NT and 16 more, so that the four 16-lane
// groups of a wavefront that add the partials of four sums read distinct LDS banks in each half
// wavefront (NT doubles apart they would all read the same banks).
__host__ __device__ constexpr int tail_part_stride(int NT) { return NT + 16; }
// Partials a sum keeps: one a thread, or with four rows a thread on 512 threads one per pair of
// lanes (added by one lane exchange first), which halves the area and leaves room in LDS for the
// Ritz bases that such a thread cannot keep in registers.
__host__ __device__ constexpr int tail_part_rows(int NT, int RPT) { return RPT >= 4 && NT <= 512 ? NT / 2 : NT; }

// The same sums through LDS when the workgroup's Wn rows of NT partials fit: every thread stores its
// Wn values, then 16 threads per value add NT / 16 partials each (a fixed order) and a row of 16
// lanes combines them by DPP.  Fewer cross-lane steps than Wn wavefront sums.
__host__ __device__ constexpr bool tail_lds_sums(int Wn, int NT, int RPT) {
  return Wn > 1 && Wn * tail_part_stride(tail_part_rows(NT, RPT)) * 8 <= 96 * 1024;
}

// One reduction an iteration (up to 4 Ritz pairs, where its 4p + 4 sums fit in LDS): the sums of
// the new direction's apply q (p^T q, q^T q, r^T q, Phi^T q, (S Phi)^T q) and of the current
// residual (r^T r, Phi^T r, (S Phi)^T r) in one pass; the next residual's dots follow from them
// and the step length.  Otherwise p^T q and the residual's dots are two reductions.
__host__ __device__ constexpr bool tail_merged(int P, int NT, int RPT) {
  return P <= 4 && tail_lds_sums(4 * P + 4, NT, RPT);
}
// Doubles a thread writes for the LDS sums (0: the sums go through wavefront partials).
__host__ __device__ constexpr int tail_sum_words(int P, int NT, int RPT) {
  return tail_merged(P, NT, RPT) ? 4 * P + 4 : (tail_lds_sums(2 * P + 1, NT, RPT) ? 2 * P + 1 : 0);
}

template <int Wn, int NT, int RPT>
__device__ inline void tail_sums_lds(const double* v, double* part, double* out_lds) {
  constexpr int G = 16;
  constexpr int ROWS = tail_part_rows(NT, RPT), ST = tail_part_stride(ROWS);
  const int tid = threadIdx.x;
  if constexpr (ROWS == NT) {
#pragma unroll
    for (int j = 0; j < Wn; ++j) part[j * ST + tid] = v[j];
  } else {
#pragma unroll
    for (int j = 0; j < Wn; ++j) {
      const double x = v[j] + dpp_f64<0xB1, 0xF>(v[j]);  // quad_perm [1,0,3,2]: this lane and its pair
      if ((tid & 1) == 0) part[j * ST + (tid >> 1)] = x;
    }
  }
  __syncthreads();
  for (int u = tid; u < Wn * G; u += NT) {  // whole rows of 16 lanes stay active together
    const int j = u / G, c = u % G;
    const double* pj = part + j * ST + c;
    // four independent chains (a fixed order), then their sum
    constexpr int KC = ROWS / G >= 8 ? 4 : 1;
    double tc[KC];
#pragma unroll
    for (int i = 0; i < KC; ++i) tc[i] = 0.0;
#pragma unroll
    for (int k = 0; k < ROWS / G; ++k) tc[k % KC] += pj[G * k];
    double t = tc[0];
#pragma unroll
    for (int i = 1; i < KC; ++i) t += tc[i];
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

// Whether the kernel keeps the thread's rows of the Ritz bases in registers (2 RPT P doubles):
// with two rows a thread up to 10 pairs; four rows a thread need their registers for the apply.
__host__ __device__ constexpr bool tail_caches_ritz(int P, int RPT, int NT) {
  return P > 0 && RPT * P <= (RPT > 2 ? 8 : 20) && NT < 1024;
}

// Rows of a thread: pairs of adjacent rows, 2 (tid + NT jj) + b for jj < RPT / 2, b in {0, 1}, so
// that one 16-byte load brings an entry of the FP64 band for both rows.
template <int NT>
__device__ inline int tail_row(int tid, int j) {
  return 2 * (tid + NT * (j >> 1)) + (j & 1);
}

__device__ inline double2 tail_ld16(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
}

__device__ inline float4 tail_ld16f(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
}

// S v for the thread's rows, v being in LDS (the padded lattice, or the whole vector for the
// dense S): a row of the band is hh stencil rows of ww consecutive entries, both in the band
// (columns of colA bytes) and in the padded direction; the dense S is one stencil row of m
// entries.  Each stencil row goes in chunks of CH entries whose loads, for all the thread's row
// pairs, are issued ahead of their multiply-adds (one load brings the entry of both rows of a
// pair; uniform column offsets in scalar registers, the pair a per-lane offset), then one chunk
// for the rest of the row, whose missing entries repeat the last one and are weighted by zero.
// ADJ: the second row of every pair starts its stencil one entry after the first (a lattice of
// even width), so both rows read one window of the direction and the compiler loads each LDS word
// once for the two.

template <int RPT, int NT, int CH, bool ADJ>
__device__ inline void tail_apply_rows(__amdgpu_buffer_rsrc_t rsA, uint32_t colA, const uint32_t* roff,
                                       const int* corner, const double* sp, int hh, int ww, int Wp, int64_t m,
                                       double* qv) {
  // with two row pairs a thread, pairs whose whole wavefront lies past m are skipped (a uniform
  // branch; with one pair every wavefront has rows)
  bool live[RPT / 2];
#pragma unroll
  for (int jj = 0; jj < RPT / 2; ++jj)
    live[jj] = RPT <= 2 || 2 * ((int64_t)(threadIdx.x & ~63) + (int64_t)NT * jj) < m;
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
        if (live[jj]) {
#pragma unroll
          for (int k = 0; k < CH; ++k) bv[jj][k] = tail_ld16(rsA, roff[jj], so + (uint32_t)k * colA);
        }
#pragma unroll
      for (int jj = 0; jj < RPT / 2; ++jj) {
        if (!live[jj]) continue;
        const double* p0 = sp + corner[2 * jj] + lrow + d0;
        if constexpr (ADJ) {
          // the pair's shared window (CH + 1 entries from an even index) in 16-byte LDS reads
          double w[CH + 1];
#pragma unroll
          for (int i = 0; i < CH / 2; ++i) {
            const double2 t2 = reinterpret_cast<const double2*>(p0)[i];
            w[2 * i] = t2.x;
            w[2 * i + 1] = t2.y;
          }
          w[CH] = p0[CH];
#pragma unroll
          for (int k = 0; k < CH; ++k) {
            qv[2 * jj] += bv[jj][k].x * w[k];
            qv[2 * jj + 1] += bv[jj][k].y * w[k + 1];
          }
        } else {
          const double* p1 = sp + corner[2 * jj + 1] + lrow + d0;
#pragma unroll
          for (int k = 0; k < CH; ++k) {
            qv[2 * jj] += bv[jj][k].x * p0[k];
            qv[2 * jj + 1] += bv[jj][k].y * p1[k];
          }
        }
      }
      so += (uint32_t)CH * colA;
    }
    if (d0 < ww) {
      const int last = ww - d0 - 1;
      double2 bv[RPT / 2][CH];
#pragma unroll
      for (int jj = 0; jj < RPT / 2; ++jj)
        if (live[jj]) {
#pragma unroll
          for (int k = 0; k < CH; ++k) bv[jj][k] = tail_ld16(rsA, roff[jj], so + (uint32_t)min(k, last) * colA);
        }
#pragma unroll
      for (int jj = 0; jj < RPT / 2; ++jj) {
        if (!live[jj]) continue;
        const double* p0 = sp + corner[2 * jj] + lrow + d0;
        const double* p1 = ADJ ? p0 + 1 : sp + corner[2 * jj + 1] + lrow + d0;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int kk = min(k, last);
          qv[2 * jj] += (k <= last ? bv[jj][k].x : 0.0) * p0[kk];
          qv[2 * jj + 1] += (k <= last ? bv[jj][k].y : 0.0) * p1[kk];
        }
      }
    }
  }
}

// The same with the FP32 band (or S) in its packed layout: four consecutive stencil entries of a
// row in 16 bytes, entry k of row r of stencil row li at float ((li ww4 / 4 + k / 4) ld + r) 4 +
// k % 4 (ww4: ww rounded up to 4, zeros past ww).  A load brings four entries of one row, so a
// row's stencil row takes ww4 / 4 loads: half the loads of the FP64 pairs, and the load unit
// takes about as long for a 16-byte load as for the 8 bytes of an FP32 pair (colQ: bytes of one
// column of quads; rowq: a row's byte offset in it).  The direction past a stencil row's last
// entry holds finite values (the next lattice row, or the zeroed slack after the padded lattice),
// which the zero weights cancel.  CH entries a chunk (a multiple of 4); the sums are in FP64.
template <int RPT, int NT, int CH, bool ADJ>
__device__ inline void tail_apply_rows_q(__amdgpu_buffer_rsrc_t rsQ, uint32_t colQ, const uint32_t* rowq,
                                         const int* corner, const double* sp, int hh, int ww4, int Wp, int64_t m,
                                         double* qv) {
  static_assert(CH % 4 == 0, "whole quads");
  constexpr int CQ = CH / 4;
  bool live[RPT / 2];
#pragma unroll
  for (int jj = 0; jj < RPT / 2; ++jj)
    live[jj] = RPT <= 2 || 2 * ((int64_t)(threadIdx.x & ~63) + (int64_t)NT * jj) < m;
#pragma unroll
  for (int j = 0; j < RPT; ++j) qv[j] = 0.0;
  for (int li = 0; li < hh; ++li) {
    uint32_t so = (uint32_t)(li * (ww4 / 4)) * colQ;
    const int lrow = li * Wp;
    int d0 = 0;
    for (; d0 + CH <= ww4; d0 += CH) {
      float4 bv[RPT][CQ];
#pragma unroll
      for (int j = 0; j < RPT; ++j)
        if (live[j / 2]) {
#pragma unroll
          for (int q = 0; q < CQ; ++q) bv[j][q] = tail_ld16f(rsQ, rowq[j], so + (uint32_t)q * colQ);
        }
      // every load of the chunk goes out before the first is used (widening each one as it lands
      // lets the compiler reuse its registers and wait for every load in turn)
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (ADJ) {
        // the pair's shared window (CH + 1 entries from an even index) in 16-byte LDS reads
#pragma unroll
        for (int jj = 0; jj < RPT / 2; ++jj) {
          if (!live[jj]) continue;
          const double* pw = sp + corner[2 * jj] + lrow + d0;
          double w[CH + 1];
#pragma unroll
          for (int i = 0; i < CH / 2; ++i) {
            const double2 t2 = reinterpret_cast<const double2*>(pw)[i];
            w[2 * i] = t2.x;
            w[2 * i + 1] = t2.y;
          }
          w[CH] = pw[CH];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int j = 2 * jj + h;
#pragma unroll
            for (int q = 0; q < CQ; ++q) {
              qv[j] += (double)bv[j][q].x * w[4 * q + h];
              qv[j] += (double)bv[j][q].y * w[4 * q + h + 1];
              qv[j] += (double)bv[j][q].z * w[4 * q + h + 2];
              qv[j] += (double)bv[j][q].w * w[4 * q + h + 3];
            }
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          if (!live[j / 2]) continue;
          const double* pj = sp + corner[j] + lrow + d0;
#pragma unroll
          for (int q = 0; q < CQ; ++q) {
            qv[j] += (double)bv[j][q].x * pj[4 * q];
            qv[j] += (double)bv[j][q].y * pj[4 * q + 1];
            qv[j] += (double)bv[j][q].z * pj[4 * q + 2];
            qv[j] += (double)bv[j][q].w * pj[4 * q + 3];
          }
        }
      }
      so += (uint32_t)CQ * colQ;
    }
    if (d0 < ww4) {
      // the rest in whole quads: missing quads repeat the last one and are weighted by zero
      const int lastq = (ww4 - d0) / 4 - 1;
      float4 bv[RPT][CQ];
#pragma unroll
      for (int j = 0; j < RPT; ++j)
        if (live[j / 2]) {
#pragma unroll
          for (int q = 0; q < CQ; ++q)
            bv[j][q] = tail_ld16f(rsQ, rowq[j], so + (uint32_t)min(q, lastq) * colQ);
        }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        if (!live[j / 2]) continue;
        const double* pj = (ADJ && (j & 1)) ? sp + corner[j - 1] + lrow + d0 + 1 : sp + corner[j] + lrow + d0;
#pragma unroll
        for (int q = 0; q < CQ; ++q) {
          const int qq = 4 * min(q, lastq);
          const double t = (double)bv[j][q].x * pj[qq] + (double)bv[j][q].y * pj[qq + 1] +
                           (double)bv[j][q].z * pj[qq + 2] + (double)bv[j][q].w * pj[qq + 3];
          qv[j] += q <= lastq ? t : 0.0;
        }
      }
    }
  }
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

// BT: element type of the band (or S) in the PCG iterations (double, or float for FP32 inner
// applies); the sweep's residual check always applies the FP64 band (or S).  MULTI: the queue
// holds (instance << kTailSysBits) | system entries over the descriptors in `table` (one launch
// for many instances); otherwise systems of the one instance `one`.
template <int P, int RPT, int NT, typename BT, bool MULTI>
__global__ __launch_bounds__(NT) void k_pcg_tail(TailInst one, const TailInst* __restrict__ table,
                                                 const int32_t* __restrict__ act, const int32_t* __restrict__ nact,
                                                 int32_t* __restrict__ qctr) {
  constexpr int W = 2 * P + 1;
  constexpr int NW = NT / 64;
  static_assert(RPT % 2 == 0, "rows come in pairs");
  // band (or S) entries per chunk: RPT / 2 * CH loads of FP64 pairs per thread, RPT * CHQ / 4
  // loads of the packed FP32 band.  Short chunks measured fastest at the n = 4096 lattice (the
  // FP64 kernel 0.56 ms per launch with 8 entries against 0.67 ms with 16; FP32 0.45 ms with 8
  // against 0.57 ms with 32)
  // With four rows a thread, 2 FP64 entries (4 entries of the packed FP32 band) a chunk still keep
  // four 16-byte loads in flight per thread, and the registers they save keep the kernel that serves
  // many instances from spilling.
  constexpr int CH = RPT >= 4 ? 2 : 8;
  constexpr int CHQ = RPT >= 4 ? 4 : 8;
  // the Ritz vectors of the thread's rows stay in registers when they fit
  constexpr bool kCache = tail_caches_ritz(P, RPT, NT);
  constexpr bool kLdsSums = tail_lds_sums(2 * P + 1, NT, RPT);
  constexpr bool kMerged = tail_merged(P, NT, RPT);
  constexpr int WM = 4 * P + 4;
  constexpr int kC = kCache ? RPT * P : 1;
  constexpr bool kLow = sizeof(BT) == 4;
  __shared__ double sred1[1][NW];
  __shared__ double sredW[W][NW];
  __shared__ double sG[3 * P * P + P + 1];
  __shared__ double scoef[2 * P + 2];
  __shared__ double sM[P * P + 1];
  __shared__ double sdot[kMerged ? WM : W];
  __shared__ int s_idx;
  // padded direction (band) or direction (dense S); then the partial sums and, when phi_lds, the
  // Ritz bases
  extern __shared__ __attribute__((aligned(16))) double sp[];
  const int tid = threadIdx.x;
  const int na = *nact;

  // The instance's values the loop uses, set when the queue reaches a system of another instance
  // (a single-instance launch sets them once).
  int cur = -1;
  int64_t m = 0;
  bool band = true;
  Grid g{};
  int Wp = 0, npad = 0, nh = 0, hh = 1, ww = 1, phi_lds = 0;
  bool adj = false;  // every row pair's stencils are one entry apart
  // the wrapped copies of a row's direction entry are written with it (no halo pass) where each
  // periodic axis is at least twice its stencil reach: then an entry has at most 3 copies
  bool hdirect = false;
  double dmin = 0.0;
  __amdgpu_buffer_rsrc_t rsA = tail_rsrc(nullptr, 0), rsI = rsA, rsF = rsA, rsG = rsA;
  uint32_t colA = 0, colI = 0, colF = 0;
  double *part = sp, *sF = sp, *sH = sp;
  // the corner of each row's stencil in the padded grid, and the byte offsets of each row pair in
  // a column of the FP64 band (pairs past m read the last pair and are discarded; an odd m leaves
  // its last pair one row into the column's padding, ld >= m + 1) and of each row in a column of
  // quads of the packed FP32 band (rows past m read row m - 1)
  int corner[RPT];
  int hcode[RPT];  // a row's wrapped copies: bit 0 along z, bit 1 its sign (-nz); bits 2, 3 along x
  uint32_t roff[RPT / 2], roffI[RPT];

  // the instance's layout, its preconditioner's small matrices, the zero halo of the padded
  // direction along axes that are not periodic (never rewritten), and its Ritz bases in LDS (the
  // previous system's last LDS reads are behind the loop's closing barrier)
  auto load_instance = [&](const TailInst& d) {
      const PCGState& st = d.st;
      const TailApply& ap = d.ap;
      const LMP& lmp = d.lmp;
      m = st.m;
      band = ap.kind == 0;
      g = ap.g;
      const int w = 2 * g.bx + 1, h = 2 * g.bz + 1;
      Wp = band ? g.nx + 2 * g.bx : 0;
      npad = band ? (g.nz + 2 * g.bz) * Wp : (int)m;
      nh = band ? (g.pz ? 2 * g.bz * Wp : 0) + (g.px ? g.nz * 2 * g.bx : 0) : 0;
      hh = band ? h : 1;
      ww = band ? w : (int)m;
      adj = band && g.nx % 2 == 0;
      hdirect = band && nh > 0 && (!g.px || g.nx >= 2 * g.bx) && (!g.pz || g.nz >= 2 * g.bz);
      phi_lds = d.phi_lds;
      if (P > 0) {
        for (int o = tid; o < 3 * P * P; o += NT) sG[o] = lmp.G[o];
        if (tid < P) sG[3 * P * P + tid] = lmp.theta[tid];
      }
      for (int o = tid; o < npad + kTailSlack; o += NT) sp[o] = 0.0;
      dmin = (P > 0) ? *lmp.dmin : 0.0;
      rsA = band ? tail_rsrc(ap.band, (int64_t)h * w * ap.ldb * 8) : tail_rsrc(ap.S, m * ap.lds * 8);
      colA = (uint32_t)((band ? ap.ldb : ap.lds) * 8);
      // the packed FP32 band (or S): (ww rounded up to 4) / 4 columns of 16-byte quads a stencil row
      rsI = !kLow ? rsA
                  : (band ? tail_rsrc(ap.band32, (int64_t)h * ((w + 3) / 4) * ap.ldb * 16)
                          : tail_rsrc(ap.S32, (m + 3) / 4 * ap.lds * 16));
      colI = kLow ? colA * 2 : colA;
      rsF = tail_rsrc(lmp.Phi, (int64_t)P * lmp.ld * 8);
      rsG = tail_rsrc(lmp.SPhi, (int64_t)P * lmp.ld * 8);
      colF = (uint32_t)(lmp.ld * 8);
      // rows of partial sums (tail_part_stride apart), then Phi (P x m), when phi_lds
      part = sp + npad + kTailSlack;
      sF = part + tail_sum_words(P, NT, RPT) * tail_part_stride(tail_part_rows(NT, RPT));
      sH = sF + (int64_t)P * m;             // S Phi (P x m)
      if (phi_lds) {  // 1: Phi only, 2: Phi and S Phi
        for (int o = tid; o < P * (int)m; o += NT) {
          const int l = o / (int)m, r = o % (int)m;
          sF[o] = tail_ld8(rsF, (uint32_t)r * 8, l * colF);
          if (phi_lds == 2) sH[o] = tail_ld8(rsG, (uint32_t)r * 8, l * colF);
        }
      }
#pragma unroll
      for (int jj = 0; jj < RPT; ++jj) {
        const int r = tail_row<NT>(tid, jj);
        corner[jj] = (band && r < m) ? (r / g.nx) * Wp + r % g.nx : 0;
        // the row's wrapped copies: at z + nz or z - nz along a periodic z within bz of an end,
        // at x + nx or x - nx likewise along x, and both together (every copy but the interior one)
        hcode[jj] = 0;
        if (hdirect && r < m) {
          const int z = r / g.nx, x = r % g.nx;
          if (g.pz && z < g.bz) hcode[jj] |= 1;
          else if (g.pz && z >= g.nz - g.bz) hcode[jj] |= 3;
          if (g.px && x < g.bx) hcode[jj] |= 4;
          else if (g.px && x >= g.nx - g.bx) hcode[jj] |= 12;
        }
        roffI[jj] = (uint32_t)min<int64_t>(r, m - 1) * 16u;
      }
#pragma unroll
      for (int jj = 0; jj < RPT / 2; ++jj) {
        const uint32_t row = (uint32_t)min<int64_t>(tail_row<NT>(tid, 2 * jj), (m - 1) & ~(int64_t)1);
        roff[jj] = row * (uint32_t)sizeof(double);
      }
      __syncthreads();
  };
  if (!MULTI) load_instance(one);

  // A system whose sweep's check leaves it above rtol is taken again at once, before the next
  // queue entry (its entry, iteration count, sweep count and inner target; the same in all threads)
  int32_t rs_e = -1;
  int rs_it = 0, rs_nsw = 0;
  double rs_thresh = 0.0;
  for (;;) {
    const bool resumed = rs_e >= 0;
    int32_t e = rs_e;
    rs_e = -1;
    if (!resumed) {
      if (tid == 0) s_idx = atomicAdd(qctr, 1);
      __syncthreads();
      const int idx = s_idx;
      __syncthreads();  // every thread has read s_idx before it is written again
      if (idx >= na) break;
      e = act[idx];
    }
    const int j = MULTI ? (int)(e >> kTailSysBits) : 0;
    const int32_t s = MULTI ? (e & ((1 << kTailSysBits) - 1)) : e;
    const TailInst& d = MULTI ? table[j] : one;
    const PCGState& st = d.st;
    const TailCheck& chk = d.chk;
    const bool check = d.r0 != nullptr && chk.b != nullptr;
    if (!resumed) {
      if (st.done[s] != 0) continue;
      // a system whose sweep budget is spent stays live for the host to finish
      if (check && chk.max_sweeps > 0 && chk.sweeps[s] >= chk.max_sweeps) continue;
    }
    if (MULTI && j != cur) {
      cur = j;
      load_instance(d);
    }
    // q = (1 + sigma) v + S v for the thread's rows: v to LDS (and its wrapped copies), then the
    // band (or S) streamed from L2 against it: the iterations' band, or the FP64 one (fp64)
    auto apply_C = [&](const double* v, double sig1, double* qv, bool fp64) {
#pragma unroll
      for (int jj = 0; jj < RPT; ++jj) {
        const int r = tail_row<NT>(tid, jj);
        if (r < m) {
          const int at = band ? corner[jj] + g.bz * Wp + g.bx : r;
          sp[at] = v[jj];
          const int hc = hcode[jj];
          if (hc != 0) {
            const int dz = (hc & 2) ? -g.nz * Wp : g.nz * Wp, dx = (hc & 8) ? -g.nx : g.nx;
            if (hc & 1) sp[at + dz] = v[jj];
            if (hc & 4) sp[at + dx] = v[jj];
            if ((hc & 5) == 5) sp[at + dz + dx] = v[jj];
          }
        }
      }
      __syncthreads();
      if (nh > 0 && !hdirect) {
        for (int t = tid; t < nh; t += NT) {
          int dst, src;
          if (tail_halo(g, Wp, t, dst, src)) sp[dst] = sp[src];
        }
        __syncthreads();
      }
      if (!kLow || fp64) {
        if (adj) tail_apply_rows<RPT, NT, CH, true>(rsA, colA, roff, corner, sp, hh, ww, Wp, m, qv);
        else tail_apply_rows<RPT, NT, CH, false>(rsA, colA, roff, corner, sp, hh, ww, Wp, m, qv);
      } else {
        const int ww4 = (ww + 3) & ~3;
        if (adj) tail_apply_rows_q<RPT, NT, CHQ, true>(rsI, colI, roffI, corner, sp, hh, ww4, Wp, m, qv);
        else tail_apply_rows_q<RPT, NT, CHQ, false>(rsI, colI, roffI, corner, sp, hh, ww4, Wp, m, qv);
      }
#pragma unroll
      for (int jj = 0; jj < RPT; ++jj) qv[jj] += sig1 * v[jj];
    };
    const int64_t base = (int64_t)s * st.ld;
    const double sig1 = 1.0 + st.sigma[s];
    const double bn = st.bnorm[s];
    const double thresh = resumed ? rs_thresh : st.thresh[s];
    // a start (r0 given) takes x = 0 and the residual r0 and begins with the first step's
    // preconditioned residual; a continuation reads x, r, p and r^T z of the batched loop
    // (a resumed sweep starts from the true residual its check left in st.r)
    const double* r0 = resumed ? st.r : d.r0;
    double* uacc = d.uacc;
    const bool start = d.r0 != nullptr;
    double rz = start ? 0.0 : st.rz[s];
    const int it0 = resumed ? rs_it : st.iters[s];
    int it = it0;
    double rv[RPT], pv[RPT], xv[RPT];
    double ph[kC], sph[kC];
#pragma unroll
    for (int jj = 0; jj < RPT; ++jj) {
      const int64_t r = tail_row<NT>(tid, jj);
      const bool ok = r < m;
      rv[jj] = ok ? (start ? r0[base + r] : st.r[base + r]) : 0.0;
      pv[jj] = (ok && !start) ? st.p[base + r] : 0.0;
      xv[jj] = (ok && !start) ? st.x[base + r] : 0.0;
      if (kCache) {
#pragma unroll
        for (int l = 0; l < P; ++l) {
          ph[(jj * P + l) % kC] = ok ? tail_ld8(rsF, (uint32_t)r * 8, l * colF) : 0.0;
          sph[(jj * P + l) % kC] = ok ? tail_ld8(rsG, (uint32_t)r * 8, l * colF) : 0.0;
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
    if constexpr (kMerged) {
    // 1 / (1 + sigma + theta_l) for this system
    double rth[P > 0 ? P : 1];
    // the squared residual norm against the squared target (no square root an iteration); the
    // relative residual is formed once the loop ends
    const double thresh2 = thresh * thresh;
    double rr_last = -1.0;
#pragma unroll
    for (int l = 0; l < P; ++l) rth[l] = 1.0 / (sig1 + sG[3 * P * P + l]);
    for (;;) {
      // the apply (the first pass of a start only prepares p: q = 0), then one reduction
      double qv[RPT];
      if (!first) apply_C(pv, sig1, qv, false);
      else {
#pragma unroll
        for (int jj = 0; jj < RPT; ++jj) qv[jj] = 0.0;
      }
      // sums: 0 p^T q, 1 q^T q, 2 r^T q, 3 r^T r, then Phi^T q, (S Phi)^T q, Phi^T r, (S Phi)^T r
      double acc[WM];
#pragma unroll
      for (int i = 0; i < WM; ++i) acc[i] = 0.0;
#pragma unroll
      for (int jj = 0; jj < RPT; ++jj) {
        const int64_t r = tail_row<NT>(tid, jj);
        if (r < m) {
          const double rj = rv[jj], qj = qv[jj];
          acc[0] += pv[jj] * qj;
          acc[1] += qj * qj;
          acc[2] += rj * qj;
          acc[3] += rj * rj;
#pragma unroll
          for (int l = 0; l < P; ++l) {
            const double a = kCache ? ph[(jj * P + l) % kC]
                                    : (phi_lds ? sF[l * m + r] : tail_ld8(rsF, (uint32_t)r * 8, l * colF));
            const double b = kCache ? sph[(jj * P + l) % kC]
                                    : (phi_lds == 2 ? sH[l * m + r] : tail_ld8(rsG, (uint32_t)r * 8, l * colF));
            acc[4 + l] += a * qj;
            acc[4 + P + l] += b * qj;
            acc[4 + 2 * P + l] += a * rj;
            acc[4 + 3 * P + l] += b * rj;
          }
        }
      }
      tail_sums_lds<WM, NT, RPT>(acc, part, sdot);
      const double* dt = sdot;
      // the step: r <- r - alpha q, and the new residual's dots from the old ones
      //   r'^T r' = r^T r - alpha (2 r^T q - alpha q^T q),  Phi^T r' = Phi^T r - alpha Phi^T q, ...
      double alpha = 0.0;
      if (!first) {
        const double tot = dt[0];
        if (!(tot > 0.0) || !isfinite(tot)) {
          if (tid == 0) atomicOr(st.flags, isfinite(tot) ? kFlagNotSPD : kFlagNumeric);
          state = 2;
          break;
        }
        alpha = rz / tot;
#pragma unroll
        for (int jj = 0; jj < RPT; ++jj) {
          if (tail_row<NT>(tid, jj) < m) {
            xv[jj] += alpha * pv[jj];
            rv[jj] -= alpha * qv[jj];
          }
        }
        ++it;
      }
      const double rr = fmax(dt[3] - alpha * (2.0 * dt[2] - alpha * dt[1]), 0.0);
      rr_last = rr;
      if (!isfinite(rr)) {
        if (tid == 0) atomicOr(st.flags, kFlagNumeric);
        state = 2;
        break;
      }
      if (rr <= thresh2) {
        state = 1;
        break;
      }
      if (it >= st.max_iter) {
        state = 2;
        break;
      }
      // the preconditioner's coefficients (as in the fused step), in every thread:
      //   c1 = Theta^{-1} Phi^T r,  c2 = Theta^{-1} [(C Phi)^T r - M(sigma) c1],
      //   gamma = (1 + sigma - beta_L) c1 + c2,  z = r - S Phi c1 - Phi gamma
      double c1[P > 0 ? P : 1], gm[P > 0 ? P : 1];
      double rzn = rr;
      if (P > 0) {
        const double beta_l = sig1 + dmin;
#pragma unroll
        for (int l = 0; l < P; ++l) c1[l] = (dt[4 + 2 * P + l] - alpha * dt[4 + l]) * rth[l];
        double tsum = 0.0;
#pragma unroll
        for (int l = 0; l < P; ++l) {
          double mc = 0.0;
#pragma unroll
          for (int j2 = 0; j2 < P; ++j2) mc += sM[l * P + j2] * c1[j2];
          const double phr = dt[4 + 2 * P + l] - alpha * dt[4 + l];
          const double sphr = dt[4 + 3 * P + l] - alpha * dt[4 + P + l];
          const double c2 = (sphr + sig1 * phr - mc) * rth[l];
          gm[l] = (sig1 - beta_l) * c1[l] + c2;
          tsum += sphr * c1[l] + phr * gm[l];
        }
        rzn -= tsum;
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
      for (int jj = 0; jj < RPT; ++jj) {
        const int64_t r = tail_row<NT>(tid, jj);
        if (r < m) {
          double z = rv[jj];
#pragma unroll
          for (int l = 0; l < P; ++l) {
            const double a = kCache ? ph[(jj * P + l) % kC]
                                    : (phi_lds ? sF[l * m + r] : tail_ld8(rsF, (uint32_t)r * 8, l * colF));
            const double b = kCache ? sph[(jj * P + l) % kC]
                                    : (phi_lds == 2 ? sH[l * m + r] : tail_ld8(rsG, (uint32_t)r * 8, l * colF));
            z -= b * c1[l] + a * gm[l];
          }
          pv[jj] = z + beta * pv[jj];
        }
      }
      // no barrier here: every thread has read the LDS direction and sdot before the next
      // direction's barrier, and part and sdot are rewritten only after it
    }
    if (rr_last >= 0.0 || !isfinite(rr_last)) relres = bn > 0.0 ? sqrt(rr_last) / bn : 0.0;
    } else {
    for (;;) {
      if (!first) {  // the apply and the step (the first pass of a start only prepares p)
        double qv[RPT];
        apply_C(pv, sig1, qv, false);
        double pq = 0.0;
#pragma unroll
        for (int jj = 0; jj < RPT; ++jj) pq += pv[jj] * qv[jj];
        const double tot = tail_sum1<NT>(pq, sred1);
        if (!(tot > 0.0) || !isfinite(tot)) {
          if (tid == 0) atomicOr(st.flags, isfinite(tot) ? kFlagNotSPD : kFlagNumeric);
          state = 2;
          break;
        }
        const double alpha = rz / tot;
#pragma unroll
        for (int jj = 0; jj < RPT; ++jj) {
          if (tail_row<NT>(tid, jj) < m) {
            xv[jj] += alpha * pv[jj];
            rv[jj] -= alpha * qv[jj];
          }
        }
        ++it;
      }  // !first
      // dots of r: r^T r, Phi^T r, (S Phi)^T r
      double acc[W];
#pragma unroll
      for (int jj = 0; jj < W; ++jj) acc[jj] = 0.0;
#pragma unroll
      for (int jj = 0; jj < RPT; ++jj) {
        const int64_t r = tail_row<NT>(tid, jj);
        if (r < m) {
          acc[0] += rv[jj] * rv[jj];
#pragma unroll
          for (int l = 0; l < P; ++l) {
            const double a = kCache ? ph[(jj * P + l) % kC]
                                    : (phi_lds ? sF[l * m + r] : tail_ld8(rsF, (uint32_t)r * 8, l * colF));
            const double b = kCache ? sph[(jj * P + l) % kC]
                                    : (phi_lds == 2 ? sH[l * m + r] : tail_ld8(rsG, (uint32_t)r * 8, l * colF));
            acc[1 + l] += a * rv[jj];
            acc[1 + P + l] += b * rv[jj];
          }
        }
      }
      if (kLdsSums) tail_sums_lds<W, NT, RPT>(acc, part, sdot);
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
      for (int jj = 0; jj < RPT; ++jj) {
        const int64_t r = tail_row<NT>(tid, jj);
        if (r < m) {
          double z = rv[jj];
#pragma unroll
          for (int l = 0; l < P; ++l) {
            const double a = kCache ? ph[(jj * P + l) % kC]
                                    : (phi_lds ? sF[l * m + r] : tail_ld8(rsF, (uint32_t)r * 8, l * colF));
            const double b = kCache ? sph[(jj * P + l) % kC]
                                    : (phi_lds == 2 ? sH[l * m + r] : tail_ld8(rsG, (uint32_t)r * 8, l * colF));
            z -= b * scoef[l] + a * scoef[P + l];
          }
          pv[jj] = z + beta * pv[jj];
        }
      }
      // no barrier here: every thread read the LDS direction before the first reduction's
      // barrier, and sred1, sredW, sdot and scoef are rewritten only after the next direction's
    }
    }  // kMerged
    // a start adds its correction to the solution; a continuation hands x, r, p back to the
    // batched loop, which adds x
    double un[RPT];
#pragma unroll
    for (int jj = 0; jj < RPT; ++jj) {
      const int64_t r = tail_row<NT>(tid, jj);
      un[jj] = 0.0;
      if (r < m) {
        if (start) {
          un[jj] = uacc[base + r] + xv[jj];
          uacc[base + r] = un[jj];
        } else {
          st.x[base + r] = xv[jj];
          st.r[base + r] = rv[jj];
          st.p[base + r] = pv[jj];
        }
      }
    }
    // the sweep's check of the new u: r = b - (1 + sigma) u - S u in FP64, kept for a further
    // sweep, and the status from ||r|| / ||b|| (every thread has left the loop's last LDS reads
    // behind the reductions' barriers)
    double rr = 0.0;
    if (check) {
      double qv[RPT];
      apply_C(un, sig1, qv, true);
      double r2 = 0.0;
#pragma unroll
      for (int jj = 0; jj < RPT; ++jj) {
        const int64_t r = tail_row<NT>(tid, jj);
        if (r < m) {
          const double rt = chk.b[base + r] - qv[jj];
          st.r[base + r] = rt;
          r2 += rt * rt;
        }
      }
      const double rn = sqrt(tail_sum1<NT>(r2, sred1));
      rr = bn > 0.0 ? rn / bn : 0.0;
    }
    const int nsw = check ? (resumed ? rs_nsw : chk.sweeps[s]) + 1 : 0;
    // the next sweep runs here only after a converged inner solve (breakdowns and the iteration
    // cap go to the status below)
    const bool again = check && state == 1 && isfinite(rr) && !(rr <= chk.rtol) && it < st.max_iter && !chk.fixed &&
                       chk.max_sweeps > 0 && nsw < chk.max_sweeps;
    if (tid == 0) {
      if (st.prof.vectors) {
        const int done_its = it - it0;
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
        chk.sweeps[s] = nsw;
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
          // the next sweep's inner target, as the status kernel sets it: rtol ||b|| / 2 for FP64
          // inner applies, else inner_rtol times the true residual (not below that)
          const double target = 0.5 * chk.rtol * bn;
          st.thresh[s] = chk.fixed ? 0.0 : (kLow ? fmax(chk.inner_rtol * rr * bn, target) : target);
        }
      }
    }
    if (again) {
      rs_e = e;
      rs_it = it;
      rs_nsw = nsw;
      const double target = 0.5 * chk.rtol * bn;
      rs_thresh = kLow ? fmax(chk.inner_rtol * rr * bn, target) : target;
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

// The queue of a launch over many instances, in two kernels.  k_batch_live: one workgroup per
// instance j orders its live systems (done == 0) as k_order_live does, its systems past the last
// whole group of grp (systems with their own shift, such as the mean update's) first, into its
// segment of `seg` (from table[j].seg) and their number into cnt[j].  k_batch_pack: one
// workgroup packs the segments, instance by instance, into `list` as (j << kTailSysBits) | s,
// with the total in *nact and the queue counter reset.
__global__ __launch_bounds__(1024) void k_batch_live(const TailInst* __restrict__ table, int32_t* __restrict__ seg,
                                                     int32_t* __restrict__ cnt) {
  __shared__ int32_t perm[kOrderQ];
  __shared__ int swave[16];
  __shared__ int total;
  const int j = blockIdx.x, t = threadIdx.x;
  const TailInst& d = table[j];
  const int32_t* done = d.st.done;
  const double* sigma = d.st.sigma;
  const int64_t S = d.st.S, G = d.grp;
  const int64_t Sg = S / G * G;    // systems in whole groups
  const int Q = (int)(Sg / G);
  const int64_t extra = S - Sg;    // they go first
  for (int q = t; q < Q; q += 1024) {
    const double kq = sigma[(int64_t)q * G];
    int rank = 0;
    for (int i = 0; i < Q; ++i) {
      const double ki = sigma[(int64_t)i * G];
      rank += (ki < kq || (ki == kq && i < q)) ? 1 : 0;
    }
    perm[rank] = q;
  }
  __syncthreads();
  // position u < extra: system Sg + u; else node perm[(u - extra) / G], member (u - extra) % G
  auto sys_at = [&](int64_t u) -> int64_t {
    return u < extra ? Sg + u : (int64_t)perm[(u - extra) / G] * G + (u - extra) % G;
  };
  const int64_t per = (S + 1023) / 1024;
  const int64_t a = t * per, b = min<int64_t>(S, a + per);
  int32_t c = 0;
  for (int64_t u = a; u < b; ++u) c += (done[sys_at(u)] == 0);
  int32_t pos = block_exclusive_scan<1024>(c, swave, &total);
  if (t == 0) cnt[j] = total;
  int32_t* out = seg + d.seg;
  for (int64_t u = a; u < b; ++u) {
    const int64_t sys = sys_at(u);
    if (done[sys] == 0) out[pos++] = (int32_t)sys;
  }
}

__global__ __launch_bounds__(1024) void k_batch_pack(const TailInst* __restrict__ table, int count,
                                                     const int32_t* __restrict__ seg, const int32_t* __restrict__ cnt,
                                                     int32_t* __restrict__ list, int32_t* __restrict__ nact,
                                                     int32_t* __restrict__ qctr) {
  __shared__ int swave[16];
  __shared__ int total;
  __shared__ int32_t start;
  const int t = threadIdx.x;
  if (t == 0) start = 0;
  __syncthreads();
  for (int j0 = 0; j0 < count; j0 += 1024) {
    const int j = j0 + t;
    const int32_t c = j < count ? cnt[j] : 0;
    const int32_t pos = start + block_exclusive_scan<1024>(c, swave, &total);
    __syncthreads();
    if (t == 0) start += total;
    if (j < count) {
      const int32_t* src = seg + table[j].seg;
      const int32_t tag = j << kTailSysBits;
      for (int32_t i = 0; i < c; ++i) list[pos + i] = tag | src[i];
    }
    __syncthreads();
  }
  if (t == 0) {
    *nact = start;
    *qctr = 0;
  }
}

// two rows a thread (one pair) up to 1024 rows, on 128, 256 or 512 threads; four rows on 512 or
// 1024 threads beyond
int tail_threads(int64_t m) { return m > 2048 ? 1024 : (m > 512 ? 512 : (m > 256 ? 256 : 128)); }

// the padded direction
size_t tail_lds_bytes(const TailApply& ap) {
  const int64_t npad = ap.kind == 0 ? (int64_t)(ap.g.nz + 2 * ap.g.bz) * (ap.g.nx + 2 * ap.g.bx) : ap.m;
  return (size_t)(npad + kTailSlack) * sizeof(double);
}

// LDS (static and dynamic) the launcher lets one workgroup take: the kernel runs one workgroup
// per CU at the sizes where it needs this much
constexpr size_t kTailLdsBig = 150 * 1024;

// The static LDS of an instantiation (read once).
hipError_t tail_static_lds(const void* fn, std::atomic<size_t>& cache, size_t* out) {
  size_t stat = cache.load();
  if (stat == ~(size_t)0) {
    hipFuncAttributes fa{};
    const hipError_t e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess) return e;
    stat = fa.sharedSizeBytes;
    cache.store(stat);
  }
  *out = stat;
  return hipSuccess;
}

// Dynamic LDS of one instance: the padded direction, the partial sums of the dots and, when the
// kernel does not keep the Ritz bases in registers, as much of them as there is room for (sets
// phi_lds: 2 both, 1 Phi only, S Phi then read from L2).  0 when the instance does not fit.
template <int P, int RPT, int NT>
size_t tail_inst_lds(TailInst& d, size_t stat) {
  size_t lds = tail_lds_bytes(d.ap);
  lds += (size_t)tail_sum_words(P, NT, RPT) * tail_part_stride(tail_part_rows(NT, RPT)) * sizeof(double);
  if (stat + lds > kTailLdsBig) return 0;
  const size_t one = (size_t)8 * P * d.st.m;  // one basis, FP64
  d.phi_lds = 0;
  if (P > 0 && !tail_caches_ritz(P, RPT, NT)) {
    if (stat + lds + 2 * one <= kTailLdsBig) d.phi_lds = 2;
    else if (stat + lds + one <= kTailLdsBig) d.phi_lds = 1;
  }
  lds += (size_t)d.phi_lds * one;
  return lds;
}

// Writes descriptors into the device table (kernel arguments carry them: capture safe).
constexpr int kPutPer = 6;
struct PutBatch {
  TailInst d[kPutPer];
};
__global__ void k_put_insts(PutBatch b, int cnt, TailInst* __restrict__ dst) {
  const int i = threadIdx.x;
  if (i < cnt) dst[i] = b.d[i];
}

// queue(): enqueues whatever builds the queue (after the table is written)
template <int P, int RPT, int NT, typename BT, bool MULTI, typename QF>
hipError_t tail_go(TailInst* descs, int count, TailInst* table, const int32_t* act, const int32_t* nact,
                   int32_t* qctr, int64_t grid, hipStream_t st, QF& queue) {
  const void* fn = (const void*)k_pcg_tail<P, RPT, NT, BT, MULTI>;
  static std::atomic<size_t> stat_cache{~(size_t)0};
  size_t stat = 0;
  hipError_t e = tail_static_lds(fn, stat_cache, &stat);
  if (e != hipSuccess) return e;
  size_t lds = 0;
  for (int j = 0; j < count; ++j) {
    if ((int64_t)RPT * NT < descs[j].st.m) return hipErrorInvalidValue;  // every row has a thread
    const size_t b = tail_inst_lds<P, RPT, NT>(descs[j], stat);
    if (b == 0) return hipErrorInvalidValue;
    lds = std::max(lds, b);
  }
  // dynamic LDS this instantiation may take (concurrent first calls raise it twice: harmless)
  static std::atomic<size_t> allowed{64 * 1024};
  if (lds > allowed.load()) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    allowed.store(lds);
  }
  if (MULTI) {
    for (int j0 = 0; j0 < count; j0 += kPutPer) {
      PutBatch b{};
      const int cnt = std::min(kPutPer, count - j0);
      for (int i = 0; i < cnt; ++i) b.d[i] = descs[j0 + i];
      hipLaunchKernelGGL(k_put_insts, dim3(1), dim3(64), 0, st, b, cnt, table + j0);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if ((e = queue()) != hipSuccess) return e;
  // no more workgroups than can be resident at once: the others would only find the queue empty
  int dev = 0, per_cu = 0, cus = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, lds);
  if (e != hipSuccess) return e;
  const int64_t resident = std::max<int64_t>((int64_t)per_cu * cus, 1);
  const dim3 gdim((unsigned)std::max<int64_t>(std::min(grid, resident), 1)), b(NT);
  hipLaunchKernelGGL((k_pcg_tail<P, RPT, NT, BT, MULTI>), gdim, b, lds, st, descs[0], MULTI ? table : nullptr, act,
                     nact, qctr);
  return hipGetLastError();
}

template <int P, typename BT, typename QF>
hipError_t tail_rows(TailInst* descs, int count, TailInst* table, const int32_t* act, const int32_t* nact,
                     int32_t* qctr, int64_t grid, hipStream_t st, QF& queue) {
  int64_t m = 0;
  for (int j = 0; j < count; ++j) m = std::max<int64_t>(m, descs[j].st.m);
  if (table) {  // many instances: one shape for all, from the largest m
    if (m <= 512) return tail_go<P, 2, 256, BT, true>(descs, count, table, act, nact, qctr, grid, st, queue);
    if (m <= 1024) return tail_go<P, 2, 512, BT, true>(descs, count, table, act, nact, qctr, grid, st, queue);
    if (m <= 2048) return tail_go<P, 4, 512, BT, true>(descs, count, table, act, nact, qctr, grid, st, queue);
    return tail_go<P, 4, 1024, BT, true>(descs, count, table, act, nact, qctr, grid, st, queue);
  }
  const int nt = tail_threads(m);
  const int64_t rpt = (m + nt - 1) / nt;
  if (nt == 128) return tail_go<P, 2, 128, BT, false>(descs, 1, nullptr, act, nact, qctr, grid, st, queue);
  if (nt == 256) return tail_go<P, 2, 256, BT, false>(descs, 1, nullptr, act, nact, qctr, grid, st, queue);
  if (nt == 1024) return tail_go<P, 4, 1024, BT, false>(descs, 1, nullptr, act, nact, qctr, grid, st, queue);
  if (rpt <= 2) return tail_go<P, 2, 512, BT, false>(descs, 1, nullptr, act, nact, qctr, grid, st, queue);
  if (rpt <= 4) return tail_go<P, 4, 512, BT, false>(descs, 1, nullptr, act, nact, qctr, grid, st, queue);
  return hipErrorInvalidValue;
}

template <int P, typename QF>
hipError_t tail_prec(TailInst* descs, int count, TailInst* table, const int32_t* act, const int32_t* nact,
                     int32_t* qctr, int64_t grid, hipStream_t st, QF& queue) {
  if (descs[0].ap.low) return tail_rows<P, float>(descs, count, table, act, nact, qctr, grid, st, queue);
  return tail_rows<P, double>(descs, count, table, act, nact, qctr, grid, st, queue);
}

// Checks one instance's descriptor.
bool tail_inst_ok(const TailInst& d) {
  const PCGState& s = d.st;
  const TailApply& ap = d.ap;
  const LMP& lmp = d.lmp;
  const TailCheck& chk = d.chk;
  if (s.m < 1 || s.m > kTailMaxM || s.m != ap.m || !tail_fits(ap) || ((d.r0 == nullptr) != (d.uacc == nullptr)) ||
      (chk.b && (!d.r0 || !chk.fdone || !chk.sweeps || !chk.relres)))
    return false;
  if (ap.kind == 0 && (!ap.band || (ap.low && !ap.band32))) return false;
  if (ap.kind == 1 && (!ap.S || (ap.low && !ap.S32))) return false;
  if (lmp.p > 0 && (!lmp.Phi || !lmp.SPhi || !lmp.G || !lmp.theta || !lmp.dmin)) return false;
  return true;
}

template <typename QF>
hipError_t tail_dispatch(TailInst* descs, int count, TailInst* table, const int32_t* act, const int32_t* nact,
                         int32_t* qctr, int64_t grid, hipStream_t st, QF&& queue) {
  if (count < 1 || !act || !nact || !qctr || (count > 1 && !table)) return hipErrorInvalidValue;
  for (int j = 0; j < count; ++j)
    if (!tail_inst_ok(descs[j]) || descs[j].lmp.p != descs[0].lmp.p || descs[j].ap.low != descs[0].ap.low)
      return hipErrorInvalidValue;
  switch (descs[0].lmp.p) {
    case 0: return tail_prec<0>(descs, count, table, act, nact, qctr, grid, st, queue);
    case 4: return tail_prec<4>(descs, count, table, act, nact, qctr, grid, st, queue);
    case 8: return tail_prec<8>(descs, count, table, act, nact, qctr, grid, st, queue);
    case 10: return tail_prec<10>(descs, count, table, act, nact, qctr, grid, st, queue);
    case 12: return tail_prec<12>(descs, count, table, act, nact, qctr, grid, st, queue);
    case 16: return tail_prec<16>(descs, count, table, act, nact, qctr, grid, st, queue);
    case 20: return tail_prec<20>(descs, count, table, act, nact, qctr, grid, st, queue);
    default: return hipErrorInvalidValue;
  }
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

namespace {

// One thread per (column of quads, row): four entries rounded to FP32 and stored as one 16-byte
// word.
__global__ void k_pack_quads(const double* __restrict__ src, int64_t hh, int64_t ww, int64_t ld, int64_t m,
                             float4* __restrict__ dst) {
  const int64_t wq = (ww + 3) / 4;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= hh * wq * ld) return;
  const int64_t r = i % ld, c = i / ld;
  const int64_t li = c / wq, k0 = (c % wq) * 4;
  float v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t k = k0 + e;
    v[e] = (k < ww && r < m) ? (float)src[(li * ww + k) * ld + r] : 0.0f;
  }
  dst[i] = float4{v[0], v[1], v[2], v[3]};
}

}  // namespace

hipError_t launch_pack_quads(const double* src, int64_t hh, int64_t ww, int64_t ld, int64_t m, float* dst,
                             hipStream_t st) {
  if (!src || !dst || hh < 1 || ww < 1 || ld < m || m < 1) return hipErrorInvalidValue;
  const int64_t n = hh * ((ww + 3) / 4) * ld;
  hipLaunchKernelGGL(k_pack_quads, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, hh, ww, ld, m,
                     reinterpret_cast<float4*>(dst));
  return hipGetLastError();
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
  TailInst d{};
  d.st = s;
  d.lmp = lmp;
  d.ap = ap;
  d.chk = chk;
  d.r0 = r0;
  d.uacc = uacc;
  return tail_dispatch(&d, 1, nullptr, act, nact, qctr, grid, st, []() { return hipSuccess; });
}

hipError_t launch_pcg_tail_multi(TailInst* descs, int count, TailInst* table, int32_t* seg, int32_t* cnt,
                                 int32_t* list, int32_t* nact, int32_t* qctr, int64_t grid, hipStream_t st) {
  if (count < 1 || count > (1 << (31 - kTailSysBits)) || !table || !seg || !cnt || !list || !nact || !qctr)
    return hipErrorInvalidValue;
  for (int j = 0; j < count; ++j) {
    const TailInst& d = descs[j];
    if (d.st.S < 1 || d.st.S >= (int64_t(1) << kTailSysBits) || d.grp < 1 || d.st.S / d.grp > kOrderQ || d.seg < 0)
      return hipErrorInvalidValue;
  }
  return tail_dispatch(descs, count, table, list, nact, qctr, grid, st, [&]() -> hipError_t {
    hipLaunchKernelGGL(k_batch_live, dim3((unsigned)count), dim3(1024), 0, st, table, seg, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_pack, dim3(1), dim3(1024), 0, st, table, count, seg, cnt, list, nact, qctr);
    return hipGetLastError();
  });
}

}  // namespace infoesrf
