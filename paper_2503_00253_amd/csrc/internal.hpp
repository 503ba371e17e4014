// Internal declarations of the InFo-ESRF HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <array>
#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/infoesrf.h"

namespace infoesrf {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
void clear_error();

#define IE_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      ::infoesrf::set_error(std::string("HIP error in ") + #call + ": " +            \
                            hipGetErrorString(e_));                                   \
      return INFOESRF_ERR_HIP;                                                        \
    }                                                                                 \
  } while (0)

#define IE_CHECK(cond, code, msg)                                                     \
  do {                                                                                \
    if (!(cond)) {                                                                    \
      ::infoesrf::set_error(msg);                                                     \
      return (code);                                                                  \
    }                                                                                 \
  } while (0)

#define IE_TRY(expr)                                                                  \
  do {                                                                                \
    int rc_ = (expr);                                                                 \
    if (rc_ < 0) return rc_;                                                          \
  } while (0)

constexpr int kMaxQ = 64;
constexpr int kMaxRitz = 32;   // p + oversample <= kMaxSketch
constexpr int64_t kDenseSMax = 16384;  // largest m of the dense form of S
constexpr int64_t kDenseSAuto = 4096;  // largest m the automatic choice assembles
constexpr int kMaxSketch = 48;  // sketch columns (small dense kernels keep k x k in LDS)
constexpr int kSysTile = 16;   // systems per MFMA column block

// Device-side flag bits set by kernels (read back into the status).
enum : int32_t { kFlagNotSPD = 1, kFlagNumeric = 2, kFlagBadInput = 4 };

// ---------------------------------------------------------------- stencil grid
// A stationary stencil on an nz x nx grid (state index z*nx + x).
struct Grid {
  int32_t nz, nx;
  int32_t pz, px;     // periodic flags
  int32_t bz, bx;     // half-extents
  const double* table;  // device (2bz+1)*(2bx+1) row-major FP64
  const float* table32; // device copy in FP32 (or null)
  const __hip_bfloat16* table16; // device copy in BF16 (or null)
};

// Precision of a covariance apply.
enum class Prec : int { F64 = 0, F32 = 1, BF16 = 2 };

// ---------------------------------------------------------------- wavefront sums
// A double moved across lanes by a DPP pattern (both 32-bit halves), lanes of rows outside
// ROWMASK reading zero.
template <int CTRL, int ROWMASK>
__device__ inline double dpp_f64(double x) {
  const long long v = __builtin_bit_cast(long long, x);
  const int lo = (int)(v & 0xffffffffll), hi = (int)(v >> 32);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xF, false);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xF, false);
  return __builtin_bit_cast(double, ((long long)h2 << 32) | (unsigned)l2);
}
// Sum over the 64 lanes of a wavefront in a fixed order (pairs, quads, half rows, rows of 16,
// then the four rows), held by lane 63: register-to-register moves instead of LDS shuffles.
__device__ inline double wave_sum_dpp(double x) {
  x += dpp_f64<0xB1, 0xF>(x);   // quad_perm [1,0,3,2]
  x += dpp_f64<0x4E, 0xF>(x);   // quad_perm [2,3,0,1]
  x += dpp_f64<0x141, 0xF>(x);  // row_half_mirror
  x += dpp_f64<0x140, 0xF>(x);  // row_mirror
  x += dpp_f64<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_f64<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

// Exclusive prefix sum of one int per thread over a workgroup of NT threads (wavefront scans by
// shuffles, then the NT / 64 wavefront totals in order); *total (LDS) receives the sum.  swave
// holds NT / 64 ints of LDS.
template <int NT>
__device__ inline int block_exclusive_scan(int v, int* swave, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) swave[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < NT / 64; ++w) {
      const int t = swave[w];
      swave[w] = run;
      run += t;
    }
    *total = run;
  }
  __syncthreads();
  return swave[wave] + x - v;
}

// ---------------------------------------------------------------- kernels (launchers)
// All launchers enqueue on `st` and return hipError_t of the launch.

// K1: mu = X 1 / N; Z = (X - mu 1^T)/sqrt(N-1), optional FP32 shadow of Z.
hipError_t launch_ens_stats(const double* X, int64_t n, int64_t N, double* mu, double* Z, float* Z32,
                            hipStream_t st);

// CSR -> CSC transpose of H (deterministic: entries of a column sorted by row) in two parts.
// launch_csc_count checks the CSR (row bounds, sorted columns in range, h_ptr[m] <= cap, the
// entries row_of / w_of can hold; else the bad-input flag) and counts each column's entries into
// col_cnt, which must be zero; launch_csc_finish forms col_ptr and, unless a flag is set, the
// sorted columns.
hipError_t launch_csc_count(const int32_t* h_ptr, const int32_t* h_idx, int64_t m, int64_t n, int64_t cap,
                            int32_t* col_cnt, int32_t* flags, hipStream_t st);
hipError_t launch_csc_finish(const int32_t* h_ptr, const int32_t* h_idx, const double* h_w, int64_t m, int64_t n,
                             int32_t* col_cnt, int32_t* col_ptr, int32_t* row_of, double* w_of, int32_t* flags,
                             hipStream_t st);

// rhs[s * ld + r] = dinv[r] * sum_e h_w[e] * Z[h_idx[e], member(s)] for systems s in [s0, s0+cnt),
// member(s) = (s - s0) % N.
hipError_t launch_obs_rhs(const int32_t* h_ptr, const int32_t* h_idx, const double* h_w, const double* r_var,
                          const double* Z, int64_t n, int64_t N, int64_t m, double* rhs, int64_t ld, int64_t s0,
                          int64_t cnt, hipStream_t st);
// The same for systems 0 .. cnt-1, writing the whole ld x spad block (zeros past m rows and past
// cnt systems).
hipError_t launch_obs_rhs_padded(const int32_t* h_ptr, const int32_t* h_idx, const double* h_w, const double* r_var,
                                 const double* Z, int64_t n, int64_t N, int64_t m, double* rhs, int64_t ld,
                                 int64_t cnt, int64_t spad, hipStream_t st);

// innovation rhs: out[s * ld + r] = dinv[r] * (y[r] - sum_e h_w[e] mu[h_idx[e]])
hipError_t launch_innovation(const int32_t* h_ptr, const int32_t* h_idx, const double* h_w, const double* r_var,
                             const double* y, const double* mu, int64_t m, int64_t n, double* out, int64_t ld,
                             int64_t s, hipStream_t st);

// diag(S)_r = dinv_r^2 * sum_{e,e'} w_e w_e' L(idx_e, idx_e') sum_i Z[idx_e,i] Z[idx_e',i]
hipError_t launch_diag_S(const int32_t* h_ptr, const int32_t* h_idx, const double* h_w, const double* r_var,
                         const double* Z, int64_t n, int64_t N, int64_t m, const Grid& g, const double* dense_L,
                         double* diagS, hipStream_t st);

// Observed-lattice members: Zt[k, i] = dinv[k] * h_w[k] * Z[idx[k], i] (m x N col-major)
// The sub-sampled stencil of the observed lattice: out[(dz + bzs) (2 bxs + 1) + dx + bxs] =
// table[(dz sz + bz) (2 bx + 1) + dx sx + bx] (formed by launch_lattice_members when out is set).
struct SubTable {
  const double* table = nullptr;
  int32_t bz = 0, bx = 0, sz = 1, sx = 1, bzs = 0, bxs = 0;
  double* out = nullptr;
};
hipError_t launch_lattice_members(const int32_t* h_idx, const double* h_w, const double* r_var, const double* Z,
                                  int64_t n, int64_t N, int64_t m, double* Zt, float* Zt32, hipStream_t st,
                                  const SubTable& sub = SubTable{});
// Sub-sampled stencil: sub[dz'][dx'] = table[dz' sz][dx' sx]
hipError_t launch_subsample_table(const double* table, int32_t bz, int32_t bx, int32_t sz, int32_t sx, int32_t bzs,
                                  int32_t bxs, double* sub, hipStream_t st);
// Lower-precision copies of a table / matrix.
hipError_t launch_convert_f32(const double* in, float* out, int64_t count, hipStream_t st);
hipError_t launch_convert_bf16(const double* in, __hip_bfloat16* out, int64_t count, hipStream_t st);

// ---------------------------------------------------------------- covariance apply (K3)
// Layout convention of the whole solver: every family of vectors (PCG state, apply inputs V
// and outputs T) is system-major: element (row r, system/column c) at c * ld + r.
// T[b * ldt + k] = sum_i Z[k,i] sum_l L[k,l] Z[l,i] V[b * ldv + l] for b < B.
// Z is column-major with leading dimension ldz; vcols = columns allocated in V.
struct CovTile {
  int rows_per_wave;  // multiple of 16
};
// Optional device-side measurement counters of a launch (see infoesrf_profile_enable).
struct ProfDev {
  unsigned long long* vectors;  // += live column count
  double* flops;                // += live column count * flops_per_vector
  double flops_per_vector;
  double* bytes;                // += live column count * bytes_per_vector
  double bytes_per_vector;
};
// B is the (padded) maximum column count; Bdev (nullable) holds the live count on the device.
// zero_counter (nullable): two int32 counters set to 0 by the launch (the next PCG step's list and
// live counts).
hipError_t launch_cov_stencil(Prec prec, const Grid& g, const void* Z, int64_t ldz, int64_t N, const void* V,
                              int64_t ldv, int64_t vcols, int64_t B, const int32_t* Bdev, void* T, int64_t ldt,
                              int rows_per_wave, hipStream_t st, const ProfDev* prof = nullptr,
                              int32_t* zero_counter = nullptr);
// BF16 apply (FP32 accumulation): Z (FP32, column-major, ldz), V system-major BF16
// (column b at V + b*ldk, vcols columns allocated), T FP32 system-fastest.  tile selects
// 16 x 32, 32 x 32, 16 x 64 or 16 x 128 (rows x systems) blocks.
hipError_t launch_cov_bf16(const Grid& g, const float* Z, int64_t ldz, int64_t N, const __hip_bfloat16* V,
                           int64_t ldk, int64_t vcols, int64_t B, const int32_t* Bdev, float* T, int64_t ldt, int tile,
                           hipStream_t st, const ProfDev* prof = nullptr, int32_t* zero_counter = nullptr);
hipError_t cov_bf16_timed(const Grid& g, const float* Z, int64_t ldz, int64_t N, const __hip_bfloat16* V,
                          int64_t ldk, int64_t vcols, int64_t B, const int32_t* Bdev, float* T, int64_t ldt, int tile,
                          hipStream_t st, int32_t* zero_counter = nullptr);
// Measured block shapes (tune.hip).  form: 0 band apply (choice = systems per block 8/16/32/64),
// 1 operator form FP64/FP32 (choice = tile 16/32/64/128), 2 operator form BF16 (tile).  prec:
// element type of the apply.  A choice of 0 means "not measured: use the built-in rule".
constexpr int kTuneBuckets = 3;  // batch sizes >= 256, 64..255, < 64
struct TuneKey {
  int form, prec, nz, nx, bz, bx, N;
};
extern thread_local int g_force_choice;  // nonzero while the tuner times a candidate
int tune_bucket(int64_t B);
int tuned_choice(const TuneKey& k, int64_t B);
void set_tuned(const TuneKey& k, int bucket, int choice);
void tune_reset();

// Explicit band of P = L o (Z Z^T) on grid g (band.hip): band[j * ldb + r] for the
// (2bz+1)(2bx+1) stencil offsets j, FP64 or FP32 entries computed in FP64 from Z (FP64,
// column-major, ldz).
hipError_t launch_band_build(Prec prec, const Grid& g, const double* Z, int64_t ldz, int64_t N, void* band,
                             int64_t ldb, hipStream_t st);
// T[:, b] = band V[:, b] for the listed columns b < B (Bdev: live count on the device), system-major
// V (ldv, vcols columns allocated) and T (ldt); FP64 or FP32.  zero_counter as for the operator form.
hipError_t launch_band_apply(Prec prec, const Grid& g, const void* band, int64_t ldb, const void* V, int64_t ldv,
                             int64_t vcols, int64_t B, const int32_t* Bdev, void* T, int64_t ldt, hipStream_t st,
                             const ProfDev* prof = nullptr, int32_t* zero_counter = nullptr);

// The final state-space apply on a declared observed lattice: P Ht R^{-1/2} u for point
// observations on the lattice needs, for each state point, only the lattice points inside its
// localization window, so the product is kept as a rectangular band of n rows x wz wx entries
// (entry (ia, ib) of state point (z, x): lattice point (ceil((z - bz - z0) / sz) + ia,
// ceil((x - bx - x0) / sx) + ib), wrapped along an axis the lattice tiles periodically, weight 0
// when outside the window or the lattice): R = L o (Z Zt^T) restricted to those entries, Zt the
// weighted lattice members R^{-1/2} H Z.  wz = 2 bz / sz + 1, wx = 2 bx / sx + 1.
struct RectGeom {
  int32_t nz, nx, pz, px, bz, bx;    // state grid, periodic flags, stencil half-extents
  int32_t z0, sz, nzo, x0, sx, nxo;  // the observed lattice
  int32_t wz, wx;                    // lattice points a window spans along z and x
  const double* table;               // (2 bz + 1) x (2 bx + 1) localization stencil, row-major
};
// Whether the rectangular form applies: along a periodic state axis the lattice must tile it, and
// the build's and the apply's LDS tiles (N members, N + 1 columns) fit in 64 KiB.
bool rect_fits(const Grid& gs, const infoesrf_lattice& lat, int64_t N);
RectGeom rect_geom(const Grid& gs, const infoesrf_lattice& lat);
// R (ldr rows, wz wx columns of entries) from Z (n x N, ldz) and Zt (m x N, ldzt).
hipError_t launch_rect_build(const RectGeom& g, const double* Z, int64_t ldz, const double* Zt, int64_t ldzt,
                             int64_t N, double* R, int64_t ldr, hipStream_t st);
// T[:, c] = R applied to column act[c] of U (m rows, ldu), for c < *nact (<= ncols); the n x ncols
// result column-major with leading dimension ldt.
hipError_t launch_rect_apply(const RectGeom& g, const double* R, int64_t ldr, const double* U, int64_t ldu,
                             const int32_t* act, const int32_t* nact, int64_t ncols, double* T, int64_t ldt,
                             hipStream_t st);
hipError_t cov_band_timed(Prec prec, const Grid& g, const void* band, int64_t ldb, const void* V, int64_t ldv,
                          int64_t vcols, int64_t B, const int32_t* Bdev, void* T, int64_t ldt, hipStream_t st,
                          int32_t* zero_counter = nullptr);
// Measurement wrapper used by the runtime: records events around the launch when profiling is on.
hipError_t cov_stencil_timed(Prec prec, const Grid& g, const void* Z, int64_t ldz, int64_t N, const void* V,
                             int64_t ldv, int64_t vcols, int64_t B, const int32_t* Bdev, void* T, int64_t ldt,
                             int rows_per_wave, hipStream_t st, int32_t* zero_counter = nullptr);
// Dense S (observation space, assembled once per call): unit columns, H^T R^{-1/2} e_k columns,
// gathered columns of S, symmetrization (+ FP32 copy), and the batched product T = S V.
hipError_t launch_unit_cols(int64_t rows, int64_t j0, int64_t bc, double* V, int64_t ldv, hipStream_t st);
hipError_t launch_scatter_unit_obs(const int32_t* h_ptr, const int32_t* h_idx, const double* h_w,
                                   const double* r_var, int64_t n, int64_t j0, int64_t bc, double* V, int64_t ldv,
                                   hipStream_t st);
hipError_t launch_gather_s_cols(int obs_domain, const double* T, int64_t ldt, const int32_t* h_ptr,
                                const int32_t* h_idx, const double* h_w, const double* r_var, int64_t n, int64_t m,
                                int64_t j0, int64_t bc, double* S, int64_t lds, hipStream_t st);
hipError_t launch_symmetrize(double* S, int64_t m, int64_t lds, float* S32, hipStream_t st);
// FP32 copy of hh stencil rows of ww columns (column-major, ld, m rows) in the persistent kernel's
// packed layout: entry k of row r of stencil row li at float ((li ww4 / 4 + k / 4) ld + r) 4 +
// k % 4, ww4 = ww rounded up to 4, zeros past ww and at rows >= m.  dst holds hh ww4 ld floats.
hipError_t launch_pack_quads(const double* src, int64_t hh, int64_t ww, int64_t ld, int64_t m, float* dst,
                             hipStream_t st);
hipError_t launch_dense_s_apply(Prec prec, const void* S, int64_t lds, int64_t m, const void* V, int64_t ldv,
                                const int32_t* nact, int64_t Bmax, void* T, int64_t ldt, int32_t* zero_counter,
                                hipStream_t st);
hipError_t launch_cov_dense(const double* L, const double* Z, int64_t n, int64_t N, const double* V, int64_t ldv,
                            int64_t B, double* T, int64_t ldt, hipStream_t st);

// ---------------------------------------------------------------- observation-space glue
// Active-system lists: act[c] = system of apply column c, *nact = live count (device).
// gather (observation domain): V[c * ldv + r] = P[act[c] * ldp + r] in the apply precision.
hipError_t launch_gather_active(Prec prec, const double* P, int64_t ldp, const int32_t* act, const int32_t* nact,
                                int64_t rows, int64_t Bmax, void* V, int64_t ldv, hipStream_t st);
// scatter (state domain): V[c * ldv + k] = sum_{e in CSC col k} w_e r^{-1/2}_{row_e} P[act[c] * ldp + row_e].
hipError_t launch_scatter_state(Prec prec, const double* P, int64_t ldp, const int32_t* act, const int32_t* nact,
                                const int32_t* col_ptr, const int32_t* row_of, const double* w_of,
                                const double* r_var, int64_t n, int64_t m, int64_t Bmax, void* V, int64_t ldv,
                                hipStream_t st);
// Q[s * ldp + r] = (1 + sigma_s) P[s * ldp + r] + (obs ? T[c * ldt + r] : r_r^{-1/2} sum_e w_e T[c * ldt + idx_e]),
// s = act[c] (sigma = -1 gives S itself).  T is FP64 for FP64 applies, FP32 otherwise.
hipError_t launch_apply_finish(Prec prec, int obs_domain, const double* P, int64_t ldp, const void* T, int64_t ldt,
                               const int32_t* act, const int32_t* nact, const double* sigma, const int32_t* h_ptr,
                               const int32_t* h_idx, const double* h_w, const double* r_var, int64_t m,
                               int64_t n_state, int64_t Bmax, double* Qv, hipStream_t st);

// ---------------------------------------------------------------- PCG (K4)
struct LMP {
  int p;               // number of Ritz pairs (0 = no preconditioner)
  const double* Phi;   // m x p column-major (Phi[j*ld + r]): a wavefront reads 64 consecutive rows
  const double* SPhi;  // m x p column-major, same ld
  int64_t ld;          // leading dimension of Phi and SPhi
  const double* theta; // p Ritz values of S
  const double* G;     // 3 p x p Gram matrices: Phi^T Phi, Phi^T S Phi, (S Phi)^T S Phi (row-major)
  const double* dmin;  // min diag(S) (1 value)
};

struct PCGState {
  int64_t m, S, ld;      // rows, systems, leading dimension (system s at s * ld)
  double *x, *r, *p;     // iterate, residual, search direction
  const double* sigma;   // per-system shift
  double* rz;            // per system r^T z
  double* thresh;        // per system absolute residual target
  double* bnorm;         // per system ||b|| (for relres)
  double* relres;        // per system recursive relative residual
  int32_t* iters;        // per system iteration counts
  int32_t* done;         // per system: 0 active, 1 converged, 2 failed/capped
  int32_t* flags;        // global error flags
  int max_iter;
  ProfDev prof;          // measurement counters (vectors = live systems of each launch), or empty
};

// One PCG iteration for every system of the list (one workgroup per system), after the apply.
// mode 0 starts a solve (dots of r, p = z); mode 1 takes the step from T = S p.  Systems still
// active are appended to act_out (*nact_out must be zero on entry) and their new p is written to
// V (apply precision, observation domain; nullable).  plain != 0 keeps retired systems in the
// list (masked solver).  m <= 4096.
// Multi-shift CG state (systems s = q N + i, system-major columns of ld; per-member scalars).
struct MscState {
  int64_t m, ld, N;
  int Q, q0;                     // nodes and the base (smallest) node
  double *x, *r, *p;             // every system's iterate and direction; r of the base systems
  const double* sigma;           // per system node s_q
  const double* bnorm;           // per system ||b||
  const double* thresh;          // per system absolute residual target
  double *zeta, *zeta_prev;      // per system residual ratios to the base residual
  double *rr, *alpha_prev, *beta_prev;  // per member base CG scalars
  int32_t* mit;                  // per member iterations taken
  double* relres;                // per system recursive relative residual
  int32_t* iters;                // per system iterations
  int32_t* done;                 // per system: 0 live, 1 converged, 2 capped or failed
  int32_t* flags;
  int max_iter;
};
hipError_t launch_msc_list(int32_t* act, int32_t* nact, int64_t q0, int64_t N, hipStream_t st);
// One multi-shift iteration for every member in the list (mode 0 starts), after the apply of S to
// the base directions (T, slot-major).  Live members are appended to act_out (*nact_out zeroed
// beforehand) with their next base direction in V (observation domain, nullable).  m <= 4096.
hipError_t launch_msc_step(const MscState& s, int mode, int obs_domain, const double* T, int64_t ldt,
                           const int32_t* act, const int32_t* nact, int32_t* act_out, int32_t* nact_out, int64_t Bmax,
                           double* V, int64_t ldv, const int32_t* h_ptr, const int32_t* h_idx, const double* h_w,
                           const double* r_var, int64_t n_state, hipStream_t st);
// Block PCG state: node q's block is the N system-major columns q N .. q N + N - 1 (ld).
struct BcgState {
  int64_t m, ld, N;
  int Q, p;                      // nodes, Ritz pairs of the preconditioner
  double *X, *R, *P, *W;         // iterate, residual, search block, W = C P
  const double *Phi, *SPhi;      // m x p Ritz vectors, ld = ldphi
  int64_t ldphi;
  const double* G;               // the preconditioner's Gram blocks (3 p x p, row-major)
  const double* theta;           // Ritz values of S
  const double* dmin;            // min diag(S)
  const double* sigma;           // per system node s_q
  const double* thresh;          // per system absolute residual target
  const double* bnorm;           // per system ||b||
  double* part;                  // per node and 128-row chunk: partial products
  int nch;                       // chunks
  double* red;                   // per node: reduced products
  double* coef;                  // per node: A, B, c1, gamma
  int32_t* bdone;                // per node: 0 iterating, 1 converged, 2 capped
  int32_t* iters;
  double* relres;
  int32_t* done;
  int32_t* flags;
  int max_iter;
};
// Sizes (doubles) of the block solver's buffers for m rows, N members, p Ritz pairs, Q nodes.
int64_t bcg_partial_doubles(int64_t m, int64_t N, int p, int Q);
int64_t bcg_reduced_doubles(int64_t N, int p, int Q);
int64_t bcg_coef_doubles(int64_t N, int p, int Q);
int bcg_chunks(int64_t m);
// One block-PCG iteration for every live node (mode 0: the start, P = M R; mode 1: iteration
// `it` after W = C P): partial products, their reduction, the per-node small solves and the
// row-wise update.  N <= 64, p <= 20.
hipError_t launch_bcg_iteration(const BcgState& s, int mode, int it, hipStream_t st);
// act = systems of the live nodes (node-major), *nact their number.
hipError_t launch_bcg_list(const int32_t* bdone, int Q, int64_t N, int32_t* act, int32_t* nact, hipStream_t st);
// In-place apply of S for the persistent finish: kind 0 = explicit band of P on the observed
// lattice g (rows = m), kind 1 = dense S (m x m, column-major, lds).
// low != 0: the PCG iterations apply FP32 copies (band32 or S32, packed by launch_pack_quads with
// the same leading dimension), widened to FP64 as they are read; the residual check applies the
// FP64 band or S.
struct TailApply {
  int kind;
  Grid g;
  const double* band;
  int64_t ldb;
  const double* S;
  int64_t lds;
  int64_t m;
  int low;
  const float* band32;
  const float* S32;
};
// Finish the listed systems (act, *nact) with one persistent launch of `grid` workgroups that take
// systems from the queue counter qctr (zeroed beforehand) and iterate each to convergence, the
// cap or a breakdown (FP64 PCG with the limited-memory preconditioner).  m <= 4096.
hipError_t launch_pcg_fused(Prec prec, const PCGState& s, const LMP& lmp, int mode, int obs_domain, int plain,
                            const void* T, int64_t ldt, const int32_t* act, const int32_t* nact, int32_t* act_out,
                            int32_t* nact_out, int64_t Bmax, void* V, int64_t ldv, const int32_t* h_ptr,
                            const int32_t* h_idx, const double* h_w, const double* r_var, int64_t n_state,
                            hipStream_t st);
// The residual sweep's status, taken in the persistent kernel after a started solve: the true
// residual r = b - (1 + sigma) u - S u of the new u (kept in the PCG state's r), its relative
// norm, and the sweep's per-system status (converged to rtol / out of iterations / continue with
// an inner threshold of rtol ||b|| / 2, 0 for a fixed count), as the status kernel sets it.
struct TailCheck {
  const double* b;   // right-hand sides (system-major, the state's ld); null: no check
  int32_t* fdone;    // final status: 1 converged, 2 failed, 3 fixed count reached
  int32_t* sweeps;   // sweeps per system (+1)
  double* relres;    // true relative residual of the sweep (the PCG state's relres is the inner one)
  double rtol;
  int fixed;
  double inner_rtol; // FP32 inner applies: the next sweep's inner target relative to the residual
  int max_sweeps;    // sweeps a system may take in all; > 0: the kernel runs them back to back,
                     // 0: one sweep a launch (the host decides on the next)
};
// r0 and uacc (both given or both null): each system starts from x = 0 with residual r0 (the
// kernel takes the first step itself) and adds its solution into uacc, then, when chk->b is
// given, takes the sweep's status; otherwise it continues the batched loop's x, r, p, r^T z and
// writes them back.
hipError_t launch_pcg_tail(const PCGState& s, const LMP& lmp, const TailApply& ap, const int32_t* act,
                           const int32_t* nact, int32_t* qctr, int64_t grid, const double* r0, double* uacc,
                           const TailCheck& chk, hipStream_t st);
// One instance of a persistent launch: its PCG state, preconditioner, in-place apply and sweep
// check, where its solves start (r0) and add their solutions (uacc), the group size of its
// shifts (systems q grp .. q grp + grp - 1 share one; systems past the last whole group have
// their own and are taken first) and its segment in the queue builder's scratch.
struct TailInst {
  PCGState st;
  LMP lmp;
  TailApply ap;
  TailCheck chk;
  const double* r0;
  double* uacc;
  int64_t seg;
  int32_t grp;
  int32_t phi_lds;  // set by the launcher: Ritz bases staged in LDS (2 both, 1 Phi only, 0 none)
};
// A queue entry of a launch over many instances: (instance << kTailSysBits) | system.
constexpr int kTailSysBits = 20;
// One persistent launch for the live systems of every instance of descs (host copies, count of
// them): writes the descriptors into `table` (device, count entries), orders each instance's live
// systems into its segment of `seg` (sum of the instances' S entries) with its count in cnt
// (count entries), packs them into `list` (same size as seg) with the total in *nact, and runs
// them.  All instances share the Ritz-basis count and the iterations' precision; m <= 4096.
hipError_t launch_pcg_tail_multi(TailInst* descs, int count, TailInst* table, int32_t* seg, int32_t* cnt,
                                 int32_t* list, int32_t* nact, int32_t* qctr, int64_t grid, hipStream_t st);
// launch_pcg_tail with the measurement hook (profile slot INFOESRF_PROF_TAIL).
hipError_t pcg_tail_timed(const PCGState& s, const LMP& lmp, const TailApply& ap, const int32_t* act,
                          const int32_t* nact, int32_t* qctr, int64_t grid, const double* r0, double* uacc,
                          const TailCheck& chk, hipStream_t st);
// Whether launch_pcg_tail takes this apply: m <= 4096, the padded lattice (or m values) within
// its LDS budget, at most one wrapped copy per side along periodic axes.
bool tail_fits(const TailApply& ap);
// (act, *nact) = the live systems (done == 0) of S = Q G systems s = q G + i that share one shift
// per group of G, node by node in order of increasing shift (ties by node), members in order;
// Q <= 4096.  A non-null qctr (the persistent kernel's queue counter) is set to zero.
hipError_t launch_order_live(const int32_t* done, const double* sigma, int64_t S, int64_t G, int32_t* act,
                             int32_t* nact, int32_t* qctr, hipStream_t st);
// The fused PCG step with the measurement hook (profile slot INFOESRF_PROF_PCG); arguments as
// launch_pcg_fused.
hipError_t pcg_fused_timed(Prec prec, const PCGState& s, const LMP& lmp, int mode, int obs_domain, int plain,
                           const void* T, int64_t ldt, const int32_t* act, const int32_t* nact, int32_t* act_out,
                           int32_t* nact_out, int64_t Bmax, void* V, int64_t ldv, const int32_t* h_ptr,
                           const int32_t* h_idx, const double* h_w, const double* r_var, int64_t n_state,
                           hipStream_t st);

// Rebuild the list of active systems (done == 0), in increasing order.  One block.
hipError_t launch_compact(const int32_t* done, int64_t S, int32_t* act, int32_t* nact, hipStream_t st);
hipError_t launch_iota(int32_t* act, int32_t* nact, int64_t S, hipStream_t st);

// ---------------------------------------------------------------- misc vector kernels
hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t st);
hipError_t launch_sub(const double* a, const double* b, double* out, int64_t count, hipStream_t st);  // out = a - b
hipError_t launch_axpy(double* x, const double* d, int64_t count, hipStream_t st);                  // x += d
// out[s] = ||v[s*ld : s*ld + m]||_2, one workgroup per system (deterministic)
hipError_t launch_col_norms(const double* v, int64_t m, int64_t S, int64_t ld, double* out, hipStream_t st);
hipError_t launch_residual_status(const double* rn, const double* bn, double tol, double* relres, int32_t* done,
                                  int64_t S, int32_t* flags, hipStream_t st);
// Quadrature combine: ubar[i * ldb + r] = sum_q p_q u[(s0 + q N + i) * ldu + r]
// (with act and nact non-null it also lists the N combined columns: act = 0 .. N-1, *nact = N)
hipError_t launch_quad_combine(const double* u, int64_t ldu, int64_t m, int64_t N, int32_t Q, const double* pw,
                               double* ubar, int64_t ldb, int64_t s0, int32_t* act, int32_t* nact, hipStream_t st);
// Final state update: out[k + i*n] = scale * (Z[k + i*n] - T[i*ldt + k])  (column-major out)
hipError_t launch_final_pert(const double* Z, const double* T, int64_t ldt, int64_t n, int64_t N, double scale,
                             double* out, hipStream_t st);
hipError_t launch_final_mean(const double* mu, const double* T, int64_t ldt, int64_t n, int64_t col, double* out,
                             hipStream_t st);
// dst[c*ldd + r] = src[c*lds + r] for r < rows, zero for rows <= r < ldd
hipError_t launch_copy_cols(const double* src, int64_t lds, int64_t rows, int64_t cols, double* dst, int64_t ldd,
                            hipStream_t st);

// ---------------------------------------------------------------- preconditioner setup (K8)
// A strided m x k operand: element (r, a) at ptr[r * rs + a * cs].
struct Strided {
  const double* ptr;
  int64_t rs, cs;
};
// Gaussian sketch by counter-based Philox4x32-10 + Box-Muller: out[j*ld + r] (system-major)
hipError_t launch_sketch(uint64_t seed, int64_t m, int k, double* out, int64_t ld, hipStream_t st);
// The same sketch over all ld rows (zeros past m), and the k columns as systems: act = 0 .. k-1,
// *nact = k, sig[0 .. nsig) = -1 (nsig >= k).
hipError_t launch_sketch_setup(uint64_t seed, int64_t m, int k, double* out, int64_t ld, int32_t* act, int32_t* nact,
                               double* sig, int nsig, hipStream_t st);
// Gram: G[a*k+b] = sum_r A(r, a) B(r, b), a,b < k (fixed order, deterministic)
hipError_t launch_gram(Strided A, Strided B, int64_t m, int k, double* G, double* scratch, hipStream_t st);
int gram_chunks(int64_t m);  // row chunks of launch_gram: scratch holds gram_chunks(m) * k * k doubles
// One-workgroup small dense kernels.
hipError_t launch_chol_inv(double* G, int k, int32_t* flags, hipStream_t st);   // G <- R^{-1} (upper), G = R^T R
// out(r, j) = sum_a A(r, a) M[a*kout + j], out(r, j) at out[r*ors + j*ocs]
hipError_t launch_right_mult(Strided A, int64_t m, int k, const double* M, int kout, double* out, int64_t ors,
                             int64_t ocs, hipStream_t st);
hipError_t launch_sym_eig(double* T, int k, double* evec, double* evals, hipStream_t st);  // Jacobi
hipError_t launch_lmp_finish(const double* evals, const double* evec, int k, int p, double* theta, double* sel,
                             hipStream_t st);                                  // top-p selection matrix
hipError_t launch_min_reduce(const double* v, int64_t count, double* out, hipStream_t st);
// The setup's small dense steps for k <= 8 sketch columns and m <= 8192 rows in two launches:
// Q = orth(Y) by Cholesky-QR twice, then theta, Phi, S Phi and the three Gram blocks from Qb and
// S Qb (all column-major with leading dimension ld <= 2^26).
bool small_basis_fits(int k, int p, int64_t m);
// (Q2, if not null, receives a second copy of Q)
hipError_t launch_cholqr2_small(const double* Y, int64_t m, int k, int64_t ld, double* Q, double* Q2, int32_t* flags,
                                hipStream_t st);
hipError_t launch_ritz_small(const double* Qb, const double* SQ, int64_t m, int k, int p, int64_t ld, double* theta,
                             double* Phi, double* SPhi, double* G, hipStream_t st);

}  // namespace infoesrf
